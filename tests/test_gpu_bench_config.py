"""The large-ring benchmark's own configuration against the oracle.

bench.py times one step of: a batch of 16 ciphertexts (N = 2^16, L = 24,
K = 6, dnum 4, scale 2^50, keys from pft_keygen seed 1 with rotation keys
2^0..2^14, seeded encryptions), the shipped NTT schedule table imported,
then eight links c <- RESCALE(HMult+relin(c, c)) and rotate-and-sum over all
2^15 slots (Alg. 2).  These tests build exactly that state through bench.py's
own helpers and run its own job_step, and compare ciphertexts 0 and 15 with
the oracle bit for bit: after the first link and after the whole step.

The only departure from bench.py is the encoder of the slot values: the
oracle's encoder produces the integer plaintexts that both sides encrypt (the
library's own encoder, used by bench.py, is checked to agree within one unit
per coefficient), so no value on the oracle side comes from the library."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import sampler as SP

pytestmark = pytest.mark.gpu

BATCH = 16
CHECKED = (0, BATCH - 1)


class BenchWorld:
    def __init__(self):
        import bench
        self.bench = bench
        self.lp, self.ctx = bench.make_context()
        op = self.op = C.Params.from_config(S.CONFIGS["C3"])
        assert self.lp.q == op.q and self.lp.p == op.p
        C.set_mul_mode(1)
        n = self.n = op.n
        slots = bench.batch_slots(n, BATCH)
        self.plains = [C.encode(z, n, op.scale) for z in slots]
        lib_plain = self.lp.encode(slots[0])
        assert np.max(np.abs(lib_plain - self.plains[0])) <= 1
        self.cts = bench.encrypt_batch(self.ctx, self.lp, self.plains)
        bench.import_tuning(self.ctx, bench.DEFAULT_TUNING)
        # the oracle's keys from its own Philox draws of the same seed
        s = self.s = SP.secret(bench.KEY_SEED, n)
        self.pk = C.public_key(op, s, *SP.public_key_draws(bench.KEY_SEED, op.q, n))
        mods = op.key_moduli()
        self.rlk = C.relin_key(op, s, *SP.switch_key_draws(bench.KEY_SEED, 0, mods, op.dnum, n))
        self.rot = {st: C.rotation_key(op, s, st, *SP.switch_key_draws(bench.KEY_SEED, SP.rotation_key_id(st, n),
                                                                          mods, op.dnum, n))
                    for st in bench.ROT_STEPS}
        self.ocs = {i: C.encrypt(op, self.pk, self.plains[i], op.L, *SP.encryption_draws(bench.ENC_SEED0 + i, n),
                                 op.scale) for i in CHECKED}

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert g.level == o.level and g.scale == o.scale
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)

    def oracle_link(self, o):
        return C.rescale(self.op, C.hmul_relin(self.op, o, o, self.rlk))


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    return BenchWorld()


def test_bench_inputs_match_oracle(world):
    for i in CHECKED:
        world.assert_same(world.cts[i], world.ocs[i])


@pytest.mark.timeout(900)
def test_bench_first_link_matches_oracle(world):
    """HMult+relin then RESCALE of the whole batch at level 24, the calls and
    schedules of the timed step."""
    out = world.bench.chain_link(world.ctx, world.cts)
    for i in CHECKED:
        world.assert_same(out[i], world.oracle_link(world.ocs[i]))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("i", CHECKED)
def test_bench_job_step_matches_oracle(world, i):
    """The whole timed step (eight links, then the 15-rotation TotalSum whose
    additions finish in the ModDown epilogue) for one checked ciphertext."""
    if not hasattr(world, "step_out"):
        world.step_out = world.bench.job_step(world.ctx, world.cts)
    o = world.ocs[i]
    for _ in range(world.bench.CHAIN_DEPTH):
        o = world.oracle_link(o)
    o = C.total_sum(world.op, o, world.bench.ROT_SLOTS, world.rot)
    world.assert_same(world.step_out[i], o)
