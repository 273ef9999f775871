"""Rotation keys beyond the HBM budget: the limited rotation-key cache
(pinned host copies, least-recently-used device slots).

Every rotation through the cache is bit-exact with the oracle, across
evictions: single rotations in an order that forces misses, the
power-of-two decomposition (more keys than slots in one call) and TotalSum
with a single slot.  Capture and late configuration are refused."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C

pytestmark = pytest.mark.gpu

SMALL = dict(log_n=12, n_q=3, q0_bits=60, q_bits=40, n_p=1, p_bits=60, dnum=3, scale=2 ** 40)
STEPS = [1, 2, 4, 8, 16]


class World:
    def __init__(self, slots):
        import paper_1908_06972_amd.ckks as L
        self.op = C.Params(**SMALL)
        self.lp = L.Params(*SMALL.values())
        C.set_mul_mode(1)
        self.n = self.op.n
        self.ctx = L.Context(self.lp)
        self.ctx.set_key_cache(slots)
        kd = S.key_draws(19, self.n, self.op.q)
        self.ctx.set_secret(kd.s)
        self.ctx.gen_public_key(kd.pk_a, kd.pk_e)
        self.pk = C.public_key(self.op, kd.s, kd.pk_a, kd.pk_e)
        self.keys = {}
        for st in STEPS:
            a, e = S.switch_key_draws(19, 900 + st, self.n, self.op.key_moduli(), self.op.dnum)
            self.ctx.gen_rotation_key(st, a, e)
            self.keys[st] = C.rotation_key(self.op, kd.s, st, a, e)

    def enc_pair(self, seed, level=3):
        m = S.plaintext_coeffs(S.rng(seed), self.n, 2 ** 40)
        d = S.enc_draws(seed + 1, self.n)
        return (self.ctx.encrypt(m, level, self.op.scale, d.v, d.e0, d.e1),
                C.encrypt(self.op, self.pk, m, level, d.v, d.e0, d.e1, self.op.scale))

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)


@pytest.fixture(scope="module")
def two_slots():
    import torch
    assert torch.cuda.is_available()
    return World(2)


def test_rotations_across_evictions(two_slots):
    w = two_slots
    g, o = w.enc_pair(40)
    before = w.ctx.key_cache_stats()
    assert before["max_resident"] == 2 and before["slots"] == 2
    for st in [1, 2, 4, 1, 8, 16, 2, 1, 4]:
        g = w.ctx.rotate(g, st)
        o = C.rotate(w.op, o, st, w.keys[st])
        w.assert_same(g, o)
    after = w.ctx.key_cache_stats()
    assert after["misses"] > before["misses"] and after["bytes_in"] > before["bytes_in"]
    assert after["slots"] == 2


def test_pow2_rotation_with_more_keys_than_slots(two_slots):
    w = two_slots
    g, o = w.enc_pair(50)
    w.assert_same(w.ctx.rotate_pow2(g, 31), C.rotate_pow2(w.op, o, 31, w.keys))
    gs = [w.enc_pair(60 + 2 * i) for i in range(3)]
    outs = w.ctx.rotate_pow2_batch([x[0] for x in gs], 21)
    for (gx, ox), out in zip(gs, outs):
        w.assert_same(out, C.rotate_pow2(w.op, ox, 21, w.keys))


def test_total_sum_single_slot():
    import torch
    assert torch.cuda.is_available()
    w = World(1)
    g, o = w.enc_pair(70)
    w.assert_same(w.ctx.total_sum(g, 32), C.total_sum(w.op, o, 32, w.keys))
    st = w.ctx.key_cache_stats()
    assert st["slots"] == 1 and st["misses"] >= 4


def test_key_cache_refusals(two_slots):
    w = two_slots
    g, _ = w.enc_pair(80)
    out = w.ctx.empty_ct(g.level)
    with pytest.raises(RuntimeError):  # no capture with a limited cache
        w.ctx.capture(lambda: w.ctx.rotate(g, 1, out=out))
    with pytest.raises(RuntimeError):  # must be set before the first rotation key
        w.ctx.set_key_cache(4)
    # the context still works after the refused capture
    w.ctx.rotate(g, 2, out=out)
    w.ctx.synchronize()


def test_plan_eviction_and_copy_ahead():
    """With the rotation order given as a plan, the cache evicts the key used
    farthest ahead and copies the next key in while the current rotation
    runs: a cyclic order over more keys than slots then hits, and every
    result stays bit-exact."""
    import torch
    assert torch.cuda.is_available()
    w = World(2)
    w.ctx.key_cache_plan(STEPS)
    g, o = w.enc_pair(90)
    before = w.ctx.key_cache_stats()
    for _ in range(3):
        for st in STEPS:
            g = w.ctx.rotate(g, st)
            o = C.rotate(w.op, o, st, w.keys[st])
    w.assert_same(g, o)
    after = w.ctx.key_cache_stats()
    assert after["prefetches"] > before["prefetches"]
    assert after["hits"] - before["hits"] >= 10  # each key after the first is copied in ahead of its use
    assert after["slots"] == 2
    # a rotation outside the plan still works and leaves results exact
    w.ctx.key_cache_plan([])
    g = w.ctx.rotate(g, 4)
    o = C.rotate(w.op, o, 4, w.keys[4])
    w.assert_same(g, o)


def test_exec_batch_rotations_through_a_limited_cache():
    """Rotations of ciphertexts at two levels in one op list run as
    concurrent groups on the executor's side streams; with two key slots
    for five keys, slots are refilled while other streams may still read
    them (ordered by events).  Every output equals the oracle."""
    import torch
    assert torch.cuda.is_available()
    w = World(2)
    ins = [w.enc_pair(200 + 2 * i, level=3 if i % 2 == 0 else 2) for i in range(10)]
    cts = [g for g, _ in ins]
    ops = []
    for i in range(10):
        out = len(cts)
        cts.append(w.ctx.empty_ct(ins[i][0].level))
        ops.append(("rotate", i, 0, out, STEPS[i % len(STEPS)], 0))
    w.ctx.exec_batch(cts, ops)
    w.ctx.synchronize()
    for i, (_, o) in enumerate(ins):
        st = STEPS[i % len(STEPS)]
        w.assert_same(cts[10 + i], C.rotate(w.op, o, st, w.keys[st]))
    assert w.ctx.key_cache_stats()["slots"] == 2
