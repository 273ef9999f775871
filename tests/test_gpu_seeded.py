"""Seeded KEYGEN and ENC on the GPU (pft_keygen, pft_encrypt_seeded) against
the oracle fed with its own Philox4x64-10 draws (oracle/sampler.py).

The keys are compared through what they produce, bit-exactly: a seeded
encryption (public key and the encryption draws), its decryption (the
secret), HMult+relin (the relinearisation key) and a rotation per step (the
rotation keys), including keys generated under a one-slot key cache."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import sampler as SP

pytestmark = pytest.mark.gpu

SMALL = dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40)
STEPS = [1, 3, 64, -1]


class World:
    def __init__(self, spec, seed, steps, cache=0):
        import paper_1908_06972_amd.ckks as L
        self.op = C.Params(**spec)
        self.lp = L.Params(*spec.values())
        C.set_mul_mode(1)
        n = self.n = self.op.n
        self.ctx = L.Context(self.lp)
        if cache:
            self.ctx.set_key_cache(cache)
        self.ctx.keygen(seed, steps)
        self.s = SP.secret(seed, n)
        self.pk = C.public_key(self.op, self.s, *SP.public_key_draws(seed, self.op.q, n))
        mods = self.op.key_moduli()
        self.rlk = C.relin_key(self.op, self.s, *SP.switch_key_draws(seed, 0, mods, self.op.dnum, n))
        self.rot = {st: C.rotation_key(self.op, self.s, st,
                                       *SP.switch_key_draws(seed, SP.rotation_key_id(st, n), mods, self.op.dnum, n))
                    for st in steps}

    def enc_pair(self, mseed, eseed, level):
        m = S.plaintext_coeffs(S.rng(mseed), self.n, 2 ** 30)
        g = self.ctx.encrypt_seeded(m, level, self.op.scale, eseed)
        o = C.encrypt(self.op, self.pk, m, level, *SP.encryption_draws(eseed, self.n), self.op.scale)
        return g, o

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    return World(SMALL, 2024, STEPS)


def test_seeded_encrypt_and_decrypt(world):
    w = world
    g, o = w.enc_pair(1, 77, w.op.L)
    w.assert_same(g, o)
    assert np.array_equal(w.ctx.decrypt(g), C.decrypt(w.op, w.s, o))
    g2, _ = w.enc_pair(1, 77, w.op.L)
    w.assert_same(g2, o)  # same seed, same ciphertext
    g3, o3 = w.enc_pair(1, 78, 2)
    w.assert_same(g3, o3)
    assert not np.array_equal(w.ctx.export(g3)[1], w.ctx.export(g)[1][:2])


def test_seeded_relin_key(world):
    w = world
    (ga, oa), (gb, ob) = w.enc_pair(2, 90, w.op.L), w.enc_pair(3, 91, w.op.L)
    w.assert_same(w.ctx.mul_relin(ga, gb), C.hmul_relin(w.op, oa, ob, w.rlk))


@pytest.mark.parametrize("step", STEPS)
def test_seeded_rotation_keys(world, step):
    w = world
    g, o = w.enc_pair(4, 100 + abs(step), 3)
    w.assert_same(w.ctx.rotate(g, step), C.rotate(w.op, o, step, w.rot[step]))


def test_seeded_keys_under_one_slot_cache():
    import torch
    assert torch.cuda.is_available()
    w = World(SMALL, 7, [2, 5], cache=1)
    g, o = w.enc_pair(5, 200, w.op.L)
    for st in [2, 5, 2]:
        g = w.ctx.rotate(g, st)
        o = C.rotate(w.op, o, st, w.rot[st])
        w.assert_same(g, o)
    assert w.ctx.key_cache_stats()["slots"] == 1


def test_seeded_keygen_single_op_config():
    """The single-op workload's parameters (N = 2^12, two 40-bit primes and a
    50-bit special prime): encrypt -> HMult+relin -> rescale -> decrypt."""
    import torch
    assert torch.cuda.is_available()
    cfg = S.CONFIGS["C1"]
    spec = dict(log_n=cfg.log_n, n_q=cfg.n_q, q0_bits=cfg.q0_bits, q_bits=cfg.q_bits, n_p=cfg.n_p,
                p_bits=cfg.p_bits, dnum=cfg.dnum, scale=2 ** cfg.log_scale)
    w = World(spec, 1, [])
    (ga, oa), (gb, ob) = w.enc_pair(101, 1001, w.op.L), w.enc_pair(102, 1002, w.op.L)
    g = w.ctx.rescale(w.ctx.mul_relin(ga, gb))
    o = C.rescale(w.op, C.hmul_relin(w.op, oa, ob, w.rlk))
    w.assert_same(g, o)
    assert np.array_equal(w.ctx.decrypt(g), C.decrypt(w.op, w.s, o))


def test_keygen_refuses_step_zero():
    import torch
    import paper_1908_06972_amd.ckks as L
    assert torch.cuda.is_available()
    op = C.Params(**SMALL)
    ctx = L.Context(L.Params(*SMALL.values()))
    with pytest.raises(RuntimeError):
        ctx.keygen(3, [op.n // 2])
    # nothing was generated: encryption still has no public key
    with pytest.raises(RuntimeError):
        ctx.encrypt_seeded(S.plaintext_coeffs(S.rng(1), op.n, 2 ** 20), op.L, op.scale, 1)


def test_keygen_twice_replaces_every_key():
    """A second pft_keygen on the same context (another seed) regenerates the
    secret, public, relinearisation and rotation keys in place: results then
    match the oracle's keys for the second seed."""
    import torch
    assert torch.cuda.is_available()
    w = World(SMALL, 5, [3])
    w2 = World.__new__(World)
    w2.__dict__.update(w.__dict__)
    w.ctx.keygen(6, [3])
    n, op = w.n, w.op
    w2.s = SP.secret(6, n)
    w2.pk = C.public_key(op, w2.s, *SP.public_key_draws(6, op.q, n))
    mods = op.key_moduli()
    w2.rlk = C.relin_key(op, w2.s, *SP.switch_key_draws(6, 0, mods, op.dnum, n))
    w2.rot = {3: C.rotation_key(op, w2.s, 3, *SP.switch_key_draws(6, SP.rotation_key_id(3, n), mods, op.dnum, n))}
    (ga, oa), (gb, ob) = w2.enc_pair(7, 307, op.L), w2.enc_pair(8, 308, op.L)
    w2.assert_same(w2.ctx.mul_relin(ga, gb), C.hmul_relin(op, oa, ob, w2.rlk))
    w2.assert_same(w2.ctx.rotate(ga, 3), C.rotate(op, oa, 3, w2.rot[3]))
    assert np.array_equal(w2.ctx.decrypt(ga), C.decrypt(op, w2.s, oa))


def test_seeded_large_ring():
    """The large-ring parameters (N = 2^16, 24 + 6 primes, dnum 4) as the
    benchmark sets them up: seeded keys and encryption, then HMult+relin,
    RESCALE and a rotation, bit-exact against the oracle's own draws."""
    import torch
    assert torch.cuda.is_available()
    cfg = S.CONFIGS["C3"]
    spec = dict(log_n=cfg.log_n, n_q=cfg.n_q, q0_bits=cfg.q0_bits, q_bits=cfg.q_bits, n_p=cfg.n_p,
                p_bits=cfg.p_bits, dnum=cfg.dnum, scale=2 ** cfg.log_scale)
    w = World(spec, 1, [1])
    (ga, oa), (gb, ob) = w.enc_pair(303, 3000, w.op.L), w.enc_pair(304, 3001, w.op.L)
    w.assert_same(ga, oa)
    g = w.ctx.rescale(w.ctx.mul_relin(ga, gb))
    o = C.rescale(w.op, C.hmul_relin(w.op, oa, ob, w.rlk))
    w.assert_same(g, o)
    w.assert_same(w.ctx.rotate(g, 1), C.rotate(w.op, o, 1, w.rot[1]))


def test_new_secret_drops_every_derived_key():
    """A key of an earlier secret never stays usable: after keygen with
    steps [1, 3] and then keygen with [3] alone, step 1 has no key; after
    pft_set_secret the public, relinearisation and rotation keys are all
    missing until generated again."""
    import torch
    from paper_1908_06972_amd.native import PFT_ENOKEY, PftError
    assert torch.cuda.is_available()
    w = World(SMALL, 11, [1, 3])
    g, _ = w.enc_pair(9, 409, w.op.L)
    w.ctx.rotate(g, 1)
    w.ctx.keygen(12, [3])
    with pytest.raises(PftError) as ei:
        w.ctx.rotate(g, 1)
    assert ei.value.code == PFT_ENOKEY
    w.ctx.rotate(g, 3)
    w.ctx.set_secret(SP.secret(13, w.n))
    for call in (lambda: w.ctx.rotate(g, 3), lambda: w.ctx.mul_relin(g, g),
                 lambda: w.ctx.encrypt_seeded(S.plaintext_coeffs(S.rng(1), w.n, 2 ** 20), w.op.L, w.op.scale, 5)):
        with pytest.raises(PftError) as ei:
            call()
        assert ei.value.code == PFT_ENOKEY
