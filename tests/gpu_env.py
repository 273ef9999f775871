"""Shared set-up of the GPU parity tests: one oracle world and one libpft
world built from the same seeded draws (synth), never from each other."""

import numpy as np

import synth as S
from oracle import ckks as C


class World:
    """Keys and helpers for one parameter set on both sides."""

    def __init__(self, cfg, seed=1, rot_steps=(), relin=True):
        import paper_1908_06972_amd.ckks as L

        self.cfg = cfg
        self.op = C.Params.from_config(cfg)
        self.lp = L.Params.from_config(cfg)
        assert self.lp.q == self.op.q and self.lp.p == self.op.p
        self.n = self.op.n
        C.set_mul_mode(1 if self.n > 4096 else 0)
        self.ctx = L.Context(self.lp)
        kd = S.key_draws(seed, self.n, self.op.q)
        self.kd = kd
        self.ctx.set_secret(kd.s)
        self.ctx.gen_public_key(kd.pk_a, kd.pk_e)
        self.pk = C.public_key(self.op, kd.s, kd.pk_a, kd.pk_e)
        self.rlk = None
        if relin:
            a, e = S.switch_key_draws(seed, 0, self.n, self.op.key_moduli(), self.op.dnum)
            self.ctx.gen_relin_key(a, e)
            self.rlk = C.relin_key(self.op, kd.s, a, e)
        self.rot = {}
        for st in rot_steps:
            self.add_rotation(st, seed)
        self.seed = seed

    def add_rotation(self, step, seed=None):
        seed = self.seed if seed is None and hasattr(self, "seed") else (seed or 1)
        a, e = S.switch_key_draws(seed, 1000 + (step % (self.n // 2)), self.n, self.op.key_moduli(), self.op.dnum)
        self.ctx.gen_rotation_key(step, a, e)
        self.rot[step] = C.rotation_key(self.op, self.kd.s, step, a, e)

    def encrypt_pair(self, m, level, enc_seed, scale=None):
        """Encrypt the integer plaintext m on both sides with the same draws."""
        scale = self.op.scale if scale is None else scale
        d = S.enc_draws(enc_seed, self.n)
        g = self.ctx.encrypt(m, level, scale, d.v, d.e0, d.e1)
        o = C.encrypt(self.op, self.pk, m, level, d.v, d.e0, d.e1, scale)
        return g, o

    def random_plain(self, seed, bound=None):
        bound = int(self.op.scale) if bound is None else bound
        return S.plaintext_coeffs(S.rng(seed), self.n, bound)

    def assert_same(self, g, o):
        """Bit-exact residue parity in coefficient form (both polynomials)."""
        host = self.ctx.export(g)
        assert g.level == o.level
        assert host.shape == (2, o.level, self.n)
        assert np.array_equal(host[0], o.c0), _first_diff(host[0], o.c0)
        assert np.array_equal(host[1], o.c1), _first_diff(host[1], o.c1)
        assert g.scale == o.scale


def _first_diff(a, b):
    idx = np.argwhere(a != b)
    if len(idx) == 0:
        return "equal"
    i = tuple(idx[0])
    return "first mismatch at %s: %d vs %d (%d mismatches)" % (i, int(a[i]), int(b[i]), len(idx))
