"""ModUp and ModDown conversions fused with the first pass of the forward
transform of their rows (k_bconv_col_b): key switching bit-exact against the
oracle with the forward schedule pinned to one that starts with a radix-16
column pass, so both fused kernels run; full and ragged digits, one and
several items, fp64 and integer rows; and the fused and unfused paths give
the same ciphertexts."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import sampler as SP

pytestmark = pytest.mark.gpu

CASES = {
    # alpha 2 (one k-block), 40-bit rows
    "a2_n12": dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40),
    # alpha 6 (three k-blocks) as in the large ring: 50-bit fp64 rows, 60-bit integer rows
    "a6_n12": dict(log_n=12, n_q=12, q0_bits=60, q_bits=50, n_p=6, p_bits=60, dnum=2, scale=2 ** 50),
    # alpha 2 at N = 2^14 (column stride 1024)
    "a2_n14": dict(log_n=14, n_q=8, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=4, scale=2 ** 40),
    # alpha 3 at N = 2^13 (schedule (4, 9), a 512-point row pass), odd K
    "a3_n13": dict(log_n=13, n_q=6, q0_bits=60, q_bits=45, n_p=3, p_bits=60, dnum=2, scale=2 ** 45),
    # alpha 4 at N = 2^15 as in the bag-of-words ring (schedule (4, 11), a
    # 2048-point row pass, two sub-problems per workgroup)
    "a4_n15": dict(log_n=15, n_q=8, q0_bits=60, q_bits=40, n_p=4, p_bits=60, dnum=2, scale=2 ** 40),
}
STEPS = [1, 5]


class World:
    def __init__(self, spec):
        import paper_1908_06972_amd.ckks as L
        self.op = C.Params(**spec)
        self.lp = L.Params(*spec.values())
        C.set_mul_mode(1)
        n = self.n = self.op.n
        self.ctx = L.Context(self.lp)
        seed = 31
        self.ctx.keygen(seed, STEPS)
        self.s = SP.secret(seed, n)
        self.pk = C.public_key(self.op, self.s, *SP.public_key_draws(seed, self.op.q, n))
        mods = self.op.key_moduli()
        self.rlk = C.relin_key(self.op, self.s, *SP.switch_key_draws(seed, 0, mods, self.op.dnum, n))
        self.rot = {st: C.rotation_key(self.op, self.s, st,
                                       *SP.switch_key_draws(seed, SP.rotation_key_id(st, n), mods, self.op.dnum, n))
                    for st in STEPS}
        cands = self.ctx.ntt_candidates()
        self.col16 = [c for c in cands if c[0][0] == 4]
        assert self.col16

    def enc_pair(self, mseed, level):
        m = S.plaintext_coeffs(S.rng(mseed), self.n, 2 ** 30)
        g = self.ctx.encrypt_seeded(m, level, self.op.scale, 500 + mseed)
        o = C.encrypt(self.op, self.pk, m, level, *SP.encryption_draws(500 + mseed, self.n), self.op.scale)
        return g, o

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)


_worlds = {}


def world(name):
    import torch
    assert torch.cuda.is_available()
    if name not in _worlds:
        _worlds[name] = World(CASES[name])
    return _worlds[name]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("flags", [0, 3])
def test_fused_modup_relin_and_rotation(name, flags):
    w = world(name)
    sched = [c for c in w.col16 if c[1] == flags][0]
    w.ctx.ntt_set_schedule(False, sched)
    w.ctx.bconv_mode(True, fused=True)
    L = w.op.L
    try:
        for level in sorted({L, L - 1, 1}):
            (ga, oa), (gb, ob) = w.enc_pair(10 + level, level), w.enc_pair(40 + level, level)
            w.assert_same(w.ctx.mul_relin(ga, gb), C.hmul_relin(w.op, oa, ob, w.rlk))
            for st in STEPS:
                w.assert_same(w.ctx.rotate(ga, st), C.rotate(w.op, oa, st, w.rot[st]))
    finally:
        w.ctx.ntt_set_schedule(False, None)


@pytest.mark.parametrize("name", ["a6_n12", "a2_n14", "a4_n15"])
def test_fused_modup_batch_equals_unfused(name):
    """Three items in one launch: the key inner product fused with the row
    pass of ModUp's rows, the fused passes alone and the unfused path
    produce the same ciphertexts, and all match the oracle."""
    w = world(name)
    sched = [c for c in w.col16 if c[1] == 0][0]
    w.ctx.ntt_set_schedule(False, sched)
    level = w.op.L - 1  # a ragged last digit
    pairs = [(w.enc_pair(70 + i, level), w.enc_pair(80 + i, level)) for i in range(3)]
    try:
        outs = {}
        for mode in ((True, True, True), (True, True, False), (True, False, False), (False, False, False)):
            w.ctx.bconv_mode(True, fused=mode[0], inner=mode[1], pairs=mode[2])
            outs[mode] = [w.ctx.export(g) for g in
                          w.ctx.mul_relin_batch([p[0][0] for p in pairs], [p[1][0] for p in pairs])]
        for mode in ((True, True, False), (True, False, False), (False, False, False)):
            for a, b in zip(outs[(True, True, True)], outs[mode]):
                assert np.array_equal(a, b)
        for ((_, oa), (_, ob)), host in zip(pairs, outs[(True, True, True)]):
            o = C.hmul_relin(w.op, oa, ob, w.rlk)
            assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)
    finally:
        w.ctx.bconv_mode(True, fused=True)
        w.ctx.ntt_set_schedule(False, None)


@pytest.mark.parametrize("name", ["a2_n12", "a6_n12"])
@pytest.mark.parametrize("first16", [True, False])
def test_rescale_fused_and_unfused(name, first16):
    """RESCALE with its expansion fused with the first transform pass
    (forward schedule starting with radix 16) and unfused (another first
    radix): single and batched, top and lowest levels, against the oracle."""
    w = world(name)
    sched = [c for c in w.ctx.ntt_candidates() if (c[0][0] == 4) == first16][0]
    w.ctx.ntt_set_schedule(False, sched)
    try:
        for level in sorted({w.op.L, 2}):
            g, o = w.enc_pair(90 + level, level)
            w.assert_same(w.ctx.rescale(g), C.rescale(w.op, o))
            gs = [w.enc_pair(120 + 3 * level + i, level) for i in range(3)]
            for (_, ox), out in zip(gs, w.ctx.rescale_batch([x[0] for x in gs])):
                w.assert_same(out, C.rescale(w.op, ox))
    finally:
        w.ctx.ntt_set_schedule(False, None)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("inv", ["col16_flags0", "col16_flags3", "other"])
def test_inverse_fused_conversions(name, inv):
    """The inverse transforms before ModUp and ModDown stop before their final
    radix-16 column pass and the conversion kernels apply it to their inputs
    (inverse schedule pinned to one ending with that pass, two flag sets), or
    run whole (another schedule): relinearisation and rotation against the
    oracle at full, ragged and lowest levels."""
    w = world(name)
    fwd = [c for c in w.col16 if c[1] == 0][0]
    if inv == "other":
        isched = [c for c in w.ctx.ntt_candidates() if c[0][0] != 4][0]
    else:
        isched = [c for c in w.col16 if c[1] == (0 if inv == "col16_flags0" else 3)][0]
    w.ctx.ntt_set_schedule(False, fwd)
    w.ctx.ntt_set_schedule(True, isched)
    L = w.op.L
    try:
        for level in sorted({L, L - 1, 1}):
            (ga, oa), (gb, ob) = w.enc_pair(150 + level, level), w.enc_pair(170 + level, level)
            w.assert_same(w.ctx.mul_relin(ga, gb), C.hmul_relin(w.op, oa, ob, w.rlk))
            for st in STEPS:
                w.assert_same(w.ctx.rotate(ga, st), C.rotate(w.op, oa, st, w.rot[st]))
            assert np.array_equal(w.ctx.decrypt(ga), C.decrypt(w.op, w.s, oa))
    finally:
        w.ctx.ntt_set_schedule(False, None)
        w.ctx.ntt_set_schedule(True, None)


@pytest.mark.parametrize("name", ["a6_n12", "a4_n15"])
def test_inner_product_row_kinds_concurrent_and_sequential(name):
    """The fused inner product's 60-bit rows run on the context's helper
    stream beside its fp64 rows, except while the family is timed per launch
    (then one after the other): both orders give the oracle's ciphertexts,
    for relinearisation and rotation of a batch."""
    import paper_1908_06972_amd.native as N
    w = world(name)
    sched = [c for c in w.col16 if c[1] == 0][0]
    w.ctx.ntt_set_schedule(False, sched)
    level = w.op.L
    pairs = [(w.enc_pair(200 + i, level), w.enc_pair(210 + i, level)) for i in range(2)]
    try:
        outs = []
        for mask in (0, 1 << 3):  # key inner product family timed: sequential
            N.check(w.ctx.lib.pft_prof_enable(w.ctx.handle, mask))
            rel = w.ctx.mul_relin_batch([p[0][0] for p in pairs], [p[1][0] for p in pairs])
            rot = w.ctx.rotate_batch([p[0][0] for p in pairs], STEPS[1])
            outs.append([w.ctx.export(g) for g in rel + rot])
        N.check(w.ctx.lib.pft_prof_enable(w.ctx.handle, 0))
        for a, b in zip(outs[0], outs[1]):
            assert np.array_equal(a, b)
        for ((_, oa), (_, ob)), host in zip(pairs, outs[0][:2]):
            o = C.hmul_relin(w.op, oa, ob, w.rlk)
            assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)
        for ((_, oa), _), host in zip(pairs, outs[0][2:]):
            o = C.rotate(w.op, oa, STEPS[1], w.rot[STEPS[1]])
            assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)
    finally:
        N.check(w.ctx.lib.pft_prof_enable(w.ctx.handle, 0))
        w.ctx.ntt_set_schedule(False, None)
