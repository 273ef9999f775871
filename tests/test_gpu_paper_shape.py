"""The paper's column-packed inference stage at its own inference shapes
(Sec. 4.1 matrix packing; Sec. 6: N = 8192, five 40-bit primes, 500000
words in 123 input ciphertexts, embedding 50): the library computes all 50
columns sum_j in_j P_{k,j} followed by TotalSum over the 4096 slots; three
sampled columns are compared bit for bit with the oracle, which computes
each of them on its own (HMULPLAIN of the 123 inputs, HADD, Alg. 2).
Integer plaintexts drawn by synth stand in for the encoded weights (no
encoder between the shared input and the compared residues)."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import colpack as CP

pytestmark = pytest.mark.gpu

SHAPE = dict(log_n=13, n_q=5, q0_bits=40, q_bits=40, n_p=1, p_bits=60, dnum=5, scale=2 ** 40)
N_IN, DIM = 123, 50
SAMPLED = (0, 23, 49)


def test_colpack_stage1_paper_shape_sampled_columns(torch_cuda):
    import paper_1908_06972_amd.ckks as L
    op = C.Params(**SHAPE)
    lp = L.Params(*SHAPE.values())
    assert op.q == lp.q and op.p == lp.p
    C.set_mul_mode(1)
    n, t, lvl = op.n, op.n // 2, op.L
    ctx = L.Context(lp)
    kd = S.key_draws(91, n, op.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    pk = C.public_key(op, kd.s, kd.pk_a, kd.pk_e)
    keys = {}
    for i in range(12):  # TotalSum over 4096 slots: steps 2^0 .. 2^11
        st = 1 << i
        a, e = S.switch_key_draws(91, 9000 + st, n, op.key_moduli(), op.dnum)
        ctx.gen_rotation_key(st, a, e)
        keys[st] = C.rotation_key(op, kd.s, st, a, e)
    g_ins, o_ins = [], []
    for j in range(N_IN):
        m = S.plaintext_coeffs(S.rng(9300 + j), n, 2 ** 30)
        d = S.enc_draws(9100 + j, n)
        g_ins.append(ctx.encrypt(m, lvl, op.scale, d.v, d.e0, d.e1))
        o_ins.append(C.encrypt(op, pk, m, lvl, d.v, d.e0, d.e1, op.scale))
    g = S.rng(9500)
    plains = np.stack([np.stack([S.plaintext_coeffs(g, n, 2 ** 20) for _ in range(N_IN)]) for _ in range(DIM)])
    pt_scale = float(op.q[lvl - 1])
    mat = ctx.ptdot_from_coeffs(plains, lvl, pt_scale)
    outs = ctx.ptdot_apply(mat, [g_ins], n_sum=t)[0]
    assert len(outs) == DIM
    for k in SAMPLED:
        o = C.total_sum(op, CP.dot_plain(op, o_ins, list(plains[k]), pt_scale), t, keys)
        host = ctx.export(outs[k])
        assert outs[k].level == o.level and outs[k].scale == o.scale
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1), k
