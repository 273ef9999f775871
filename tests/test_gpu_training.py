"""The encrypted-weight forward pass and the softmax approximation (Sec. 4.2)
on the GPU.

Bit-exact parity with the oracle uses integer plaintexts drawn by synth for
the encrypted diagonals and the inputs (both sides encrypt the same integer
polynomials with the same randomness, so no encoder sits between the shared
input and the compared residues).  The library's float path (its own
encoder) is checked against fp64: the matrix-vector product against M v and
the whole predict step against Alg. 1 steps 2-3 followed by the polynomial
X^2/8 + X/2 + 1/4."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM
from oracle import training as T

pytestmark = pytest.mark.gpu

TRAIN = dict(log_n=12, n_q=6, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=3, scale=2 ** 40)
DIM, CLS = 16, 4


class World:
    def __init__(self):
        import paper_1908_06972_amd.ckks as L
        self.L = L
        self.op = C.Params(**TRAIN)
        self.lp = L.Params(*TRAIN.values())
        assert self.op.q == self.lp.q and self.op.p == self.lp.p
        C.set_mul_mode(1)
        self.n = self.op.n
        self.t = self.n // 2
        self.ctx = L.Context(self.lp)
        kd = S.key_draws(23, self.n, self.op.q)
        self.kd = kd
        self.ctx.set_secret(kd.s)
        self.ctx.gen_public_key(kd.pk_a, kd.pk_e)
        self.pk = C.public_key(self.op, kd.s, kd.pk_a, kd.pk_e)
        a, e = S.switch_key_draws(23, 0, self.n, self.op.key_moduli(), self.op.dnum)
        self.ctx.gen_relin_key(a, e)
        self.rlk = C.relin_key(self.op, kd.s, a, e)
        self.keys = {}
        for st in sorted(set(PM.rotation_steps(DIM, self.t) + PM.rotation_steps(CLS, DIM))):
            a, e = S.switch_key_draws(23, 4000 + st, self.n, self.op.key_moduli(), self.op.dnum)
            self.ctx.gen_rotation_key(st, a, e)
            self.keys[st] = C.rotation_key(self.op, kd.s, st, a, e)

    def enc_pair(self, m, level, scale, seed):
        d = S.enc_draws(seed, self.n)
        return (self.ctx.encrypt(m, level, scale, d.v, d.e0, d.e1),
                C.encrypt(self.op, self.pk, m, level, d.v, d.e0, d.e1, scale))

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert g.level == o.level and g.scale == o.scale
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)

    def enc_diag_pairs(self, n_o, n_in, level, seed, bound):
        """Encrypted integer diagonals, [n_in][G][b] on both sides."""
        b, G = PM.bsgs_plan(n_o, n_in)
        qs = float(self.op.q[level - 1])
        g = S.rng(seed)
        gpu, orc, k = [], [], 0
        for c in range(n_in):
            oc = []
            for gg in range(G):
                og = []
                for r in range(b):
                    pair = self.enc_pair(S.plaintext_coeffs(g, self.n, bound), level, qs, seed * 100 + k)
                    gpu.append(pair[0])
                    og.append(pair[1])
                    k += 1
                oc.append(og)
            orc.append(oc)
        return gpu, orc


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    return World()


@pytest.mark.parametrize("value,level", [(2.0, 6), (-0.25, 3), (0.5, 1), (-3.0, 2)])
def test_add_const_parity(world, value, level):
    w = world
    x = w.enc_pair(S.plaintext_coeffs(S.rng(31), w.n, 2 ** 40), level, w.op.scale, 310)
    g = w.ctx.add_const_batch([x[0]], [value])[0]
    w.assert_same(g, T.hadd_const(w.op, x[1], value))


@pytest.mark.parametrize("n_o,n_i,n_in,lvl,docs", [(DIM, 2048, 2, 6, 2), (CLS, DIM, 1, 4, 3), (8, 64, 1, 3, 1)])
def test_ctmatvec_parity(world, n_o, n_i, n_in, lvl, docs):
    w = world
    steps = set(PM.rotation_steps(n_o, n_i))
    if not steps <= set(w.keys):
        for st in sorted(steps - set(w.keys)):
            a, e = S.switch_key_draws(23, 4000 + st, w.n, w.op.key_moduli(), w.op.dnum)
            w.ctx.gen_rotation_key(st, a, e)
            w.keys[st] = C.rotation_key(w.op, w.kd.s, st, a, e)
    gdiag, odiag = w.enc_diag_pairs(n_o, n_in, lvl, 40 + n_o, 2 ** 20)
    ins = [[w.enc_pair(S.plaintext_coeffs(S.rng(500 + 2 * d + c), w.n, 2 ** 30), lvl, w.op.scale,
                       600 + 2 * d + c) for c in range(n_in)] for d in range(docs)]
    outs = w.ctx.ctmatvec(gdiag, n_o, n_i, n_in, [[x[0] for x in doc] for doc in ins])
    for doc, g in zip(ins, outs):
        o = T.ctmatvec(w.op, [x[1] for x in doc], odiag, n_o, n_i, w.rlk, w.keys)
        w.assert_same(g, o)


def test_softmax_approx_parity(world):
    w = world
    xs = [w.enc_pair(S.plaintext_coeffs(S.rng(70 + i), w.n, 2 ** 40), 4, w.op.scale, 700 + i) for i in range(3)]
    from paper_1908_06972_amd import training as GT
    outs = GT.softmax_approx(w.ctx, [x[0] for x in xs])
    for x, g in zip(xs, outs):
        w.assert_same(g, T.softmax_approx(w.op, x[1], w.rlk))


def test_predict_encrypted_parity(world):
    """The whole predict step on integer inputs: residues bit-exact."""
    w = world
    from paper_1908_06972_amd import training as GT
    L = w.op.L
    g1, o1 = w.enc_diag_pairs(DIM, 2, L, 81, 2 ** 20)
    g2, o2 = w.enc_diag_pairs(CLS, 1, L - 2, 82, 2 ** 20)
    model = GT.EncryptedBowModel(g1, g2, DIM, CLS, 2, w.t)
    ins = [[w.enc_pair(S.plaintext_coeffs(S.rng(830 + 2 * d + c), w.n, 2 ** 30), L, w.op.scale, 840 + 2 * d + c)
            for c in range(2)] for d in range(2)]
    words = [37, 120]
    outs = GT.predict_encrypted(w.ctx, model, [[x[0] for x in doc] for doc in ins], words)
    for doc, wd, g in zip(ins, words, outs):
        o = T.predict_encrypted(w.op, [x[1] for x in doc], o1, o2, DIM, CLS, float(wd), w.rlk, w.keys)
        assert g.level == 1
        w.assert_same(g, o)


def _lib_enc(w, z, level, scale, seed):
    d = S.enc_draws(seed, w.n)
    return w.ctx.encrypt(w.lp.encode(z, scale), level, scale, d.v, d.e0, d.e1)


def _lib_dec(w, ct, n_slots):
    res = w.ctx.decrypt(ct)
    return w.lp.decode(res, ct.scale, n_slots).real


def _lib_diags(w, M, n_o, n_i, n_in, level, seed):
    qs = float(w.op.q[level - 1])
    D = PM.prerotated_diagonals(M, n_o, n_i, n_in, w.t)
    out, k = [], 0
    for per_c in D:
        for per_g in per_c:
            for d in per_g:
                out.append(_lib_enc(w, d, level, qs, seed + k))
                k += 1
    return out


def test_predict_encrypted_values(world):
    """Library encoder end to end: scores against Alg. 1 steps 2-3 and the
    softmax polynomial in fp64."""
    w = world
    from paper_1908_06972_amd import training as GT
    t, L = w.t, w.op.L
    V = 2 * t
    counts, words = S.bow_documents(91, 2, V, 20, 80)
    H, O = S.bow_weights(92, V, DIM, CLS)
    seed = [9500]

    def draws():
        seed[0] += 1
        d = S.enc_draws(seed[0], w.n)
        return d.v, d.e0, d.e1
    # stage 1 through the oracle's diagonal layout and the library encoder,
    # stage 2 through the library's own diagonal encoder
    model = GT.EncryptedBowModel(_lib_diags(w, H.T, DIM, t, 2, L, 9000),
                                 GT.encrypt_diagonals(w.ctx, O.T, CLS, DIM, 1, L - 2, draws), DIM, CLS, 2, t)
    docs = []
    for d in range(len(words)):
        v = counts[d].astype(np.float64)
        docs.append([_lib_enc(w, v[c * t:(c + 1) * t], L, w.op.scale, 9900 + 2 * d + c) for c in range(2)])
    outs = GT.predict_encrypted(w.ctx, model, docs, list(words))
    for d, g in enumerate(outs):
        got = _lib_dec(w, g, CLS)
        want = T.softmax_approx_plain(PM.inference_plain(counts[d].astype(np.float64), H, O, words[d]))
        assert np.max(np.abs(got - want)) <= 1e-5


def test_ctmatvec_errors(world):
    w = world
    x = w.enc_pair(S.plaintext_coeffs(S.rng(1), w.n, 2 ** 20), 4, w.op.scale, 11)[0]
    y = w.enc_pair(S.plaintext_coeffs(S.rng(2), w.n, 2 ** 20), 3, w.op.scale, 12)[0]
    b, G = PM.bsgs_plan(CLS)
    with pytest.raises(RuntimeError):  # diagonals at a different level than the input
        w.ctx.ctmatvec([y] * (b * G), CLS, DIM, 1, [[x]])
    with pytest.raises(RuntimeError):  # n_o not a power of two
        w.ctx.ctmatvec([x] * 3, 3, DIM, 1, [[x]])
    with pytest.raises(RuntimeError):  # no rotation keys for the baby steps 5..7 of n_o = 32
        w.ctx.ctmatvec([x] * 32, 32, 64, 1, [[x]])
