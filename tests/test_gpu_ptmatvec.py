"""PtMatVec and the encrypted bag-of-words inference on the GPU.

Bit-exact parity with the oracle uses integer plaintexts for the diagonals
drawn by synth (so no encoder sits between the shared input and the
compared residues); the library's own float path (host encoder of the
diagonals) is checked against fp64 M v and against the plaintext fasttext
scores (Alg. 1 steps 2-3) at the bag-of-words shapes."""

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM

pytestmark = pytest.mark.gpu

SMALL = dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40)


class SmallWorld:
    def __init__(self, steps):
        import paper_1908_06972_amd.ckks as L
        self.op = C.Params(**SMALL)
        self.lp = L.Params(*SMALL.values())
        assert self.op.q == self.lp.q and self.op.p == self.lp.p
        C.set_mul_mode(1)
        self.n = self.op.n
        self.ctx = L.Context(self.lp)
        kd = S.key_draws(9, self.n, self.op.q)
        self.kd = kd
        self.ctx.set_secret(kd.s)
        self.ctx.gen_public_key(kd.pk_a, kd.pk_e)
        self.pk = C.public_key(self.op, kd.s, kd.pk_a, kd.pk_e)
        self.keys = {}
        for st in steps:
            a, e = S.switch_key_draws(9, 2000 + st, self.n, self.op.key_moduli(), self.op.dnum)
            self.ctx.gen_rotation_key(st, a, e)
            self.keys[st] = C.rotation_key(self.op, kd.s, st, a, e)

    def enc_pair(self, m, level, seed):
        d = S.enc_draws(seed, self.n)
        return (self.ctx.encrypt(m, level, self.op.scale, d.v, d.e0, d.e1),
                C.encrypt(self.op, self.pk, m, level, d.v, d.e0, d.e1, self.op.scale))

    def assert_same(self, g, o):
        host = self.ctx.export(g)
        assert g.level == o.level and g.scale == o.scale
        assert np.array_equal(host[0], o.c0) and np.array_equal(host[1], o.c1)


@pytest.fixture(scope="module")
def small():
    import torch
    assert torch.cuda.is_available()
    steps = sorted(set(PM.rotation_steps(16, 2048) + PM.rotation_steps(4, 16) + PM.rotation_steps(16, 16, 9)))
    return SmallWorld(steps)


def _random_plains(seed, n_in, n_o, n, bound):
    b, G = PM.bsgs_plan(n_o, n_in)
    g = S.rng(seed)
    arr = np.stack([np.stack([np.stack([S.plaintext_coeffs(g, n, bound) for _ in range(b)]) for _ in range(G)])
                    for _ in range(n_in)])
    return arr  # [n_in][G][b][N]


def test_ptmatvec_parity(small):
    w = small
    t = w.n // 2
    n_o, n_i, n_in, lvl = 16, t, 2, 4
    plains = _random_plains(5, n_in, n_o, w.n, 2 ** 30)
    pt_scale = float(w.op.q[lvl - 1])
    mat = w.ctx.ptmat_from_coeffs(plains, n_o, n_i, n_in, lvl, pt_scale)
    assert (mat.b, mat.G) == PM.bsgs_plan(n_o, n_in)
    docs = [[w.enc_pair(S.plaintext_coeffs(S.rng(100 + 2 * d + c), w.n, 2 ** 40), lvl, 200 + 2 * d + c)
             for c in range(n_in)] for d in range(3)]
    outs = w.ctx.ptmatvec(mat, [[x[0] for x in doc] for doc in docs])
    for doc, g in zip(docs, outs):
        o = PM.ptmatvec(w.op, [x[1] for x in doc], plains, n_o, n_i, w.keys, pt_scale)
        w.assert_same(g, o)


def test_periodic_ptmatvec_parity(small):
    """Stage-2 shape: n_o = 4 outputs from a 16-periodic input, one ciphertext."""
    w = small
    plains = _random_plains(6, 1, 4, w.n, 2 ** 30)
    pt_scale = float(w.op.q[1])
    mat = w.ctx.ptmat_from_coeffs(plains, 4, 16, 1, 2, pt_scale)
    g, o = w.enc_pair(S.plaintext_coeffs(S.rng(7), w.n, 2 ** 40), 2, 300)
    w.assert_same(w.ctx.ptmatvec(mat, [[g]])[0], PM.ptmatvec(w.op, [o], plains, 4, 16, w.keys, pt_scale))


def test_inference_chain_parity(small):
    """stage 1 -> rescale -> x 1/w -> rescale -> stage 2 -> rescale, batched
    over documents, bit-exact per document."""
    w = small
    t = w.n // 2
    p1 = _random_plains(8, 2, 16, w.n, 2 ** 20)
    p2 = _random_plains(9, 1, 4, w.n, 2 ** 20)
    s1, s2 = float(w.op.q[3]), float(w.op.q[1])
    m1 = w.ctx.ptmat_from_coeffs(p1, 16, t, 2, 4, s1)
    m2 = w.ctx.ptmat_from_coeffs(p2, 4, 16, 1, 2, s2)
    words = [57, 312, 1]
    docs = [[w.enc_pair(S.plaintext_coeffs(S.rng(400 + 2 * d + c), w.n, 2 ** 36), 4, 500 + 2 * d + c)
             for c in range(2)] for d in range(len(words))]
    h = w.ctx.rescale_batch(w.ctx.ptmatvec(m1, [[x[0] for x in doc] for doc in docs]))
    h = w.ctx.rescale_batch(w.ctx.mul_const_batch(h, [1.0 / x for x in words]))
    s = w.ctx.rescale_batch(w.ctx.ptmatvec(m2, [[x] for x in h]))
    for d, doc in enumerate(docs):
        o = C.rescale(w.op, PM.ptmatvec(w.op, [x[1] for x in doc], p1, 16, t, w.keys, s1))
        m, ms = PM.constant_plain(w.op, 1.0 / words[d], o.level)
        o = C.rescale(w.op, C.hmul_plain(w.op, o, m, ms))
        o = C.rescale(w.op, PM.ptmatvec(w.op, [o], p2, 4, 16, w.keys, s2))
        w.assert_same(s[d], o)


def test_ptmatvec_float_path(small):
    """Library encoder of the diagonals: decrypted result equals fp64 M v."""
    w = small
    t = w.n // 2
    g = np.random.default_rng(12)
    M = g.normal(0, 0.1, size=(16, 2 * t))
    vs = [g.uniform(-1, 1, t) for _ in range(2)]
    mat = w.ctx.ptmat(M, 16, t, 2, 4)
    cts = []
    for i, v in enumerate(vs):
        d = S.enc_draws(50 + i, w.n)
        cts.append(w.ctx.encrypt(w.lp.encode(v), 4, w.op.scale, d.v, d.e0, d.e1))
    out = w.ctx.rescale(w.ctx.ptmatvec(mat, [cts])[0])
    y = w.lp.decode(w.ctx.decrypt(out), out.scale, t).real
    want = (M @ np.concatenate(vs))[np.arange(t) % 16]
    assert np.max(np.abs(y - want)) <= 1e-5


@pytest.mark.parametrize("n_docs", [4])
def test_bow_inference_c4(n_docs):
    """Bag-of-words shapes: N = 2^15, 16 limbs, vocabulary 32768 (two input
    ciphertexts), embedding 64, 8 classes; scores against Alg. 1 in fp64 and
    argmax equality."""
    import torch
    assert torch.cuda.is_available()
    import paper_1908_06972_amd.ckks as L
    from paper_1908_06972_amd.inference import BowModel, encrypted_inference, split_counts
    cfg = S.CONFIGS["C4"]
    lp = L.Params.from_config(cfg)
    ctx = L.Context(lp)
    n = lp.n
    kd = S.key_draws(44, n, lp.q)
    ctx.set_secret(kd.s)
    ctx.gen_public_key(kd.pk_a, kd.pk_e)
    H, O = S.bow_weights(404, 32768, 64, 8)
    model = BowModel(ctx, H, O, lp.L)
    assert model.n_in == 2
    for st in model.rotation_steps():
        a, e = S.switch_key_draws(44, 3000 + st, n, lp.key_moduli(), lp.dnum)
        ctx.gen_rotation_key(st, a, e)
    counts, words = S.bow_documents(405, n_docs, 32768)
    inputs = []
    for d in range(n_docs):
        cts = []
        for c, v in enumerate(split_counts(counts[d], model.n_in, model.t)):
            r = S.enc_draws(4000 + 2 * d + c, n)
            cts.append(ctx.encrypt(lp.encode(v), lp.L, lp.scale, r.v, r.e0, r.e1))
        inputs.append(cts)
    scores = encrypted_inference(ctx, model, inputs, words)
    for d in range(n_docs):
        assert scores[d].level == lp.L - 3
        got = lp.decode(ctx.decrypt(scores[d]), scores[d].scale, model.classes).real
        want = PM.inference_plain(counts[d].astype(np.float64), H, O, words[d])
        assert np.max(np.abs(got - want)) <= 1e-5
        srt = np.sort(want)
        if srt[-1] - srt[-2] > 2e-5:
            assert np.argmax(got) == np.argmax(want)


def test_ptmatvec_many_inputs_giant_steps_only(small):
    """70 input ciphertexts: the plan takes b = 1 (giant steps only) and the
    inputs are staged in several batches; bit-exact with the oracle."""
    w = small
    n_o, n_i, n_in, lvl = 4, 16, 70, 3
    assert PM.bsgs_plan(n_o, n_in) == (1, 4)
    plains = _random_plains(7, n_in, n_o, w.n, 2 ** 20)
    pt_scale = float(w.op.q[lvl - 1])
    mat = w.ctx.ptmat_from_coeffs(plains, n_o, n_i, n_in, lvl, pt_scale)
    assert (mat.b, mat.G) == (1, 4)
    doc = [w.enc_pair(S.plaintext_coeffs(S.rng(900 + c), w.n, 2 ** 30), lvl, 1000 + c) for c in range(n_in)]
    g = w.ctx.ptmatvec(mat, [[x[0] for x in doc]])[0]
    o = PM.ptmatvec(w.op, [x[1] for x in doc], plains, n_o, n_i, w.keys, pt_scale)
    w.assert_same(g, o)


def test_ptmatvec_sixteen_giant_steps(small):
    """9 input ciphertexts and 16 outputs: the plan takes b = 1 and G = 16,
    so the giant steps' inner sums come from two passes over the inputs
    (eight giant steps each); two documents, bit-exact with the oracle."""
    w = small
    n_o, n_i, n_in, lvl = 16, 16, 9, 3
    assert PM.bsgs_plan(n_o, n_in) == (1, 16)
    plains = _random_plains(11, n_in, n_o, w.n, 2 ** 20)
    pt_scale = float(w.op.q[lvl - 1])
    mat = w.ctx.ptmat_from_coeffs(plains, n_o, n_i, n_in, lvl, pt_scale)
    assert (mat.b, mat.G) == (1, 16)
    docs = [[w.enc_pair(S.plaintext_coeffs(S.rng(1100 + n_in * d + c), w.n, 2 ** 30), lvl, 1200 + n_in * d + c)
             for c in range(n_in)] for d in range(2)]
    outs = w.ctx.ptmatvec(mat, [[x[0] for x in doc] for doc in docs])
    for doc, g in zip(docs, outs):
        w.assert_same(g, PM.ptmatvec(w.op, [x[1] for x in doc], plains, n_o, n_i, w.keys, pt_scale))
