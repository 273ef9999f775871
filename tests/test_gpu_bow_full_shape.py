"""Encrypted bag-of-words inference at its full shape against the oracle.

Shape: N = 2^15, 16 ciphertext primes (+4 special, dnum 4), vocabulary 32768
over two input ciphertexts of 16384 slots, embedding 64, 8 classes, a batch
of 32 documents on the GPU (Sec. 4.1, Alg. 1 steps 2-3 by HMULPLAIN, HADD and
ROTATE: stage 1 v H, RESCALE, the 1/w average, RESCALE, stage 2 h O,
RESCALE).

The pre-rotated diagonals of H^T (64 per input ciphertext) and of O^T (8)
and the documents' count vectors are encoded by the oracle's encoder, and
both sides take those integer plaintexts (pft_ptmat_create_from_coeffs on
the library side), so the first and last documents of the batch are compared
bit for bit through the whole three-level chain; their decoded scores also
match Alg. 1 steps 2-3 in fp64."""

import types

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM
from tests.gpu_env import World

pytestmark = pytest.mark.gpu

N_DOCS = 32
CHECKED = (0, N_DOCS - 1)
DIM, CLASSES, N_IN = 64, 8, 2


class BowWorld:
    def __init__(self):
        from paper_1908_06972_amd.inference import encrypted_inference, split_counts
        cfg = S.CONFIGS["C4"]
        t = (1 << cfg.log_n) // 2
        self.t = t
        steps = sorted(set(PM.rotation_steps(DIM, t, N_IN) + PM.rotation_steps(CLASSES, DIM, 1)))
        self.w = w = World(cfg, seed=45, rot_steps=steps, relin=False)
        op, n, L = w.op, w.n, w.op.L
        H, O = S.bow_weights(404, N_IN * t, DIM, CLASSES)
        self.H, self.O = H, O
        self.s1, self.s2 = float(op.q[L - 1]), float(op.q[L - 3])
        enc = lambda v, scale: C.encode(v, n, scale)  # noqa: E731
        self.p1 = np.array([[[enc(d, self.s1) for d in per_g] for per_g in per_c]
                            for per_c in PM.prerotated_diagonals(H.T, DIM, t, N_IN, t)])
        self.p2 = np.array([[[enc(d, self.s2) for d in per_g] for per_g in per_c]
                            for per_c in PM.prerotated_diagonals(O.T, CLASSES, DIM, 1, t)])
        m1 = w.ctx.ptmat_from_coeffs(self.p1, DIM, t, N_IN, L, self.s1)
        m2 = w.ctx.ptmat_from_coeffs(self.p2, CLASSES, DIM, 1, L - 2, self.s2)
        assert (m1.b, m1.G) == PM.bsgs_plan(DIM, N_IN) and (m2.b, m2.G) == PM.bsgs_plan(CLASSES, 1)
        self.counts, self.words = S.bow_documents(405, N_DOCS, N_IN * t)
        self.plains = [[enc(v, op.scale) for v in split_counts(self.counts[d], N_IN, t)] for d in range(N_DOCS)]
        pairs = [[w.encrypt_pair(m, L, 4500 + N_IN * d + c) if d in CHECKED else None
                  for c, m in enumerate(self.plains[d])] for d in range(N_DOCS)]
        gpu_in = []
        for d in range(N_DOCS):
            if d in CHECKED:
                gpu_in.append([p[0] for p in pairs[d]])
            else:
                gpu_in.append([w.ctx.encrypt(m, L, op.scale, *_draws(4500 + N_IN * d + c, n))
                               for c, m in enumerate(self.plains[d])])
        self.oracle_in = {d: [p[1] for p in pairs[d]] for d in CHECKED}
        model = types.SimpleNamespace(stage1=m1, stage2=m2)
        self.scores = encrypted_inference(w.ctx, model, gpu_in, list(self.words))

    def oracle_scores(self, d):
        op, t, keys = self.w.op, self.t, self.w.rot
        o = C.rescale(op, PM.ptmatvec(op, self.oracle_in[d], self.p1, DIM, t, keys, self.s1))
        m, ms = PM.constant_plain(op, 1.0 / float(self.words[d]), o.level)
        o = C.rescale(op, C.hmul_plain(op, o, m, ms))
        return C.rescale(op, PM.ptmatvec(op, [o], self.p2, CLASSES, DIM, keys, self.s2))


def _draws(seed, n):
    d = S.enc_draws(seed, n)
    return d.v, d.e0, d.e1


@pytest.fixture(scope="module")
def bow():
    import torch
    assert torch.cuda.is_available()
    return BowWorld()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("d", CHECKED)
def test_bow_full_shape_matches_oracle(bow, d):
    g = bow.scores[d]
    assert g.level == bow.w.op.L - 3
    bow.w.assert_same(g, bow.oracle_scores(d))
    got = bow.w.lp.decode(bow.w.ctx.decrypt(g), g.scale, CLASSES).real
    want = PM.inference_plain(bow.counts[d].astype(np.float64), bow.H, bow.O, bow.words[d])
    assert np.max(np.abs(got - want)) <= 1e-5
