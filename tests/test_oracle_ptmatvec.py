"""Pins of the oracle's PtMatVec (diagonal method with baby-step/giant-step)
and of the encrypted bag-of-words inference (Sec. 4.1, Alg. 1 steps 2-3).

The BSGS identity is checked on plain slot vectors against a direct matrix
product for many shapes; the encrypted evaluation is checked against fp64
M v and the inference scores against Alg. 1 in fp64 (argmax equality: the
paper's "no accuracy loss" claim for inference)."""

import math

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM


@pytest.mark.parametrize("n_o", [1, 2, 4, 8, 16, 32, 64, 128, 1024])
def test_bsgs_plan(n_o):
    b, G = PM.bsgs_plan(n_o)
    assert b * G == n_o and b >= G and b & (b - 1) == 0
    assert b == 2 ** math.ceil(math.log2(n_o) / 2)


@pytest.mark.parametrize("n_o,n_in", [(n_o, n_in) for n_o in (1, 2, 4, 8, 16, 64, 256) for n_in in (1, 2, 3, 5, 17, 123)])
def test_bsgs_plan_minimises_rotations(n_o, n_in):
    """b minimises n_in (b - 1) + (n_o/b - 1) over powers of two (brute
    force), the larger b on ties."""
    b, G = PM.bsgs_plan(n_o, n_in)
    cost = lambda bb: n_in * (bb - 1) + n_o // bb - 1  # noqa: E731
    cands = [1 << k for k in range(int(math.log2(n_o)) + 1)]
    best = min(cost(bb) for bb in cands)
    assert cost(b) == best and b == max(bb for bb in cands if cost(bb) == best) and b * G == n_o


def test_bsgs_plan_examples():
    assert PM.bsgs_plan(64, 1) == (8, 8) and PM.bsgs_plan(64, 2) == (8, 8)
    assert PM.bsgs_plan(64, 123) == (1, 64)  # many inputs: giant steps only
    assert PM.bsgs_plan(16, 5) == (2, 8)


@pytest.mark.parametrize("n_o,n_i,n_in,t", [(4, 16, 1, 16), (8, 64, 2, 64), (8, 64, 1, 512), (64, 1024, 2, 1024),
                                            (16, 16, 1, 256), (1, 8, 3, 32), (16, 64, 5, 64), (64, 64, 9, 128)])
def test_slot_bsgs_equals_matvec(n_o, n_i, n_in, t):
    """Slot k of the BSGS result equals (M v)_{k mod n_o}, where the input is
    n_in vectors of t slots, each periodic with period n_i."""
    g = np.random.default_rng(n_o * 1000 + n_i + n_in)
    M = g.normal(size=(n_o, n_in * n_i))
    parts = [g.normal(size=n_i) for _ in range(n_in)]
    vs = [np.tile(p, t // n_i) for p in parts]
    P = PM.prerotated_diagonals(M, n_o, n_i, n_in, t)
    y = PM.slot_bsgs(P, vs, n_o, n_i)
    want = M @ np.concatenate(parts)
    assert np.allclose(y, want[np.arange(t) % n_o], atol=1e-9)


def test_rotation_steps():
    assert PM.rotation_steps(64, 16384) == list(range(1, 8)) + [8 * g for g in range(1, 8)] + \
        [64 * 2 ** s for s in range(8)]
    assert PM.rotation_steps(8, 64) == [1, 2, 3, 4, 8, 16, 32]


SMALL = dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40)


@pytest.fixture(scope="module")
def small():
    P = C.Params(**SMALL)
    C.set_mul_mode(1)
    kd = S.key_draws(9, P.n, P.q)
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    steps = sorted(set(PM.rotation_steps(16, 2048) + PM.rotation_steps(4, 16)))
    keys = {}
    for st in steps:
        a, e = S.switch_key_draws(9, 2000 + st, P.n, P.key_moduli(), P.dnum)
        keys[st] = C.rotation_key(P, kd.s, st, a, e)
    return P, kd, pk, keys


def _enc(P, pk, z, level, seed):
    d = S.enc_draws(seed, P.n)
    return C.encrypt(P, pk, C.encode(z, P.n, P.scale), level, d.v, d.e0, d.e1, P.scale)


def _dec(P, kd, ct, n_slots):
    return C.decode(C.decrypt(P, kd.s, ct), P.q[:ct.level], P.n, ct.scale, n_slots).real


def _encode_plains(P, M, n_o, n_i, n_in, level):
    t = P.n // 2
    pt_scale = float(P.q[level - 1])
    diags = PM.prerotated_diagonals(M, n_o, n_i, n_in, t)
    plains = [[[C.encode(d, P.n, pt_scale) for d in per_g] for per_g in per_c] for per_c in diags]
    return plains, pt_scale


def test_encrypted_ptmatvec(small):
    P, kd, pk, keys = small
    t = P.n // 2
    n_o, n_i, n_in = 16, t, 2
    g = np.random.default_rng(12)
    M = g.normal(0, 0.1, size=(n_o, n_in * n_i))
    vs = [g.uniform(-1, 1, t) for _ in range(n_in)]
    cts = [_enc(P, pk, v, P.L, 50 + i) for i, v in enumerate(vs)]
    plains, pt_scale = _encode_plains(P, M, n_o, n_i, n_in, P.L)
    out = C.rescale(P, PM.ptmatvec(P, cts, plains, n_o, n_i, keys, pt_scale))
    assert out.level == P.L - 1 and abs(out.scale / P.scale - 1) < 1e-12
    y = _dec(P, kd, out, t)
    want = (M @ np.concatenate(vs))[np.arange(t) % n_o]
    # input noise ~2^-26 per slot times the row L1 norm of M (~330), plus one
    # key switch per rotation and the plaintext rounding (N/scale per term)
    assert np.max(np.abs(y - want)) <= 1e-5


def test_encrypted_inference_matches_plain(small):
    """Alg. 1 steps 2-3 under encryption: v H (stage 1), times 1/w, then h O
    (stage 2), one rescale after each; scores and argmax against fp64."""
    P, kd, pk, keys = small
    t = P.n // 2
    V, dim, classes = 2 * t, 16, 4
    counts, w = S.bow_documents(31, 3, V, 20, 80)
    H, O = S.bow_weights(32, V, dim, classes)
    plains1, s1 = _encode_plains(P, H.T, dim, t, 2, P.L)
    plains2, s2 = _encode_plains(P, O.T, classes, dim, 1, P.L - 2)
    for d in range(len(w)):
        v = counts[d].astype(np.float64)
        cts = [_enc(P, pk, v[c * t:(c + 1) * t], P.L, 70 + 2 * d + c) for c in range(2)]
        h = C.rescale(P, PM.ptmatvec(P, cts, plains1, dim, t, keys, s1))
        m, ms = PM.constant_plain(P, 1.0 / w[d], h.level)
        h = C.rescale(P, C.hmul_plain(P, h, m, ms))
        s = C.rescale(P, PM.ptmatvec(P, [h], plains2, classes, dim, keys, s2))
        assert s.level == 1
        scores = _dec(P, kd, s, classes)
        want = PM.inference_plain(v, H, O, w[d])
        assert np.max(np.abs(scores - want)) <= 1e-5
        srt = np.sort(want)
        if srt[-1] - srt[-2] > 2e-5:
            assert np.argmax(scores) == np.argmax(want)
