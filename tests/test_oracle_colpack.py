"""Pins of the oracle's column-packed inference (Sec. 4.1, the paper's own
matrix packing: vertically packed H, one TotalSum per column, horizontally
packed O).

Plain slot vectors: the packing helpers against direct slicing, and
TotalSum-by-rotations against the slot sum.  Encrypted (N = 2^12): stage 1
leaves (v H)_j in every slot of h_j; the scores against Alg. 1 steps 2-3 in
fp64 with argmax equality; stage 1 costs exactly n log2(t) rotations."""

import functools
import math

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import colpack as CP
from oracle import ptmatvec as PM

SMALL = dict(log_n=12, n_q=4, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=2, scale=2 ** 40)
DIM, CLS = 8, 4


def test_packing_helpers():
    g = np.random.default_rng(1)
    t = 64
    H = g.normal(size=(3 * t - 10, 5))
    cols = CP.column_slots(H, t)
    assert cols.shape == (5, 3, t)
    for j in range(5):
        assert np.array_equal(cols[j].reshape(-1)[:H.shape[0]], H[:, j])
        assert not cols[j].reshape(-1)[H.shape[0]:].any()
    O = g.normal(size=(5, 3))
    rows = CP.row_slots(O, t)
    assert np.array_equal(rows[:, :3], O) and not rows[:, 3:].any()


def test_totalsum_by_rotations_is_slot_sum():
    """Alg. 2 on plain slots: x + rot(x, 1), then + rot(., 2), ... leaves the
    sum of all t slots in every slot."""
    g = np.random.default_rng(2)
    t = 256
    x = g.normal(size=t)
    y = x.copy()
    for i in range(int(math.log2(t))):
        y = y + np.roll(y, -(1 << i))
    assert np.allclose(y, x.sum(), atol=1e-9)


@functools.lru_cache(maxsize=1)
def make_small():
    P = C.Params(**SMALL)
    C.set_mul_mode(1)
    kd = S.key_draws(15, P.n, P.q)
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    t = P.n // 2
    keys = {}
    for i in range(int(math.log2(t))):
        a, e = S.switch_key_draws(15, 5000 + (1 << i), P.n, P.key_moduli(), P.dnum)
        keys[1 << i] = C.rotation_key(P, kd.s, 1 << i, a, e)
    return P, kd, pk, keys


@pytest.fixture(scope="module")
def small():
    C.set_mul_mode(1)
    return make_small()


def _enc(P, pk, z, level, seed):
    d = S.enc_draws(seed, P.n)
    return C.encrypt(P, pk, C.encode(z, P.n, P.scale), level, d.v, d.e0, d.e1, P.scale)


def _dec(P, kd, ct, n_slots):
    return C.decode(C.decrypt(P, kd.s, ct), P.q[:ct.level], P.n, ct.scale, n_slots).real


def _plains(P, slots, level):
    qs = float(P.q[level - 1])
    return [[C.encode(v, P.n, qs) for v in row] for row in slots], qs


def _model(P, V, seed):
    t = P.n // 2
    H, O = S.bow_weights(seed, V, DIM, CLS)
    ph, sh = _plains(P, CP.column_slots(H, t), P.L)
    po = [C.encode(v, P.n, float(P.q[P.L - 3])) for v in CP.row_slots(O, t)]
    return H, O, ph, sh, po, float(P.q[P.L - 3])


def test_stage1_replicates_column_dot(small):
    P, kd, pk, keys = small
    t = P.n // 2
    V = 3 * t - 100  # ragged: the last input ciphertext is zero padded
    H, O, ph, sh, _, _ = _model(P, V, 33)
    counts, _ = S.bow_documents(34, 1, V, 20, 60)
    v = np.zeros(3 * t)
    v[:V] = counts[0]
    cts = [_enc(P, pk, v[c * t:(c + 1) * t], P.L, 340 + c) for c in range(3)]
    hs = [C.rescale(P, h) for h in CP.stage1(P, cts, ph, sh, keys)]
    want = counts[0].astype(np.float64) @ H
    for j, h in enumerate(hs):
        got = _dec(P, kd, h, t)
        assert np.max(np.abs(got - want[j])) <= 1e-5


def test_stage1_rotation_count(small, monkeypatch):
    """n TotalSums of log2(t) rotations each: n log2(t) key switches."""
    P, kd, pk, keys = small
    t = P.n // 2
    H, O, ph, sh, _, _ = _model(P, 2 * t, 35)
    cts = [_enc(P, pk, np.zeros(t), P.L, 350 + c) for c in range(2)]
    calls = []
    real = C.rotate
    monkeypatch.setattr(C, "rotate", lambda *a, **k: calls.append(1) or real(*a, **k))
    CP.stage1(P, cts, ph, sh, keys)
    assert len(calls) == DIM * int(math.log2(t))


def test_encrypted_colpack_inference(small):
    P, kd, pk, keys = small
    t = P.n // 2
    V = 2 * t
    H, O, ph, sh, po, so = _model(P, V, 36)
    counts, w = S.bow_documents(37, 2, V, 20, 80)
    for d in range(len(w)):
        v = counts[d].astype(np.float64)
        cts = [_enc(P, pk, v[c * t:(c + 1) * t], P.L, 360 + 2 * d + c) for c in range(2)]
        s = CP.inference(P, cts, ph, sh, po, so, float(w[d]), keys, PM.constant_plain)
        assert s.level == P.L - 3
        scores = _dec(P, kd, s, CLS)
        want = PM.inference_plain(v, H, O, w[d])
        assert np.max(np.abs(scores - want)) <= 1e-5
        srt = np.sort(want)
        if srt[-1] - srt[-2] > 2e-5:
            assert np.argmax(scores) == np.argmax(want)
