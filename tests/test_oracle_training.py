"""Pins of the oracle's encrypted-weight forward pass and degree-2 softmax
approximation (Sec. 4.2: the predict step of training with encrypted
weights, HMUL in place of HMULPLAIN, softmax ~ X^2/8 + X/2 + 1/4).

Exact: HADDPLAIN of a constant changes the decryption by exactly the
constant polynomial round(value * scale).  Within the noise bounds: the
encrypted-weight matrix-vector product against fp64 M v; one relinearisation
per giant step against one per diagonal product; the softmax approximation
against the polynomial in fp64; the whole predict step against Alg. 1 steps
2-3 followed by the polynomial, in fp64."""

import functools

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from oracle import ptmatvec as PM
from oracle import training as T

# six levels: stage 1, 1/w, stage 2, the square, 1/8 -- and one left
TRAIN = dict(log_n=12, n_q=6, q0_bits=60, q_bits=40, n_p=2, p_bits=60, dnum=3, scale=2 ** 40)
DIM, CLS = 16, 4


@functools.lru_cache(maxsize=1)
def make_train():
    P = C.Params(**TRAIN)
    C.set_mul_mode(1)
    kd = S.key_draws(21, P.n, P.q)
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(21, 0, P.n, P.key_moduli(), P.dnum)
    rlk = C.relin_key(P, kd.s, a, e)
    t = P.n // 2
    steps = sorted(set(PM.rotation_steps(DIM, t) + PM.rotation_steps(CLS, DIM)))
    keys = {}
    for st in steps:
        a, e = S.switch_key_draws(21, 3000 + st, P.n, P.key_moduli(), P.dnum)
        keys[st] = C.rotation_key(P, kd.s, st, a, e)
    return P, kd, pk, rlk, keys


@pytest.fixture(scope="module")
def train():
    C.set_mul_mode(1)
    return make_train()


def _enc(P, pk, z, level, scale, seed):
    d = S.enc_draws(seed, P.n)
    return C.encrypt(P, pk, C.encode(z, P.n, scale), level, d.v, d.e0, d.e1, scale)


def _dec(P, kd, ct, n_slots):
    return C.decode(C.decrypt(P, kd.s, ct), P.q[:ct.level], P.n, ct.scale, n_slots).real


def _enc_diags(P, pk, M, n_o, n_i, n_in, level, seed):
    """Pre-rotated diagonals of M, each encrypted at scale q_{level-1}."""
    t = P.n // 2
    qs = float(P.q[level - 1])
    D = PM.prerotated_diagonals(M, n_o, n_i, n_in, t)
    out, k = [], 0
    for per_c in D:
        rows = []
        for per_g in per_c:
            row = []
            for d in per_g:
                row.append(_enc(P, pk, d, level, qs, seed + k))
                k += 1
            rows.append(row)
        out.append(rows)
    return out


@pytest.mark.parametrize("value", [2.0, -0.25, 0.5, -3.0])
def test_hadd_const_exact(train, value):
    P, kd, pk, _, _ = train
    g = np.random.default_rng(5)
    ct = _enc(P, pk, g.uniform(-1, 1, 8), 3, P.scale, 600)
    out = T.hadd_const(P, ct, value)
    diff = C.crt_lift(C.sub(C.decrypt(P, kd.s, out), C.decrypt(P, kd.s, ct), P.q[:3]), P.q[:3])
    want = [0] * P.n
    want[0] = round(value * P.scale)  # exact here: value * 2^40 is an integer
    assert [int(x) for x in diff] == want
    assert out.scale == ct.scale


def test_softmax_polynomial_form():
    """(X + 2)^2 / 8 - 1/4 and X^2/8 + X/2 + 1/4 agree (the evaluation order
    the oracle uses versus the paper's form)."""
    x = np.linspace(-4, 4, 101)
    assert np.allclose((x + 2) ** 2 / 8 - 0.25, T.softmax_approx_plain(x), atol=1e-14)
    assert T.softmax_approx_plain(0.0) == 0.25 and T.softmax_approx_plain(-2.0) == -0.25
    assert T.softmax_approx_plain(2.0) == 1.75  # 4/8 + 2/2 + 1/4


def test_encrypted_softmax_approx(train):
    P, kd, pk, rlk, _ = train
    g = np.random.default_rng(7)
    z = g.uniform(-2, 2, 64)
    ct = _enc(P, pk, z, 3, P.scale, 610)
    y = T.softmax_approx(P, ct, rlk)
    assert y.level == 1
    got = _dec(P, kd, y, 64)
    assert np.max(np.abs(got - T.softmax_approx_plain(z))) <= 1e-6


def test_encrypted_ctmatvec(train):
    P, kd, pk, rlk, keys = train
    t = P.n // 2
    n_o, n_i, n_in = DIM, t, 2
    g = np.random.default_rng(11)
    M = g.normal(0, 0.1, size=(n_o, n_in * n_i))
    vs = [g.uniform(-1, 1, t) for _ in range(n_in)]
    lvl = P.L
    cts = [_enc(P, pk, v, lvl, P.scale, 620 + i) for i, v in enumerate(vs)]
    E = _enc_diags(P, pk, M, n_o, n_i, n_in, lvl, 700)
    out = C.rescale(P, T.ctmatvec(P, cts, E, n_o, n_i, rlk, keys))
    assert out.level == lvl - 1 and abs(out.scale / P.scale - 1) < 1e-12
    y = _dec(P, kd, out, t)
    want = (M @ np.concatenate(vs))[np.arange(t) % n_o]
    assert np.max(np.abs(y - want)) <= 1e-5


def test_lazy_relin_matches_per_product(train):
    """One relinearisation of the summed tensors decrypts to the sum of the
    individually relinearised products (up to key-switching noise)."""
    P, kd, pk, rlk, _ = train
    g = np.random.default_rng(13)
    xs = [_enc(P, pk, g.uniform(-1, 1, 32), 3, P.scale, 640 + i) for i in range(4)]
    ys = [_enc(P, pk, g.uniform(-1, 1, 32), 3, P.scale, 650 + i) for i in range(4)]
    lazy = T.relin_tensor(P, T._tensor_sum(P, list(zip(xs, ys))), rlk, P.scale ** 2)
    each = None
    for x, y in zip(xs, ys):
        h = C.hmul_relin(P, x, y, rlk)
        each = h if each is None else C.hadd(P, each, h)
    a = _dec(P, kd, C.rescale(P, lazy), 32)
    b = _dec(P, kd, C.rescale(P, each), 32)
    assert np.max(np.abs(a - b)) <= 1e-6


def test_predict_encrypted_matches_plain(train):
    """Sec. 4.2 predict with encrypted H and O, then the softmax polynomial,
    against Alg. 1 steps 2-3 and the polynomial in fp64."""
    P, kd, pk, rlk, keys = train
    t = P.n // 2
    V = 2 * t
    counts, w = S.bow_documents(41, 1, V, 20, 80)
    H, O = S.bow_weights(42, V, DIM, CLS)
    v = counts[0].astype(np.float64)
    cts = [_enc(P, pk, v[c * t:(c + 1) * t], P.L, P.scale, 660 + c) for c in range(2)]
    EH = _enc_diags(P, pk, H.T, DIM, t, 2, P.L, 800)
    EO = _enc_diags(P, pk, O.T, CLS, DIM, 1, P.L - 2, 900)
    y = T.predict_encrypted(P, cts, EH, EO, DIM, CLS, float(w[0]), rlk, keys)
    assert y.level == 1
    got = _dec(P, kd, y, CLS)
    want = T.softmax_approx_plain(PM.inference_plain(v, H, O, w[0]))
    assert np.max(np.abs(got - want)) <= 1e-5
