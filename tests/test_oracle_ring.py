"""Pins of the oracle's ring layer against mathematics it does not share code
with: sympy primality and CRT, big-integer polynomial products, Horner
evaluation at the roots of X^N+1, and exact floor/round of Eq. (1)."""

import math

import numpy as np
import pytest
import sympy

from oracle import ckks as C
from oracle import _ring
from synth import CONFIGS
from tests.intpoly import bitrev, crt_value, evaluate, negacyclic_int


def _rand_res(g, q, n):
    return g.integers(0, q, size=n, dtype=np.uint64)


def test_is_prime_matches_sympy():
    g = np.random.default_rng(7)
    cands = [int(x) | 1 for x in g.integers(2 ** 39, 2 ** 61, size=400, dtype=np.uint64)]
    cands += [2, 3, 4, 561, 1105, 3215031751, 2 ** 61 - 1, 2 ** 59 + 1]
    for x in cands:
        assert C.is_prime(x) == sympy.isprime(x), x


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_prime_chain(name):
    cfg = CONFIGS[name]
    q, p = C.prime_chain(cfg.log_n, cfg.n_q, cfg.q0_bits, cfg.q_bits, cfg.n_p, cfg.p_bits)
    two_n = 2 * cfg.n
    assert len(q) == cfg.n_q and len(p) == cfg.n_p
    assert len(set(q + p)) == len(q + p)
    for x in q + p:
        assert sympy.isprime(x) and x % two_n == 1 and x < 2 ** 60 + 1
    assert q[0].bit_length() == cfg.q0_bits
    assert all(x.bit_length() == cfg.q_bits for x in q[1:])
    assert all(x.bit_length() == cfg.p_bits for x in p)
    # last prime of the chain is the smallest: strictly descending (Sec. 5.1)
    assert all(q[i] > q[i + 1] for i in range(len(q) - 1))
    # "largest": no skipped prime = 1 mod 2N between consecutive q_1.. picks
    for lo, hi in zip(q[1:], q[2:]):
        for cand in range(hi + two_n, lo, two_n):
            assert not sympy.isprime(cand)
    top = (2 ** cfg.q0_bits - 2) // two_n * two_n + 1
    for cand in range(q[0] + two_n, top + 1, two_n):
        assert not sympy.isprime(cand)


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_root_of_unity(name):
    cfg = CONFIGS[name]
    q, p = C.prime_chain(cfg.log_n, cfg.n_q, cfg.q0_bits, cfg.q_bits, cfg.n_p, cfg.p_bits)
    n = cfg.n
    for m in (q + p)[:6]:
        psi = C.root_2n(m, n)
        assert pow(psi, n, m) == m - 1          # psi^N = -1: order exactly 2N
        g = C.smallest_non_residue(m)
        assert sympy.legendre_symbol(g, m) == -1
        assert all(sympy.legendre_symbol(h, m) == 1 for h in range(2, g))


@pytest.mark.parametrize("n,q", [(8, 97), (16, 12289), (32, 2 ** 40 - 87)])
def test_schoolbook_matches_bigint(n, q):
    g = np.random.default_rng(n)
    a = _rand_res(g, q, n)
    b = _rand_res(g, q, n)
    out = np.empty(n, dtype=np.uint64)
    _ring.lib().or_mul_limb(_ring.ptr(a), _ring.ptr(b), _ring.ptr(out), n, q, 0, 0)
    ref = [x % q for x in negacyclic_int([int(x) for x in a], [int(x) for x in b], n)]
    assert [int(x) for x in out] == ref


@pytest.mark.parametrize("log_n", [3, 4, 5])
def test_ntt_definition_is_evaluation(log_n):
    n = 1 << log_n
    q = C.largest_primes(2 * n, 30, 1)[0]
    psi = C.root_2n(q, n)
    g = np.random.default_rng(log_n)
    a = _rand_res(g, q, n)
    out = np.empty(n, dtype=np.uint64)
    _ring.lib().or_ntt_definition(_ring.ptr(a), _ring.ptr(out), n, q, psi)
    for k in range(n):
        x = pow(psi, 2 * bitrev(k, log_n) + 1, q)
        assert int(out[k]) == evaluate(a, x, q)


@pytest.mark.parametrize("log_n", [4, 8, 10, 12])
def test_ntt_fast_matches_definition(log_n):
    n = 1 << log_n
    q = C.largest_primes(2 * n, 59, 1)[0]
    psi = C.root_2n(q, n)
    g = np.random.default_rng(100 + log_n)
    a = _rand_res(g, q, n)
    d = np.empty(n, dtype=np.uint64)
    f = np.empty(n, dtype=np.uint64)
    back = np.empty(n, dtype=np.uint64)
    L = _ring.lib()
    L.or_ntt_definition(_ring.ptr(a), _ring.ptr(d), n, q, psi)
    L.or_ntt_fast(_ring.ptr(a), _ring.ptr(f), n, q, psi)
    L.or_intt_fast(_ring.ptr(f), _ring.ptr(back), n, q, psi)
    assert np.array_equal(d, f)
    assert np.array_equal(back, a)


@pytest.mark.parametrize("log_n,bits", [(6, 40), (11, 60), (13, 50)])
def test_mul_modes_agree(log_n, bits):
    n = 1 << log_n
    q = C.largest_primes(2 * n, bits, 1)[0]
    psi = C.root_2n(q, n)
    g = np.random.default_rng(log_n)
    a = _rand_res(g, q, n)
    b = _rand_res(g, q, n)
    o0 = np.empty(n, dtype=np.uint64)
    o1 = np.empty(n, dtype=np.uint64)
    L = _ring.lib()
    L.or_mul_limb(_ring.ptr(a), _ring.ptr(b), _ring.ptr(o0), n, q, psi, 0)
    L.or_mul_limb(_ring.ptr(a), _ring.ptr(b), _ring.ptr(o1), n, q, psi, 1)
    assert np.array_equal(o0, o1)


def test_mul_transform_spot_check_2_16():
    """At N = 2^16 the transform product is checked at sampled coefficients
    against the convolution sum computed with Python integers."""
    n = 1 << 16
    q = C.largest_primes(2 * n, 60, 1)[0]
    psi = C.root_2n(q, n)
    g = np.random.default_rng(5)
    a = _rand_res(g, q, n)
    b = _rand_res(g, q, n)
    out = np.empty(n, dtype=np.uint64)
    _ring.lib().or_mul_limb(_ring.ptr(a), _ring.ptr(b), _ring.ptr(out), n, q, psi, 1)
    ai = a.astype(object)
    bi = b.astype(object)
    for k in [0, 1, n - 1, n // 2] + [int(x) for x in g.integers(0, n, 4)]:
        pos = int(np.dot(ai[:k + 1], bi[k::-1]))
        negs = int(np.dot(ai[k + 1:], bi[:k:-1])) if k + 1 < n else 0
        assert int(out[k]) == (pos - negs) % q, k


@pytest.mark.parametrize("log_n", [3, 5])
def test_automorphism_is_substitution(log_n):
    """NTT_def(a(X^kappa))[k] must equal a(x^kappa) at x = psi^(2 brv(k)+1)."""
    n = 1 << log_n
    q = C.largest_primes(2 * n, 40, 1)[0]
    psi = C.root_2n(q, n)
    g = np.random.default_rng(9)
    a = _rand_res(g, q, n)
    for step in (1, 2, 3, n // 2 - 1):
        kappa = C.galois_element(step, n)
        out = C.automorphism(a[None, :], kappa, [q], n)[0]
        for k in range(n):
            x = pow(psi, 2 * bitrev(k, log_n) + 1, q)
            assert evaluate(out, x, q) == evaluate(a, pow(x, kappa, q), q)


def test_automorphism_composes():
    n = 64
    q = C.largest_primes(2 * n, 40, 1)[0]
    g = np.random.default_rng(2)
    a = _rand_res(g, q, n)[None, :]
    k1, k2 = C.galois_element(3, n), C.galois_element(5, n)
    two = C.automorphism(C.automorphism(a, k1, [q], n), k2, [q], n)
    one = C.automorphism(a, k1 * k2 % (2 * n), [q], n)
    assert np.array_equal(two, one)
    assert C.galois_element(n // 2, n) == 1  # 5 has order N/2 mod 2N


def test_base_convert_crt_property():
    """Y = sum_i [x_i (D/s_i)^-1]_{s_i} (D/s_i) satisfies Y = x mod D and
    0 <= (Y - [x]_D)/D < m (checked with sympy CRT); out_t = Y mod t."""
    n = 64
    src = C.largest_primes(128, 40, 3)
    dst = C.largest_primes(128, 50, 2) + C.largest_primes(128, 60, 1)
    g = np.random.default_rng(3)
    x = np.stack([_rand_res(g, s, n) for s in src])
    out = C.base_convert(x, src, dst, n)
    D = math.prod(src)
    for k in range(n):
        X = crt_value(x[:, k], src)
        us = []
        for t, tv in enumerate(dst):
            cands = [u for u in range(len(src)) if (X + u * D) % tv == int(out[t, k])]
            assert cands, (k, t)
            us.append(set(cands))
        assert set.intersection(*us)


@pytest.mark.parametrize("mode", ["round", "floor"])
def test_rescale_matches_bigint_division(mode):
    """Eq. (1) with the rounding offset: c'_k = floor((c + h)/q_last) mod q_k
    for the integer c in [0, Q_l) that the residues represent."""
    P = C.Params(5, 4, 40, 30, 1, 40, 2, 2 ** 20)
    n = P.n
    g = np.random.default_rng(11)
    c0 = np.stack([_rand_res(g, q, n) for q in P.q])
    c1 = np.stack([_rand_res(g, q, n) for q in P.q])
    out = C.rescale(P, C.Ciphertext(c0, c1, 2.0 ** 40), mode=mode)
    ql = P.q[-1]
    h = (ql - 1) // 2 if mode == "round" else 0
    for src, dst in ((c0, out.c0), (c1, out.c1)):
        for k in range(n):
            c = crt_value(src[:, k], P.q)
            v = (c + h) // ql
            for i, q in enumerate(P.q[:-1]):
                assert int(dst[i, k]) == v % q


def test_crt_lift_roundtrip():
    mods = C.largest_primes(64, 50, 5)
    Q = math.prod(mods)
    g = np.random.default_rng(4)
    xs = [int(g.integers(0, 2 ** 62)) * int(g.integers(0, 2 ** 62)) * int(g.integers(1, 2 ** 62)) % Q for _ in range(16)]
    xs += [0, 1, Q - 1, Q // 2, Q // 2 + 1]
    res = np.array([[x % m for x in xs] for m in mods], dtype=np.uint64)
    assert C.crt_lift(res, mods, centered=False) == xs
    cen = C.crt_lift(res, mods, centered=True)
    assert cen == [x if x <= Q // 2 else x - Q for x in xs]
