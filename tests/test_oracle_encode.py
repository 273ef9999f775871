"""Pins of the oracle's ENCODE/DECODE (Sec. 3.4) by closed forms: constant
slots encode to a constant polynomial, the slot vector zeta^(5^j) encodes to
scale*X, and decode inverts encode up to rounding."""

import numpy as np
import pytest

from oracle import ckks as C


@pytest.mark.parametrize("log_n", [4, 10, 12])
def test_constant_slots_encode_to_constant(log_n):
    n = 1 << log_n
    scale = 2.0 ** 30
    for c in (0.75, -0.3125, 1.0):
        m = C.encode(np.full(n // 2, c), n, scale)
        assert m[0] == round(c * scale)
        assert not np.any(m[1:])


@pytest.mark.parametrize("log_n", [4, 10, 12])
def test_root_slots_encode_to_x(log_n):
    n = 1 << log_n
    scale = 2.0 ** 30
    e = C.slot_exponents(n, n // 2)
    z = np.exp(1j * np.pi * e / n)  # zeta^(5^j)
    m = C.encode(z, n, scale)
    want = np.zeros(n, dtype=np.int64)
    want[1] = int(scale)
    assert np.array_equal(m, want)


def test_decode_of_x_is_roots():
    n = 64
    scale = 2.0 ** 20
    mu = np.zeros(n)
    mu[1] = scale
    z = C.decode_ints(mu, n, scale, n // 2)
    e = C.slot_exponents(n, n // 2)
    assert np.allclose(z, np.exp(1j * np.pi * e / n), atol=1e-12)


def test_slot_exponents_cover_half_the_odd_residues():
    n = 256
    e = C.slot_exponents(n, n // 2)
    allodd = set(range(1, 2 * n, 2))
    s = set(int(x) for x in e)
    assert len(s) == n // 2
    assert s | {2 * n - x for x in s} == allodd  # with conjugates: all primitive roots


def test_encode_matches_direct_sum():
    n = 128
    g = np.random.default_rng(1)
    z = g.uniform(-1, 1, 40) + 1j * g.uniform(-1, 1, 40)
    assert np.array_equal(C.encode(z, n, 2.0 ** 35), C.encode_definition(z, n, 2.0 ** 35))


@pytest.mark.parametrize("log_n", [6, 12])
def test_decode_inverts_encode(log_n):
    n = 1 << log_n
    scale = 2.0 ** 40
    g = np.random.default_rng(log_n)
    z = g.uniform(-1, 1, n // 2) + 1j * g.uniform(-1, 1, n // 2)
    back = C.decode_ints(C.encode(z, n, scale), n, scale, n // 2)
    # rounding error per coefficient <= 1/2, so per slot <= N/(2 scale)
    assert np.max(np.abs(back - z)) <= n / (2 * scale)


def test_sparse_slots_zero_padded():
    n = 64
    scale = 2.0 ** 30
    z = np.array([0.5 + 0.25j, -0.125])
    back = C.decode_ints(C.encode(z, n, scale), n, scale, n // 2)
    assert np.allclose(back[:2], z, atol=1e-7)
    assert np.allclose(back[2:], 0, atol=1e-7)
