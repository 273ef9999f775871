"""Pins of the oracle's seeded sampler (oracle/sampler.py).

The generator is checked against numpy's own Philox4x64-10 bit generator
(an independent implementation of the same published definition), the
128-bit products against Python integers, the uniform map against its
big-integer definition and its bucket counts, and the discrete-Gaussian
table against what the distribution fixes: exact symmetry, mean 0 and a
variance equal to sigma^2 up to the exponentially small Poisson-summation
term and the six-sigma truncation."""

import math
from decimal import Decimal

import numpy as np
import pytest

from oracle import sampler as SP

KEYS = [0, 7 | (5 << 64), (2 ** 64 - 1) | ((2 ** 63 + 12345) << 64), 0x0123456789ABCDEF | (0xFEDCBA9876543210 << 64)]
CTRS = [[0, 0, 0, 0], [41, 3, 0, 0], [2 ** 40, 9, 17, 23], [2 ** 63, 2 ** 64 - 1, 1, 2 ** 62]]


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("ctr", CTRS)
def test_philox_matches_numpy(key, ctr):
    # numpy advances its 256-bit counter (with carries) before producing a
    # block: the block of counter c is the first output after seeding c - 1
    c = sum(w << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    bg = np.random.Philox(key=key, counter=np.array([(c >> (64 * i)) & SP.MASK64 for i in range(4)], dtype=np.uint64))
    ref = bg.random_raw(4)
    c = [np.array([x], dtype=np.uint64) for x in ctr]
    got = np.array([w[0] for w in SP.philox4x64_10(c, (key & SP.MASK64, key >> 64))], dtype=np.uint64)
    assert np.array_equal(ref, got)


def test_philox_vectorised_equals_scalar():
    key = (0x1234, 0x5678)
    j = np.arange(1000, dtype=np.uint64) * np.uint64(7919)
    z = np.full(1000, 3, dtype=np.uint64)
    vec = SP.philox4x64_10((j, z, z, z), key)
    for i in (0, 1, 517, 999):
        one = SP.philox4x64_10(([j[i]], [3], [3], [3]), key)
        assert all(v[i] == o[0] for v, o in zip(vec, one))


def test_mulhilo_against_python_ints():
    g = np.random.default_rng(5)
    a = np.concatenate([g.integers(0, 2 ** 64, 2000, dtype=np.uint64, endpoint=False),
                        np.array([0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 64 - 1], dtype=np.uint64)])
    b = np.concatenate([g.integers(0, 2 ** 64, 2000, dtype=np.uint64, endpoint=False),
                        np.array([2 ** 64 - 1, 2 ** 64 - 1, 2 ** 32 + 1, 2 ** 64 - 1, 2 ** 64 - 1], dtype=np.uint64)])
    hi, lo = SP.mulhilo(a, b)
    for x, y, h, l in zip(a.tolist(), b.tolist(), hi.tolist(), lo.tolist()):
        assert (h << 64) | l == x * y


def test_uniform_is_its_definition_and_in_range():
    w0, w1 = SP.blocks(9, SP.PK_A, 3000)
    for q in [3, 97, (1 << 50) - 27, (1 << 60) - 93, (1 << 64) - 59]:
        u = SP.uniform(w0, w1, q)
        ref = [((int(b) << 64 | int(a)) * q) >> 128 for a, b in zip(w0.tolist(), w1.tolist())]
        assert u.tolist() == ref
        assert int(u.max()) < q


def test_uniform_buckets_are_flat():
    n = 1 << 16
    w0, w1 = SP.blocks(10, SP.KS_A, n, key_id=3, digit=1, limb=2)
    for q in (7, 97):
        counts = np.bincount(SP.uniform(w0, w1, q).astype(np.int64), minlength=q)
        exp = n / q
        assert np.all(np.abs(counts - exp) < 5 * math.sqrt(exp))


def _table_moments(table):
    t = [0] + list(table) + [1 << 64]
    b = len(table) // 2
    p = [Decimal(t[i + 1] - t[i]) / Decimal(1 << 64) for i in range(len(t) - 1)]
    xs = range(-b, b + 1)
    mean = sum(x * pi for x, pi in zip(xs, p))
    var = sum(x * x * pi for x, pi in zip(xs, p)) - mean * mean
    return float(mean), float(var), p


def test_cdt_shape_and_symmetry():
    t = SP.gaussian_cdt()
    assert len(t) == 2 * SP.BOUND
    assert all(0 <= a < b < (1 << 64) for a, b in zip(t, t[1:]))
    # F(k) + F(-k-1) = 1 and 2^64 F(k) is never an integer
    assert all(t[i] + t[len(t) - 1 - i] == (1 << 64) - 1 for i in range(len(t)))


@pytest.mark.parametrize("sigma,bound", [("3.2", 19), ("1.0", 8), ("2.5", 15)])
def test_cdt_variance_is_sigma_squared(sigma, bound):
    """The discrete Gaussian on Z has variance sigma^2 minus a term of order
    sigma^4 exp(-2 pi^2 sigma^2) (Poisson summation); truncation at six
    standard deviations removes less than 1e-5 more."""
    mean, var, p = _table_moments(SP.gaussian_cdt(Decimal(sigma), bound))
    s2 = float(sigma) ** 2
    assert abs(mean) < 1e-15
    assert abs(var - s2) < 1e-5 * max(1.0, s2)
    # the mode is 0 and the probabilities fall off as exp(-x^2 / 2 sigma^2)
    b = bound
    ratio = float(p[b + 1] / p[b])
    assert abs(ratio - math.exp(-1.0 / (2 * s2))) < 1e-12


def test_gaussian_and_ternary_draws():
    n = 1 << 17
    g = SP.gaussian(SP.blocks(11, SP.ENC_E0, n)[0])
    assert abs(g.mean()) < 5 * 3.2 / math.sqrt(n)
    assert abs(g.var() - 10.24) < 0.02 * 10.24
    assert np.abs(g).max() <= SP.BOUND
    s = SP.secret(12, n)
    counts = np.bincount(s + 1, minlength=3)
    assert set(np.unique(s).tolist()) == {-1, 0, 1}
    assert np.all(np.abs(counts - n / 3) < 5 * math.sqrt(n / 3))


def test_streams_are_separate():
    n = 64
    base = SP.blocks(1, SP.KS_A, n, key_id=0, digit=0, limb=0)[0]
    for kw in [dict(purpose=SP.KS_E), dict(key_id=1), dict(digit=1), dict(limb=1), dict(seed=2)]:
        args = dict(seed=1, purpose=SP.KS_A, key_id=0, digit=0, limb=0)
        args.update(kw)
        other = SP.blocks(args["seed"], args["purpose"], n, args["key_id"], args["digit"], args["limb"])[0]
        assert not np.array_equal(base, other)


def test_key_draw_shapes():
    q = [(1 << 40) - 87, (1 << 40) - 167]
    a, e = SP.public_key_draws(3, q, 256)
    assert a.shape == (2, 256) and e.shape == (256,)
    assert all(int(a[i].max()) < q[i] for i in range(2))
    a, e = SP.switch_key_draws(3, SP.rotation_key_id(5, 256), q + [(1 << 50) - 111], 2, 256)
    assert a.shape == (2, 3, 256) and e.shape == (2, 256)
    assert SP.rotation_key_id(-1, 256) == 128 and SP.rotation_key_id(0, 256) == 1
    v, e0, e1 = SP.encryption_draws(3, 256)
    assert v.shape == e0.shape == e1.shape == (256,)
