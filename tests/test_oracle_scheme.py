"""Pins of the oracle's CKKS layer (Sec. 3.4, hybrid key switching).

Tiny ring (N = 16): exact identities with Python-integer polynomials
(KEYGEN, ENC/DEC, the HMUL tensor, the switching-key gadget, ModUp's CRT
property, the key-switching error bound).
C1 ring (N = 4096): decryption of HMUL+relin, RESCALE, ROTATE and TotalSum
against fp64 slot arithmetic within the noise bounds of tests/noise.py."""

import math

import numpy as np
import pytest

import synth as S
from oracle import ckks as C
from tests import noise
from tests.intpoly import crt_value, negacyclic_int

TINY = dict(log_n=4, n_q=3, q0_bits=30, q_bits=25, n_p=2, p_bits=30, dnum=2, scale=2 ** 10)


def _ints(a):
    return [int(x) for x in a]


def _sub_int(params, s, kappa):
    """s(X^kappa) as an integer polynomial, by substituting X^j -> X^(j kappa)
    and reducing with X^N = -1."""
    n = params.n
    out = [0] * n
    for j, c in enumerate(s):
        e = j * kappa % (2 * n)
        if e < n:
            out[e] += int(c)
        else:
            out[e - n] -= int(c)
    return out


@pytest.fixture(scope="module")
def tiny():
    P = C.Params(**TINY)
    kd = S.key_draws(3, P.n, P.q)
    C.set_mul_mode(0)
    return P, kd


def test_public_key_exact(tiny):
    P, kd = tiny
    b, a = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    for i, q in enumerate(P.q):
        a_s = negacyclic_int(_ints(a[i]), _ints(kd.s), P.n)
        assert [(int(b[i, k]) + a_s[k] - int(kd.pk_e[k])) % q for k in range(P.n)] == [0] * P.n


def test_encrypt_decrypt_exact(tiny):
    """DEC(ENC(m)) = m + e v + e0 + e1 s exactly, as integers modulo each q_i."""
    P, kd = tiny
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    d = S.enc_draws(5, P.n)
    m = S.plaintext_coeffs(S.rng(6), P.n, 2 ** 20)
    for level in (3, 2, 1):
        ct = C.encrypt(P, pk, m, level, d.v, d.e0, d.e1, P.scale)
        dec = C.decrypt(P, kd.s, ct)
        ev = negacyclic_int(_ints(kd.pk_e), _ints(d.v), P.n)
        e1s = negacyclic_int(_ints(d.e1), _ints(kd.s), P.n)
        want = [int(m[k]) + ev[k] + int(d.e0[k]) + e1s[k] for k in range(P.n)]
        for i, q in enumerate(P.q[:level]):
            assert _ints(dec[i]) == [w % q for w in want]


@pytest.mark.parametrize("which", ["relin", "rot1", "rot5"])
def test_switch_key_gadget_exact(tiny, which):
    """b_j + a_j s - e_j = [t in digit j] (P mod q_t) s' on every limb t."""
    P, kd = tiny
    a, e = S.switch_key_draws(3, 1, P.n, P.key_moduli(), P.dnum)
    if which == "relin":
        key = C.relin_key(P, kd.s, a, e)
        s_prime = negacyclic_int(_ints(kd.s), _ints(kd.s), P.n)
    else:
        step = int(which[3:])
        key = C.rotation_key(P, kd.s, step, a, e)
        s_prime = _sub_int(P, kd.s, C.galois_element(step, P.n))
    mods = P.key_moduli()
    for j in range(P.dnum):
        digit = range(j * P.alpha, min((j + 1) * P.alpha, P.L))
        for t, m in enumerate(mods):
            a_s = negacyclic_int(_ints(key.a[j][t]), _ints(kd.s), P.n)
            lhs = [(int(key.b[j][t, k]) + a_s[k] - int(e[j][k])) % m for k in range(P.n)]
            g = (P.P % m) if t in digit else 0
            assert lhs == [g * x % m for x in s_prime], (j, t)


def test_tensor_exact(tiny):
    """(c00 + c01 s)(c10 + c11 s) = d0 + d1 s + d2 s^2 modulo each q_i."""
    P, kd = tiny
    g = np.random.default_rng(8)
    cts = []
    for _ in range(2):
        c0 = np.stack([g.integers(0, q, P.n, dtype=np.uint64) for q in P.q])
        c1 = np.stack([g.integers(0, q, P.n, dtype=np.uint64) for q in P.q])
        cts.append(C.Ciphertext(c0, c1, 1.0))
    d0, d1, d2 = C.tensor(P, cts[0], cts[1])
    s = _ints(kd.s)
    s2 = negacyclic_int(s, s, P.n)
    for i, q in enumerate(P.q):
        x = [a + b for a, b in zip(_ints(cts[0].c0[i]), negacyclic_int(_ints(cts[0].c1[i]), s, P.n))]
        y = [a + b for a, b in zip(_ints(cts[1].c0[i]), negacyclic_int(_ints(cts[1].c1[i]), s, P.n))]
        lhs = negacyclic_int(x, y, P.n)
        rhs = [a + b + c for a, b, c in zip(_ints(d0[i]), negacyclic_int(_ints(d1[i]), s, P.n),
                                          negacyclic_int(_ints(d2[i]), s2, P.n))]
        assert [v % q for v in lhs] == [v % q for v in rhs]


def test_mod_up_crt_property(tiny):
    P, _ = tiny
    g = np.random.default_rng(9)
    level = 3
    d = np.stack([g.integers(0, q, P.n, dtype=np.uint64) for q in P.q[:level]])
    exts = C.mod_up(P, d, level)
    mods = P.q[:level] + P.p
    for digit, ext in zip(P.digits(level), exts):
        src = [P.q[i] for i in digit]
        D = math.prod(src)
        assert np.array_equal(ext[digit], d[digit])
        for k in range(P.n):
            X = crt_value(d[digit, k], src)
            ok = [u for u in range(len(digit)) if all((X + u * D) % m == int(ext[t, k]) for t, m in enumerate(mods))]
            assert ok, k


@pytest.mark.parametrize("level", [3, 2, 1])
def test_key_switch_error_bound(tiny, level):
    """ks0 + ks1 s - d s' is a small integer polynomial: at most
    (K+1)(1+h_s) + sum_j N |digit_j| D_j max|e| / P per coefficient."""
    P, kd = tiny
    a, e = S.switch_key_draws(3, 2, P.n, P.key_moduli(), P.dnum)
    key = C.relin_key(P, kd.s, a, e)
    g = np.random.default_rng(10 + level)
    d = np.stack([g.integers(0, q, P.n, dtype=np.uint64) for q in P.q[:level]])
    k0, k1 = C.key_switch(P, d, key, level)
    s = _ints(kd.s)
    s2 = negacyclic_int(s, s, P.n)
    Q = math.prod(P.q[:level])
    h_s = sum(abs(x) for x in s)
    bound = (P.K + 1) * (1 + h_s)
    for digit in P.digits(level):
        bound += P.n * len(digit) * math.prod(P.q[i] for i in digit) * int(np.max(np.abs(e))) / P.P
    lhs = []
    for i, q in enumerate(P.q[:level]):
        ks = [a_ + b_ for a_, b_ in zip(_ints(k0[i]), negacyclic_int(_ints(k1[i]), s, P.n))]
        dss = negacyclic_int(_ints(d[i]), s2, P.n)
        lhs.append([(x - y) % q for x, y in zip(ks, dss)])
    lhs = np.array(lhs, dtype=np.uint64)
    err = C.crt_lift(lhs, P.q[:level], centered=True)
    assert max(abs(x) for x in err) <= bound
    assert Q > 1000 * bound  # the bound is meaningful at this size


# ---------------------------------------------------------------------------
# C1: N = 4096, the scheme against fp64 slot arithmetic
# ---------------------------------------------------------------------------

def c1_env():
    cfg = S.CONFIGS["C1"]
    P = C.Params.from_config(cfg)
    C.set_mul_mode(1)
    kd = S.key_draws(1, P.n, P.q)
    pk = C.public_key(P, kd.s, kd.pk_a, kd.pk_e)
    a, e = S.switch_key_draws(1, 0, P.n, P.key_moduli(), P.dnum)
    rlk = C.relin_key(P, kd.s, a, e)
    z1 = S.slots_uniform(S.rng(101), P.n // 2)
    z2 = S.slots_uniform(S.rng(102), P.n // 2)
    d1, d2 = S.enc_draws(1001, P.n), S.enc_draws(1002, P.n)
    ct1 = C.encrypt(P, pk, C.encode(z1, P.n, P.scale), P.L, d1.v, d1.e0, d1.e1, P.scale)
    ct2 = C.encrypt(P, pk, C.encode(z2, P.n, P.scale), P.L, d2.v, d2.e0, d2.e1, P.scale)
    h = 2 * P.n / 3
    return dict(P=P, kd=kd, pk=pk, rlk=rlk, z1=z1, z2=z2, ct1=ct1, ct2=ct2,
                fresh=noise.fresh(P.n, h, h, P.scale) + P.n / P.scale)


@pytest.fixture(scope="module")
def c1():
    return c1_env()


def _dec(env, ct):
    P = env["P"]
    return C.decode(C.decrypt(P, env["kd"].s, ct), P.q[:ct.level], P.n, ct.scale, P.n // 2)


def _ks_bound(P, scale):
    h = 2 * P.n / 3
    dmax = max(math.prod(P.q[i] for i in dg) for dg in P.digits(P.L))
    return noise.key_switch(P.n, h, P.dnum, dmax, P.alpha, P.P, P.K, scale)


def test_c1_fresh(c1):
    assert np.max(np.abs(_dec(c1, c1["ct1"]) - c1["z1"])) <= c1["fresh"]


def test_c1_hmul_relin_rescale(c1):
    P = c1["P"]
    prod = C.hmul_relin(P, c1["ct1"], c1["ct2"], c1["rlk"])
    want = c1["z1"] * c1["z2"]
    b_mul = 2 * math.sqrt(2) * c1["fresh"] + c1["fresh"] ** 2 + _ks_bound(P, prod.scale)
    assert np.max(np.abs(_dec(c1, prod) - want)) <= b_mul
    rs = C.rescale(P, prod)
    assert rs.level == 1 and rs.scale == prod.scale / P.q[1]
    b_rs = b_mul + noise.rescale_round(P.n, 2 * P.n / 3, rs.scale)
    assert np.max(np.abs(_dec(c1, rs) - want)) <= b_rs


@pytest.mark.parametrize("step", [1, 3, -1, 1000])
def test_c1_rotate(c1, step):
    P = c1["P"]
    a, e = S.switch_key_draws(1, 100 + step, P.n, P.key_moduli(), P.dnum)
    key = C.rotation_key(P, c1["kd"].s, step, a, e)
    r = C.rotate(P, c1["ct1"], step, key)
    want = np.roll(c1["z1"], -step)
    assert np.max(np.abs(_dec(c1, r) - want)) <= c1["fresh"] + _ks_bound(P, r.scale)


def test_c1_rotate_pow2(c1):
    """Power-of-two decomposition: slots equal the direct rotation by the full
    step (within one key-switch error per set bit), and a single-bit step is
    exactly the direct rotation."""
    P = c1["P"]
    keys = {}
    for k in range(4):
        a, e = S.switch_key_draws(1, 200 + k, P.n, P.key_moduli(), P.dnum)
        keys[1 << k] = C.rotation_key(P, c1["kd"].s, 1 << k, a, e)
    for step, hw in ((11, 3), (13 - P.n // 2, 3)):   # 11 = 8 + 2 + 1; a negative step reduces mod N/2
        r = C.rotate_pow2(P, c1["ct1"], step, keys)
        want = np.roll(c1["z1"], -step)
        assert np.max(np.abs(_dec(c1, r) - want)) <= c1["fresh"] + hw * _ks_bound(P, r.scale)
    one = C.rotate_pow2(P, c1["ct1"], 4, keys)
    direct = C.rotate(P, c1["ct1"], 4, keys[4])
    assert np.array_equal(one.c0, direct.c0) and np.array_equal(one.c1, direct.c1)


def test_c1_total_sum(c1):
    P = c1["P"]
    t = P.n // 2
    keys = {}
    for i in range(int(math.log2(t))):
        a, e = S.switch_key_draws(1, 200 + i, P.n, P.key_moduli(), P.dnum)
        keys[1 << i] = C.rotation_key(P, c1["kd"].s, 1 << i, a, e)
    out = C.total_sum(P, c1["ct1"], t, keys)
    k = int(math.log2(t))
    bound = 2 ** k * (c1["fresh"] + k * _ks_bound(P, out.scale))
    assert np.max(np.abs(_dec(c1, out) - c1["z1"].sum())) <= bound


def test_c1_plain_ops(c1):
    P = c1["P"]
    w = S.slots_uniform(S.rng(7), P.n // 2)
    pt = C.encode(w, P.n, P.scale)
    s = C.hadd_plain(P, c1["ct1"], pt)
    assert np.max(np.abs(_dec(c1, s) - (c1["z1"] + w))) <= c1["fresh"] + P.n / P.scale
    m = C.hmul_plain(P, c1["ct1"], pt, P.scale)
    b = 2 * math.sqrt(2) * (c1["fresh"] + P.n / P.scale)
    assert np.max(np.abs(_dec(c1, m) - c1["z1"] * w)) <= b
    add = C.hadd(P, c1["ct1"], c1["ct2"])
    assert np.max(np.abs(_dec(c1, add) - (c1["z1"] + c1["z2"]))) <= 2 * c1["fresh"]
    with pytest.raises(ValueError):
        C.hadd(P, c1["ct1"], C.mod_drop(P, c1["ct2"], 1))
