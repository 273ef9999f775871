"""CPU oracle of the CKKS hot path of PrivFT (arXiv:1908.06972).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the HIP product never
does, and the two share no code.  Randomness is not drawn here: every random
polynomial is an argument (see the `synth` package), so the oracle is a pure
function of its inputs.

Representation: an RNS polynomial is a uint64 numpy array [limbs, N] in
coefficient form, limb i reduced modulo the i-th modulus of the list it is
used with.  Ring products go through ring_oracle.c (schoolbook, or that file's
own textbook transform for large N); additions, negations and the CRT are
written here with numpy and Python integers.

Parity status of each function:
  pinned   primes/psi (sympy, Euler's criterion), ring product (big-integer
           brute force), transform (definition), automorphism (big-integer
           substitution), base conversion (big-integer CRT), rescale (big-integer
           floor/round, Eq. (1)), encode/decode (closed forms, round trip), key
           switching and the full scheme (decryption within the noise bound),
           rotation (slot roll), TotalSum (slot sum).
Nothing here is "parity unpinned".

Readings of the paper that this file implements (each is listed again in
the design notes):
  * ENC draws v from the ternary distribution and forms
    (b*v + e0 + mu, a*v + e1) so that DEC = c0 + c1*s (Sec. 3.4; the printed
    ENC swaps a and b and names u but uses v).
  * RESCALE rounds: it adds h = (q_last - 1)/2 before the exact division of
    Eq. (1) (Sec. 3.4 defines a rounding; Alg. 3 as printed floors, which is
    mode "floor").
  * Slot j sits at zeta^(5^j mod 2N), zeta = exp(i pi / N); ROTATE by r > 0 is
    X -> X^(5^r mod 2N) and moves slot j+r to slot j (left rotation).
  * TotalSum adds rotations by 2^i for i = 0 .. log2(t) - 1 (Alg. 2 prints
    i = 1 .. log2 N).
  * Key switching, which the paper only cites, is the hybrid method with dnum
    digits of alpha = ceil(L/dnum) consecutive ciphertext primes and K special
    primes P = p_0...p_{K-1}, using the fast (approximate) base conversion.
"""

import math

import numpy as np

from . import _ring

# --------------------------------------------------------------------------
# Parameters (SETUP, Sec. 3.4; prime order from Sec. 5.1)
# --------------------------------------------------------------------------

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin, exact for n < 3.3e24 with these bases."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def largest_primes(two_n: int, bits: int, count: int, exclude=()) -> list:
    """The `count` largest primes p < 2^bits with p = 1 mod 2N, descending,
    skipping `exclude`.  Each must have exactly `bits` bits."""
    out = []
    k = (2 ** bits - 2) // two_n
    while len(out) < count:
        p = k * two_n + 1
        if p < 2 ** (bits - 1):
            raise ValueError("not enough %d-bit primes = 1 mod %d" % (bits, two_n))
        if p not in exclude and is_prime(p):
            out.append(p)
        k -= 1
    return out


def prime_chain(log_n: int, n_q: int, q0_bits: int, q_bits: int, n_p: int, p_bits: int):
    """q_0 = largest q0_bits-bit prime; q_1..q_{L-1} = the next L-1 largest
    q_bits-bit primes (strictly descending, so the last prime is the smallest,
    Sec. 5.1); the K special primes are the largest unused p_bits-bit primes."""
    two_n = 2 << log_n
    q0 = largest_primes(two_n, q0_bits, 1)
    rest = largest_primes(two_n, q_bits, n_q - 1, exclude=set(q0))
    q = q0 + rest
    p = largest_primes(two_n, p_bits, n_p, exclude=set(q))
    return q, p


def smallest_non_residue(q: int) -> int:
    g = 2
    while pow(g, (q - 1) // 2, q) != q - 1:
        g += 1
    return g


def root_2n(q: int, n: int) -> int:
    """psi = g^((q-1)/2N) for the smallest quadratic non-residue g; psi^N = -1,
    so psi is a primitive 2N-th root of unity mod q."""
    return pow(smallest_non_residue(q), (q - 1) // (2 * n), q)


class Params:
    def __init__(self, log_n, n_q, q0_bits, q_bits, n_p, p_bits, dnum, scale):
        self.log_n = log_n
        self.n = 1 << log_n
        self.q, self.p = prime_chain(log_n, n_q, q0_bits, q_bits, n_p, p_bits)
        self.L = n_q
        self.K = n_p
        self.dnum = dnum
        self.alpha = -(-n_q // dnum)
        self.scale = float(scale)
        self.psi = {m: root_2n(m, self.n) for m in self.q + self.p}
        self.P = math.prod(self.p)

    @classmethod
    def from_config(cls, cfg):
        return cls(cfg.log_n, cfg.n_q, cfg.q0_bits, cfg.q_bits, cfg.n_p, cfg.p_bits, cfg.dnum, cfg.scale)

    def key_moduli(self):
        return self.q + self.p

    def key_rows(self, level):
        """Rows of a switching key used at `level`: q-limbs 0..level-1, then the
        K special limbs (stored after all L q-limbs)."""
        return list(range(level)) + [self.L + k for k in range(self.K)]

    def digits(self, level):
        """Digit j = q-limbs [j*alpha, min((j+1)*alpha, level))."""
        a = self.alpha
        return [list(range(j * a, min((j + 1) * a, level))) for j in range(-(-level // a))]


# --------------------------------------------------------------------------
# RNS polynomial helpers
# --------------------------------------------------------------------------

def _col(mods):
    return np.array([int(m) for m in mods], dtype=np.uint64)[:, None]


def rns_from_int(x: np.ndarray, mods) -> np.ndarray:
    """Signed integer polynomial (int64 [N]) reduced modulo every modulus."""
    x = np.asarray(x, dtype=np.int64)
    return np.stack([np.mod(x, np.int64(m)).astype(np.uint64) for m in mods])


def add(a, b, mods):
    return (a + b) % _col(mods)


def sub(a, b, mods):
    q = _col(mods)
    return (a + q - b) % q


def neg(a, mods):
    q = _col(mods)
    return (q - a) % q


def ring_mul(params, a, b, mods):
    """Limb-wise product in Z_q[X]/(X^N+1)."""
    a = _ring.u64(a)
    b = _ring.u64(b)
    out = np.empty_like(a)
    m = _ring.u64([int(x) for x in mods])
    psi = _ring.u64([params.psi[int(x)] for x in mods])
    _ring.lib().or_poly_mul(_ring.ptr(a), _ring.ptr(b), _ring.ptr(out), params.n,
                            _ring.ptr(m), _ring.ptr(psi), len(mods))
    return out


def scalar_mul(a, consts, mods):
    """Limb i times the integer consts[i], modulo mods[i]."""
    a = _ring.u64(a)
    out = np.empty_like(a)
    L = _ring.lib()
    for i, (c, m) in enumerate(zip(consts, mods)):
        L.or_scalar_mul(_ring.ptr(a[i]), int(c) % int(m), _ring.ptr(out[i]), a.shape[1], int(m))
    return out


def automorphism(a, kappa, mods, n):
    """a(X) -> a(X^kappa) limb by limb."""
    a = _ring.u64(a)
    out = np.empty_like(a)
    for i, m in enumerate(mods):
        _ring.lib().or_automorphism(_ring.ptr(a[i]), _ring.ptr(out[i]), n, int(m), int(kappa))
    return out


def base_convert(x, src, dst, n):
    """Fast base conversion of x [len(src), N] to the primes dst."""
    x = _ring.u64(x)
    out = np.empty((len(dst), n), dtype=np.uint64)
    s = _ring.u64([int(m) for m in src])
    d = _ring.u64([int(m) for m in dst])
    _ring.lib().or_base_convert(_ring.ptr(x), _ring.ptr(s), len(src), _ring.ptr(d), len(dst),
                                _ring.ptr(out), n)
    return out


def crt_lift(res, mods, centered=True):
    """Exact CRT reconstruction of every coefficient as a Python integer,
    optionally centred into (-Q/2, Q/2]."""
    Q = math.prod(int(m) for m in mods)
    terms = []
    for i, m in enumerate(mods):
        m = int(m)
        hat = Q // m
        terms.append((hat, pow(hat % m, -1, m), m))
    n = res.shape[1]
    out = []
    for k in range(n):
        x = 0
        for i, (hat, inv, m) in enumerate(terms):
            x += (int(res[i, k]) * inv % m) * hat
        x %= Q
        if centered and x > Q // 2:
            x -= Q
        out.append(x)
    return out


def set_mul_mode(mode: int):
    """0 = schoolbook (definition), 1 = the oracle's own transform."""
    _ring.lib().or_set_mul_mode(mode)


def get_mul_mode() -> int:
    return _ring.lib().or_get_mul_mode()


# --------------------------------------------------------------------------
# ENCODE / DECODE (Sec. 3.4; done on the client CPU per Sec. 5.1)
# --------------------------------------------------------------------------

def slot_exponents(n: int, n_slots: int) -> np.ndarray:
    """5^j mod 2N for j < n_slots: slot j is the evaluation at zeta^(5^j)."""
    e = np.empty(n_slots, dtype=np.int64)
    x = 1
    for j in range(n_slots):
        e[j] = x
        x = x * 5 % (2 * n)
    return e


def _round_half_away(x: np.ndarray) -> np.ndarray:
    return np.sign(x) * np.floor(np.abs(x) + 0.5)


def encode(z, n: int, scale: float) -> np.ndarray:
    """mu_k = round((2 scale / N) Re sum_j z_j zeta^(-(5^j) k)), k < N.

    This inverts the canonical embedding restricted to the slots zeta^(5^j)
    and their conjugates (the paper's round(IDFT(2^rho v))).  The sum is taken
    as one length-2N FFT of the vector holding z_j at index 5^j mod 2N."""
    z = np.asarray(z, dtype=np.complex128)
    if len(z) > n // 2:
        raise ValueError("at most N/2 slots")
    Z = np.zeros(2 * n, dtype=np.complex128)
    Z[slot_exponents(n, len(z))] = z
    s = np.fft.fft(Z)[:n]  # sum_r Z[r] exp(-2 pi i r k / 2N) = sum_j z_j zeta^(-5^j k)
    m = _round_half_away((2.0 * scale / n) * s.real)
    if np.any(np.abs(m) >= 2.0 ** 62):
        raise OverflowError("encoded coefficient exceeds 2^62")
    return m.astype(np.int64)


def encode_definition(z, n: int, scale: float) -> np.ndarray:
    """O(N * slots) direct evaluation of the same sum (used to pin `encode`)."""
    z = np.asarray(z, dtype=np.complex128)
    e = slot_exponents(n, len(z))
    k = np.arange(n)
    m = np.zeros(n)
    for j in range(len(z)):
        m += (z[j] * np.exp(-1j * np.pi * ((e[j] * k) % (2 * n)) / n)).real
    return _round_half_away((2.0 * scale / n) * m).astype(np.int64)


def decode_ints(mu, n: int, scale: float, n_slots: int) -> np.ndarray:
    """z_j = (1/scale) sum_k mu_k zeta^((5^j) k) for an integer polynomial mu."""
    mu = np.asarray(mu, dtype=np.float64)
    M = np.zeros(2 * n, dtype=np.float64)
    M[:n] = mu
    s = np.fft.ifft(M) * (2 * n)  # sum_k mu_k exp(+2 pi i r k / 2N)
    return s[slot_exponents(n, n_slots)] / scale


def decode(res, mods, n: int, scale: float, n_slots: int) -> np.ndarray:
    """DECODE of RNS residues: centred CRT lift, then the slot evaluation."""
    mu = [float(x) for x in crt_lift(res, mods, centered=True)]
    return decode_ints(mu, n, scale, n_slots)


# --------------------------------------------------------------------------
# Ciphertexts and KEYGEN / ENC / DEC (Sec. 3.4)
# --------------------------------------------------------------------------

class Ciphertext:
    def __init__(self, c0, c1, scale):
        self.c0 = c0
        self.c1 = c1
        self.scale = float(scale)

    @property
    def level(self):
        return self.c0.shape[0]

    def copy(self):
        return Ciphertext(self.c0.copy(), self.c1.copy(), self.scale)


class SwitchKey:
    """Per digit j: (b_j, a_j), each [L+K, N] coefficient form, with
    b_j + a_j s = e_j + [limb t in digit j] (P mod q_t) s' on every limb t."""

    def __init__(self, b, a):
        self.b = b
        self.a = a


class Keys:
    def __init__(self):
        self.s = None
        self.pk = None
        self.rlk = None
        self.rot = {}


def public_key(params, s, a, e):
    """b = -a s + e over the L ciphertext primes (KEYGEN, Sec. 3.4)."""
    mods = params.q
    s_r = rns_from_int(s, mods)
    b = add(neg(ring_mul(params, a, s_r, mods), mods), rns_from_int(e, mods), mods)
    return (b, _ring.u64(a))


def switch_key(params, s, s_prime, a, e):
    """Switching key from s' (RNS over all L+K moduli) to s, hybrid form with
    dnum digits: the gadget of digit j is P on its q-limbs and 0 elsewhere."""
    mods = params.key_moduli()
    s_r = rns_from_int(s, mods)
    bs, as_ = [], []
    for j in range(params.dnum):
        aj = _ring.u64(a[j])
        bj = add(neg(ring_mul(params, aj, s_r, mods), mods), rns_from_int(e[j], mods), mods)
        for t in range(j * params.alpha, min((j + 1) * params.alpha, params.L)):
            q = params.q[t]
            term = scalar_mul(s_prime[t:t + 1], [params.P % q], [q])
            bj[t] = add(bj[t:t + 1], term, [q])[0]
        bs.append(bj)
        as_.append(aj)
    return SwitchKey(bs, as_)


def relin_key(params, s, a, e):
    mods = params.key_moduli()
    s_r = rns_from_int(s, mods)
    return switch_key(params, s, ring_mul(params, s_r, s_r, mods), a, e)


def galois_element(step: int, n: int) -> int:
    """kappa = 5^(step mod N/2) mod 2N (left rotation by `step` slots)."""
    return pow(5, step % (n // 2), 2 * n)


def rotation_key(params, s, step, a, e):
    mods = params.key_moduli()
    kappa = galois_element(step, params.n)
    s_rot = automorphism(rns_from_int(s, mods), kappa, mods, params.n)
    return switch_key(params, s, s_rot, a, e)


def encrypt(params, pk, m, level, v, e0, e1, scale):
    """ENC of the integer plaintext m at `level` limbs:
    (b v + e0 + m, a v + e1) (Sec. 3.4, as read)."""
    mods = params.q[:level]
    b, a = pk[0][:level], pk[1][:level]
    v_r = rns_from_int(v, mods)
    c0 = add(add(ring_mul(params, b, v_r, mods), rns_from_int(e0, mods), mods), rns_from_int(m, mods), mods)
    c1 = add(ring_mul(params, a, v_r, mods), rns_from_int(e1, mods), mods)
    return Ciphertext(c0, c1, scale)


def decrypt(params, s, ct):
    """DEC: c0 + c1 s modulo q_l (Sec. 3.4)."""
    mods = params.q[:ct.level]
    return add(ct.c0, ring_mul(params, ct.c1, rns_from_int(s, mods), mods), mods)


# --------------------------------------------------------------------------
# Homomorphic operations (Sec. 3.4) and key switching
# --------------------------------------------------------------------------

def hadd(params, x, y):
    if x.level != y.level:
        raise ValueError("level mismatch")
    mods = params.q[:x.level]
    return Ciphertext(add(x.c0, y.c0, mods), add(x.c1, y.c1, mods), x.scale)


def hadd_plain(params, x, m):
    mods = params.q[:x.level]
    return Ciphertext(add(x.c0, rns_from_int(m, mods), mods), x.c1.copy(), x.scale)


def hmul_plain(params, x, m, m_scale):
    """(c0 pt, c1 pt) for the integer plaintext polynomial m."""
    mods = params.q[:x.level]
    pt = rns_from_int(m, mods)
    return Ciphertext(ring_mul(params, x.c0, pt, mods), ring_mul(params, x.c1, pt, mods), x.scale * m_scale)


def tensor(params, x, y):
    """HMUL before relinearisation: (c00 c10, c00 c11 + c01 c10, c01 c11)."""
    if x.level != y.level:
        raise ValueError("level mismatch")
    mods = params.q[:x.level]
    d0 = ring_mul(params, x.c0, y.c0, mods)
    d1 = add(ring_mul(params, x.c0, y.c1, mods), ring_mul(params, x.c1, y.c0, mods), mods)
    d2 = ring_mul(params, x.c1, y.c1, mods)
    return d0, d1, d2


def mod_up(params, d, level):
    """Digit decomposition + fast base conversion of d [level, N]: returns one
    [level+K, N] polynomial per digit, equal to d on the digit's own limbs."""
    qs = params.q[:level]
    ext_all = []
    for digit in params.digits(level):
        others = [i for i in range(level) if i not in digit]
        dst = [qs[i] for i in others] + params.p
        conv = base_convert(d[digit], [qs[i] for i in digit], dst, params.n)
        ext = np.empty((level + params.K, params.n), dtype=np.uint64)
        ext[digit] = d[digit]
        ext[others] = conv[:len(others)]
        ext[level:] = conv[len(others):]
        ext_all.append(ext)
    return ext_all


def mod_down(params, acc, level):
    """(acc_i - Conv_{P -> q_i}(acc_P)) * P^-1 mod q_i for i < level."""
    qs = params.q[:level]
    conv = base_convert(acc[level:], params.p, qs, params.n)
    diff = sub(acc[:level], conv, qs)
    return scalar_mul(diff, [pow(params.P % q, -1, q) for q in qs], qs)


def key_switch(params, d, key, level):
    """Hybrid key switching of d [level, N] (coefficient form) with `key`:
    returns (ks0, ks1) with ks0 + ks1 s ~ d s'."""
    rows = params.key_rows(level)
    mods = params.q[:level] + params.p
    acc0 = np.zeros((level + params.K, params.n), dtype=np.uint64)
    acc1 = np.zeros_like(acc0)
    for j, ext in enumerate(mod_up(params, d, level)):
        acc0 = add(acc0, ring_mul(params, ext, key.b[j][rows], mods), mods)
        acc1 = add(acc1, ring_mul(params, ext, key.a[j][rows], mods), mods)
    return mod_down(params, acc0, level), mod_down(params, acc1, level)


def hmul_relin(params, x, y, rlk):
    """HMUL followed by relinearisation (Table 2's HMUL+REL; no rescale)."""
    d0, d1, d2 = tensor(params, x, y)
    k0, k1 = key_switch(params, d2, rlk, x.level)
    mods = params.q[:x.level]
    return Ciphertext(add(d0, k0, mods), add(d1, k1, mods), x.scale * y.scale)


def rescale(params, x, mode="round"):
    """RESCALE by the last prime q_last of the level (Eq. (1), Alg. 3):
    c'_k = (c_k + h - r) q_last^-1 mod q_k with r = (c_last + h) mod q_last,
    h = (q_last - 1)/2 (round) or 0 (floor)."""
    lvl = x.level
    if lvl < 2:
        raise ValueError("cannot rescale at level 1")
    ql = params.q[lvl - 1]
    h = (ql - 1) // 2 if mode == "round" else 0
    if mode not in ("round", "floor"):
        raise ValueError(mode)
    out = []
    for c in (x.c0, x.c1):
        r = (c[lvl - 1] + np.uint64(h)) % np.uint64(ql)
        limbs = []
        for k in range(lvl - 1):
            qk = np.uint64(params.q[k])
            # c_k + h - r, every term reduced below q_k first (sums stay < 2^62)
            t = (c[k] + np.uint64(h) % qk + qk - r % qk) % qk
            limbs.append(t)
        diff = np.stack(limbs)
        qs = params.q[:lvl - 1]
        out.append(scalar_mul(diff, [pow(ql, -1, qk) for qk in qs], qs))
    return Ciphertext(out[0], out[1], x.scale / ql)


def mod_drop(params, x, level):
    return Ciphertext(x.c0[:level].copy(), x.c1[:level].copy(), x.scale)


def rotate(params, x, step, key):
    """ROTATE by `step` slots to the left: X -> X^kappa on both polynomials,
    then key switching of c1 from s(X^kappa) back to s."""
    kappa = galois_element(step, params.n)
    mods = params.q[:x.level]
    c0 = automorphism(x.c0, kappa, mods, params.n)
    c1 = automorphism(x.c1, kappa, mods, params.n)
    k0, k1 = key_switch(params, c1, key, x.level)
    return Ciphertext(add(c0, k0, mods), k1, x.scale)


def rotate_pow2(params, x, step, rot_keys):
    """ROTATE by `step` from power-of-two keys, the cost model of the paper's
    ROTATE (Sec. 6.5: one automorphism and key switch per set bit of the step):
    with r = step mod N/2, rotate by 2^k for every set bit k of r in ascending
    order, each with rot_keys[2^k]."""
    half = params.n // 2
    r = step % half
    k = 0
    while (1 << k) < half:
        if (r >> k) & 1:
            x = rotate(params, x, 1 << k, rot_keys[1 << k])
        k += 1
    return x


def total_sum(params, x, n_slots, rot_keys):
    """Alg. 2 (TotalSum): ct <- ct + ROTATE(ct, 2^i) for i = 0..log2(t)-1."""
    for i in range(int(math.log2(n_slots))):
        x = hadd(params, x, rotate(params, x, 1 << i, rot_keys[1 << i]))
    return x
