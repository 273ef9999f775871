"""Seeded draws of key generation and encryption -- TEST INFRASTRUCTURE ONLY
(imported by tests/ and nothing else).

SETUP (Sec. 3.4, the CKKS description) fixes the distributions the scheme
draws from: X_key for the secret (ternary coefficients in this workload),
the uniform distribution over R_q for the masks a and, for encryption, a
ternary v, and the zero-centred discrete Gaussian X_err of standard
deviation sigma = 3.2 (Sec. 6.4, CKKS parameter selection) for the errors.  Seeded
KEYGEN and ENC take their draws from a counter-based generator, so one seed
gives the same draws on every machine and in every order of evaluation.

Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC 2011).  State: a counter of four 64-bit
words and a key of two.  A round multiplies counter words 0 and 2 by the
constants M0 and M1 (full 128-bit products) and forms
  (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0));
ten rounds, the key advanced by the Weyl constants (W0, W1) before each
round after the first.  The output block is the final counter value.

Streams: key = (seed, purpose 2^56 + key_id 2^8 + digit), counter =
(coefficient j, limb i, 0, 0); one block per coefficient (and limb), of
which words w0 (and w1) are used:
  ternary   (w0 mod 3) - 1
  uniform   floor((w1 2^64 + w0) q / 2^128)       (bias below q / 2^128)
  Gaussian  -B + #{k : T_k <= w0}
with the cumulative table T of the discrete Gaussian on -B..B (B = 19, six
standard deviations): rho(x) = exp(-x^2 / (2 sigma^2)),
F(k) = sum_{x <= k} rho(x) / sum_x rho(x) and T_k = floor(2^64 F(k)) for
k = -B .. B-1 (2B thresholds).

Purposes: 1 secret, 2 public-key mask, 3 public-key error, 4 switching-key
masks, 5 switching-key errors, 6 encryption v, 7 encryption e0, 8
encryption e1.  key_id 0 is the relinearisation key; rotation by `step`
uses 1 + (step mod N/2).
"""

from decimal import Decimal, localcontext

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1

SIGMA = Decimal("3.2")
BOUND = 19

SECRET, PK_A, PK_E, KS_A, KS_E, ENC_V, ENC_E0, ENC_E1 = range(1, 9)

_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo(a, b):
    """(hi, lo) 64-bit halves of the 128-bit products a * b (uint64 arrays,
    or an array and a scalar), from 32-bit partial products."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    ll, lh, hl, hh = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (ll & _LO32) | ((mid & _LO32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64-10 blocks of the counters ctr = (c0, c1, c2, c3) (uint64
    arrays of one shape) under key = (k0, k1) (Python ints)."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64).copy() for c in ctr)
    k0, k1 = key[0] & MASK64, key[1] & MASK64
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK64, (k1 + W1) & MASK64
        h0, l0 = mulhilo(c0, np.uint64(M0))
        h1, l1 = mulhilo(c2, np.uint64(M1))
        c0, c1, c2, c3 = h1 ^ c1 ^ np.uint64(k0), l1, h0 ^ c3 ^ np.uint64(k1), l0
    return c0, c1, c2, c3


def stream_key(seed, purpose, key_id=0, digit=0):
    return (int(seed) & MASK64, (purpose << 56) | (int(key_id) << 8) | int(digit))


def blocks(seed, purpose, n, key_id=0, digit=0, limb=0):
    """Words w0, w1 of the blocks of coefficients 0..n-1 of one stream."""
    j = np.arange(n, dtype=np.uint64)
    z = np.zeros(n, dtype=np.uint64)
    w0, w1, _, _ = philox4x64_10((j, z + np.uint64(limb), z, z), stream_key(seed, purpose, key_id, digit))
    return w0, w1


def ternary(w0):
    return (w0 % np.uint64(3)).astype(np.int64) - 1


def uniform(w0, w1, q):
    """floor((w1 2^64 + w0) q / 2^128) for q < 2^64."""
    h1, l1 = mulhilo(w1, np.uint64(q))
    h0, _ = mulhilo(w0, np.uint64(q))
    s = l1 + h0
    return h1 + (s < l1).astype(np.uint64)


def gaussian_cdt(sigma=SIGMA, bound=BOUND):
    """The 2 bound thresholds T_k = floor(2^64 F(k)), k = -bound .. bound-1,
    computed in 60-digit decimal arithmetic (Python ints)."""
    with localcontext() as ctx:
        ctx.prec = 60
        two_var = 2 * Decimal(sigma) * Decimal(sigma)
        rho = [(Decimal(-x * x) / two_var).exp() for x in range(-bound, bound + 1)]
        total = sum(rho)
        out, acc = [], Decimal(0)
        for r in rho[:-1]:
            acc += r
            out.append(int((acc * (1 << 64)) // total))
    return out


def gaussian(w0, table=None):
    t = np.array(gaussian_cdt() if table is None else table, dtype=np.uint64)
    bound = len(t) // 2
    return np.searchsorted(t, w0, side="right").astype(np.int64) - bound


# ---- the draws of KEYGEN and ENC from one seed


def secret(seed, n):
    return ternary(blocks(seed, SECRET, n)[0])


def public_key_draws(seed, q, n):
    """(a [L][n] uniform mod q_i, e [n])."""
    a = np.stack([uniform(*blocks(seed, PK_A, n, limb=i), qi) for i, qi in enumerate(q)])
    return a, gaussian(blocks(seed, PK_E, n)[0])


def switch_key_draws(seed, key_id, moduli, dnum, n):
    """(a [dnum][L+K][n] uniform mod the key moduli, e [dnum][n])."""
    a = np.stack([np.stack([uniform(*blocks(seed, KS_A, n, key_id, d, i), m) for i, m in enumerate(moduli)])
                  for d in range(dnum)])
    e = np.stack([gaussian(blocks(seed, KS_E, n, key_id, d)[0]) for d in range(dnum)])
    return a, e


def rotation_key_id(step, n):
    return 1 + (int(step) % (n // 2))


def encryption_draws(seed, n):
    """(v, e0, e1) of ENC."""
    return (ternary(blocks(seed, ENC_V, n)[0]), gaussian(blocks(seed, ENC_E0, n)[0]),
            gaussian(blocks(seed, ENC_E1, n)[0]))
