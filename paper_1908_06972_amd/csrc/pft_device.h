// pft_device.h -- device-side data structures and 64-bit modular arithmetic
// for gfx950.  Residues are uint64 below primes q < 2^60.
//
// Three reductions are used, chosen per operand kind:
//   * Shoup (constant multiplier w with w' = floor(w 2^64 / q)): twiddles and
//     per-prime constants; result in [0, 2q) before the optional final
//     subtraction.
//   * Montgomery REDC (R = 2^64) for sums of products whose constant factor
//     was stored pre-multiplied by R: base-conversion matrices, switching keys.
//   * Barrett (mu = floor(2^(2b)/q), b = bit length of q) for products of two
//     variable residues (the HMUL tensor, NTT-domain plaintext products).
// All three are built from 64x64 products that the compiler lowers to
// v_mul_lo_u32 / v_mul_hi_u32 / v_mad_u64_u32, which issue at full rate on
// gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PFT_MAX_POLYS 128  // polynomials per NTT launch
#define PFT_MAX_ITEMS 64   // ciphertexts per batched launch
#define PFT_SMALL_POLYS 8  // operands of the small elementwise kernels

struct DevMod {
    uint64_t q;
    uint64_t two_q;
    uint64_t mu;          // floor(2^(2b) / q)
    uint64_t mont_neg_qinv;  // -q^-1 mod 2^64
    uint64_t n_inv, n_inv_sh;      // N^-1 mod q and its Shoup companion
    uint64_t last_inv, last_inv_sh; // psi^-brv(1) * N^-1: fused last inverse stage
    uint32_t bits;
    uint32_t fp;          // 1 if q < 2^50: the NTT runs its butterflies in fp64
    // fp64 forms for the NTT when fp != 0: q, 1/q, and each constant c with
    // its quotient c/q, all rounded to nearest (c < q < 2^50 is exact).
    double qd, qinv;
    double n_inv_d, n_inv_q;
    double last_inv_d, last_inv_q;
};

// One twiddle.  Integer limbs: w and its Shoup companion floor(w 2^64 / q).
// fp64 limbs (DevMod::fp): the bit patterns of the doubles w and w/q.
struct TwPair {
    uint64_t w;
    uint64_t wp;
};

// A set of RNS polynomials processed by one NTT launch.  Limb i (0 <= i <
// n_limbs) of polynomial p sits at row r = i + (i >= gap_at[p] ? gap_len[p] : 0)
// of ptr[p] (rows are N words apart); row r is reduced modulo modulus index
// r < split ? off0 + r : off1 + (r - split).  The first pass of a transform
// reads each row from src_delta words past it (0: in place) and writes it in
// place.
struct PolyBatch {
    uint64_t* ptr[PFT_MAX_POLYS];
    uint8_t gap_at[PFT_MAX_POLYS];
    uint8_t gap_len[PFT_MAX_POLYS];
    uint32_t n_polys;
    uint32_t n_limbs;
    uint32_t split, off0, off1;
    int64_t src_delta;
};

__device__ __forceinline__ uint32_t pb_row(const PolyBatch& b, uint32_t p, uint32_t i) {
    return i + (i >= b.gap_at[p] ? (uint32_t)b.gap_len[p] : 0u);
}
__device__ __forceinline__ uint32_t pb_mod(const PolyBatch& b, uint32_t row) {
    return row < b.split ? b.off0 + row : b.off1 + (row - b.split);
}

// Up to eight polynomials of n_limbs consecutive rows starting at row
// `first`, same modulus rule as PolyBatch (small elementwise launches).
struct SmallBatch {
    uint64_t* ptr[PFT_SMALL_POLYS];
    uint32_t n_polys;
    uint32_t n_limbs;
    uint32_t first;
    uint32_t split, off0, off1;
};
__device__ __forceinline__ uint32_t sb_mod(const SmallBatch& b, uint32_t row) {
    return row < b.split ? b.off0 + row : b.off1 + (row - b.split);
}

// Per-ciphertext device pointers of a batched launch.
struct ItemPtrs {
    uint64_t* p[PFT_MAX_ITEMS];
};

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// a*w mod q in [0, 2q) for any a < 2^64 (Shoup).
__device__ __forceinline__ uint64_t shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    return a * w - mulhi64(a, wp) * q;
}
__device__ __forceinline__ uint64_t shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t r = shoup_lazy(a, w, wp, q);
    return r >= q ? r - q : r;
}

// ---- fp64 arithmetic for primes q < 2^50 (the NTT butterflies, base-conversion folds)
//
// A residue is held as an integer-valued double of either sign; every value
// stays an integer below 2^53 in magnitude, so sums and differences are exact.
// fmulmod(a, w) returns a w - k q with k = rint(fl(a fl(w/q))): the product
// a w is split exactly into hi + lo (hi = fl(a w), lo = fma(a, w, -hi)); then
// fma(-k, q, hi) is exact because the true value is an integer of magnitude
// below 2^53, and adding lo is exact for the same reason.  The quotient is off
// from a w / q by at most 1/2 + |a| 2^-52 (two roundings), so with |a| <= c q
// and q < 2^50 the result lies within (1/2 + c/4) q of zero.  freduce(x) =
// x - rint(x/q) q lies within q/2 (+ a vanishing error) for the magnitudes
// used here.  Forward butterfly with X reduced: inputs within B q give outputs
// within (1 + B/4) q; inverse with X + Y reduced: within max(1/2, 1/2 + B/2) q.
// The lazy schedules of the NTT keep every magnitude below 4.5q < 2^53.
__device__ __forceinline__ double as_f(uint64_t v) { return __builtin_bit_cast(double, v); }
__device__ __forceinline__ uint64_t as_u(double v) { return __builtin_bit_cast(uint64_t, v); }

__device__ __forceinline__ double fmulmod(double a, double w, double wq, double q) {
#pragma clang fp contract(off)
    const double hi = a * w;
    const double lo = __builtin_fma(a, w, -hi);
    const double k = __builtin_rint(a * wq);
    return __builtin_fma(-k, q, hi) + lo;
}
__device__ __forceinline__ double freduce(double x, double q, double qinv) {
#pragma clang fp contract(off)
    return __builtin_fma(-__builtin_rint(x * qinv), q, x);
}

// u64 below 2^52 -> double: the bits of 2^52 + v, minus 2^52.
__device__ __forceinline__ uint64_t fp_from_u64(uint64_t v) {
#pragma clang fp contract(off)
    return as_u(as_f(v | 0x4330000000000000ull) - 4503599627370496.0);
}
// double residue -> canonical u64 in [0, q): reduce to within q/2, lift the
// negative half by q, then read the mantissa of 2^52 + r.
__device__ __forceinline__ uint64_t fp_to_u64(uint64_t v, double q, double qinv) {
#pragma clang fp contract(off)
    double r = freduce(as_f(v), q, qinv);
    r = r < 0.0 ? r + q : r;
    return as_u(r + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull;
}

// (hi:lo) * 2^-64 mod q for hi:lo < q * 2^64; result in [0, q).
__device__ __forceinline__ uint64_t mont_redc(uint64_t lo, uint64_t hi, uint64_t q, uint64_t neg_qinv) {
    uint64_t m = lo * neg_qinv;
    uint64_t r = hi + mulhi64(m, q) + (lo != 0 ? 1u : 0u);
    return r >= q ? r - q : r;
}

// 128-bit accumulator helpers
struct Acc128 {
    uint64_t lo, hi;
};
__device__ __forceinline__ void mac128(Acc128& acc, uint64_t a, uint64_t b) {
    uint64_t lo = a * b;
    uint64_t hi = mulhi64(a, b);
    acc.lo += lo;
    acc.hi += hi + (acc.lo < lo ? 1u : 0u);
}

// a*b mod q for a, b < q (Barrett, HAC 14.42 with base 2).
__device__ __forceinline__ uint64_t mul_barrett(uint64_t a, uint64_t b, const DevMod& m) {
    uint64_t lo = a * b, hi = mulhi64(a, b);
    uint32_t bits = m.bits;
    uint64_t x1 = (lo >> (bits - 1)) | (hi << (65 - bits));
    uint64_t plo = x1 * m.mu, phi = mulhi64(x1, m.mu);
    uint64_t qh = (plo >> (bits + 1)) | (phi << (63 - bits));
    uint64_t r = lo - qh * m.q;
    if (r >= m.q) r -= m.q;
    if (r >= m.q) r -= m.q;
    return r;
}

__device__ __forceinline__ uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
    uint64_t r = a + b;
    return r >= q ? r - q : r;
}
__device__ __forceinline__ uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) {
    return a >= b ? a - b : a + q - b;
}

// index of the bit-reversal of k over log_n bits
__device__ __forceinline__ uint32_t brev_n(uint32_t k, uint32_t log_n) {
    return __brev(k) >> (32 - log_n);
}
