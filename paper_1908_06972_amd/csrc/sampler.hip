// sampler.hip -- seeded draws of KEYGEN and ENC on the device.
//
// SETUP (Sec. 3.4, the CKKS description) draws the secret from X_key (ternary
// coefficients here), masks uniformly from R_q and errors from the
// zero-centred discrete Gaussian X_err, sigma = 3.2 (Sec. 6.4, CKKS parameter
// selection).  The seeded entry points take every draw from a counter-based
// generator so that a seed fixes the keys and ciphertexts on any device and
// in any launch order.
//
// Generator: Philox4x64-10 (Salmon, Moraes, Dror and Shaw, SC 2011).  Four
// 64-bit counter words, two key words; each of ten rounds replaces the
// counter (c0, c1, c2, c3) by
//   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
// with the key advanced by the Weyl increments (W0, W1) before every round
// but the first.
//
// Streams: key (seed, purpose 2^56 + key_id 2^8 + digit), counter
// (coefficient j, limb i, 0, 0); words w0, w1 of the block give
//   ternary    (w0 mod 3) - 1
//   uniform    floor((w1 2^64 + w0) q / 2^128)
//   Gaussian   -B + #{k : T_k <= w0}
// with T the 2B thresholds floor(2^64 F(k)) of the discrete Gaussian's
// cumulative distribution on -B..B (B = 19, six standard deviations),
// computed on the host in 120-bit fixed point.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pft_kernels.h"

namespace {

constexpr uint64_t PH_M0 = 0xD2E7470EE14C6C93ull, PH_M1 = 0xCA5A826395121157ull;
constexpr uint64_t PH_W0 = 0x9E3779B97F4A7C15ull, PH_W1 = 0xBB67AE8584CAA73Bull;
constexpr uint32_t SAMPLE_TB = 256;

__device__ __forceinline__ void philox_block(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        const uint64_t h0 = __umul64hi(PH_M0, c[0]), l0 = PH_M0 * c[0];
        const uint64_t h1 = __umul64hi(PH_M1, c[2]), l1 = PH_M1 * c[2];
        const uint64_t n0 = h1 ^ c[1] ^ k0, n2 = h0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = l1;
        c[2] = n2;
        c[3] = l0;
    }
}

// out[i][j] = uniform residue mod q_i from block (j, i) of the stream (k0, k1)
__global__ void k_sample_uniform(uint64_t k0, uint64_t k1, SampleModuli mods, uint64_t* __restrict__ out,
                                 uint32_t n) {
    const uint32_t j = blockIdx.x * SAMPLE_TB + threadIdx.x;
    const uint32_t i = blockIdx.y;
    if (j >= n) return;
    uint64_t c[4] = {j, i, 0, 0};
    philox_block(c, k0, k1);
    const uint64_t q = mods.q[i];
    const uint64_t h1 = __umul64hi(c[1], q), l1 = c[1] * q, h0 = __umul64hi(c[0], q);
    const uint64_t s = l1 + h0;
    out[(size_t)i * n + j] = h1 + (s < l1 ? 1u : 0u);
}

// out[j] = ternary (kind 0) or discrete-Gaussian (kind 1) coefficient j
__global__ void k_sample_small(uint32_t kind, uint64_t k0, uint64_t k1, GaussianCdt cdt, int64_t* __restrict__ out,
                               uint32_t n) {
    const uint32_t j = blockIdx.x * SAMPLE_TB + threadIdx.x;
    if (j >= n) return;
    uint64_t c[4] = {j, 0, 0, 0};
    philox_block(c, k0, k1);
    const uint64_t w = c[0];
    int64_t x;
    if (kind == 0) {
        x = (int64_t)(w % 3u) - 1;
    } else {
        int64_t cnt = 0;
        for (uint32_t k = 0; k < cdt.count; ++k) cnt += cdt.t[k] <= w ? 1 : 0;
        x = cnt - (int64_t)(cdt.count / 2);
    }
    out[j] = x;
}

// ---- the cumulative table in unsigned 128-bit fixed point, 120 fraction bits

typedef unsigned __int128 u128;
constexpr int FB = 120;

// floor(a b / 2^120) for a, b < 2^123
u128 fx_mul(u128 a, u128 b) {
    const uint64_t a0 = (uint64_t)a, a1 = (uint64_t)(a >> 64), b0 = (uint64_t)b, b1 = (uint64_t)(b >> 64);
    const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
    const u128 mid = p01 + p10 + (p00 >> 64);  // < 2^124
    return (p11 << (128 - FB)) + (mid >> (FB - 64));
}

u128 fx_pow(u128 base, uint32_t e) {
    u128 r = (u128)1 << FB;
    while (e) {
        if (e & 1u) r = fx_mul(r, base);
        base = fx_mul(base, base);
        e >>= 1;
    }
    return r;
}

// floor(2^64 num / den) for num < den < 2^126
uint64_t fx_ratio64(u128 num, u128 den) {
    uint64_t qt = 0;
    u128 rem = num;
    for (int b = 0; b < 64; ++b) {
        rem <<= 1;
        qt <<= 1;
        if (rem >= den) {
            rem -= den;
            qt |= 1u;
        }
    }
    return qt;
}

}  // namespace

// sigma^2 = 10.24 = 256 / 25: rho(x) = exp(-x^2 / (2 sigma^2)) = r^(x^2) with
// r = exp(-25/512), summed from its Taylor series (alternating terms kept as
// two non-negative sums).
int gaussian_cdt_host(uint64_t* t, uint32_t capacity) {
    const uint32_t B = PFT_GAUSS_BOUND;
    if (capacity < 2 * B) return -1;
    u128 pos = 0, neg = 0, term = (u128)1 << FB;
    for (uint32_t k = 0; k < 40; ++k) {
        if (k & 1u)
            neg += term;
        else
            pos += term;
        term = term * 25u / (512u * (k + 1u));
    }
    const u128 r = pos - neg;
    u128 rho[2 * PFT_GAUSS_BOUND + 1];
    u128 total = 0;
    for (uint32_t i = 0; i <= 2 * B; ++i) {
        const int32_t x = (int32_t)i - (int32_t)B;
        rho[i] = fx_pow(r, (uint32_t)(x * x));
        total += rho[i];
    }
    u128 acc = 0;
    for (uint32_t i = 0; i < 2 * B; ++i) {
        acc += rho[i];
        t[i] = fx_ratio64(acc, total);
    }
    return (int)(2 * B);
}

void launch_sample_uniform(uint64_t k0, uint64_t k1, const SampleModuli& mods, uint32_t rows, uint64_t* out,
                           uint32_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_sample_uniform, dim3((n + SAMPLE_TB - 1) / SAMPLE_TB, rows), dim3(SAMPLE_TB), 0, st, k0, k1,
                       mods, out, n);
}

void launch_sample_small(uint32_t kind, uint64_t k0, uint64_t k1, const GaussianCdt& cdt, int64_t* out, uint32_t n,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_sample_small, dim3((n + SAMPLE_TB - 1) / SAMPLE_TB), dim3(SAMPLE_TB), 0, st, kind, k0, k1,
                       cdt, out, n);
}
