// bconv_device.h -- device helpers of the exact base conversion on the
// matrix cores (ModUp / ModDown of hybrid key switching), shared by the
// conversion kernels and the ModUp kernel fused with the first transform pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pft_device.h"
#include "pft_kernels.h"

namespace {

// ---- base conversion on the matrix cores -------------------------------
// The contraction y_t = sum_i x_i h_{i,t} mod m_t in signed base-256 digits
// (operand tables and the exactness bound are built on the host):
// Z_{t,b} = sum_{i,a} x_{i,a} v_{(i,a),t,b} by v_mfma_i32_32x32x16_i8 with the
// constant digits as A (32 rows = 4 targets x 8 digits b) and the input
// digits as B (32 columns = 32 coefficients, k = 8 i_local + a), then
// y_t = sum_b 256^b Z_{t,b} mod m_t on the VALU.
typedef int v16i __attribute__((ext_vector_type(16)));

// balanced base-256 digits of v < 2^60 as packed int8: v + 0x80..80 carries
// exactly as the balanced digits do, and each biased byte minus 128 is the
// digit (the same bits as the byte XOR 0x80)
__device__ __forceinline__ long split_digits(uint64_t v) {
    return (long)((v + 0x8080808080808080ull) ^ 0x8080808080808080ull);
}

// sum_b 256^b Z_b mod m for the 8 digit sums of one target (|Z_b| < 2^21).
// lo = sum_{b<4} 256^b Z_b and hi = sum_{b>=4} 256^(b-4) Z_b are integers
// below 2^46 in magnitude, exact in fp64; the value is lo + 2^32 hi.
//  m < 2^50: lo + fmulmod(hi, 2^32 mod m) and one fp64 reduction (the error
//    analysis of fmulmod / freduce applies with |hi| < 2^46).
//  m >= 2^50: the quotient k = round((lo + 2^32 hi) / m) has |k| < 2^29 and
//    comes from fp64 (error below 2^-21); the remainder is formed exactly in
//    integers mod 2^64 as (lo + 2^32 hi + 2^30 m) - (k + 2^30) m, which lies
//    within (1/2 + 2^-21) m of zero, then one conditional add of m.
// RAW: for m < 2^50 return the bits of the reduced double itself (an
// integer of magnitude at most m/2 + 1), the input form of the fp64
// transform passes, instead of the canonical u64.
template <bool RAW = false>
__device__ __forceinline__ uint64_t fold_digits(const int (&z)[8], const BconvRed& rc) {
#pragma clang fp contract(off)
    const double lo = __builtin_fma((double)(z[3] * 256 + z[2]), 65536.0, (double)(z[1] * 256 + z[0]));
    const double hi = __builtin_fma((double)(z[7] * 256 + z[6]), 65536.0, (double)(z[5] * 256 + z[4]));
    if (rc.fp) {
        double y = freduce(lo + fmulmod(hi, rc.c32, rc.c32q, rc.md), rc.md, rc.minv);
        if (RAW) return as_u(y);
        y = y < 0.0 ? y + rc.md : y;  // [0, m)
        return as_u(y + 0x1p52) ^ 0x4330000000000000ull;
    }
    const double s = __builtin_fma(hi, 0x1p32, lo);
    const uint32_t k = (uint32_t)__builtin_fma(s, rc.minv, 0x1p30 + 0.5);  // floor: k + 2^30
    // two's complement of an integer |v| < 2^51 in the low bits of v + 1.5 2^52
    const uint64_t lo64 = as_u(lo + 0x1.8p52) - 0x4338000000000000ull;
    const uint32_t hi32 = (uint32_t)as_u(hi + 0x1.8p52);
    const uint64_t r = lo64 + ((uint64_t)hi32 << 32) + rc.cq0 + (uint64_t)k * rc.negm;
    return (int64_t)r < 0 ? r + rc.m : r;
}

// the two targets of this lane in accumulator tile acc: u = 0, 1
template <int U>
__device__ __forceinline__ void tile_digits(const v16i& acc, int (&z)[8]) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        z[b] = acc[4 * U + b];
        z[4 + b] = acc[8 + 4 * U + b];
    }
}

// the fold constants of every modulus (at most 64) into LDS, so that the
// per-target reads in the fold are short-latency
__device__ __forceinline__ void stage_red(const KsConsts& kc, BconvRed* s_red) {
    const uint32_t words = (kc.L + kc.K) * (uint32_t)(sizeof(BconvRed) / 8);
    const uint64_t* src = reinterpret_cast<const uint64_t*>(kc.red);
    uint64_t* dst = reinterpret_cast<uint64_t*>(s_red);
    for (uint32_t w = threadIdx.x; w < words; w += blockDim.x) dst[w] = src[w];
    __syncthreads();
}

}  // namespace
