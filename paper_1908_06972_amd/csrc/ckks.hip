// ckks.hip -- limb-parallel kernels of the CKKS homomorphic operations
// (Sec. 3.4 HADD/HMUL/HMULPLAIN/ROTATE, Sec. 5.1 RESCALE) and of hybrid key
// switching (ModUp base conversion, key inner product, ModDown).
//
// Every kernel maps one thread to one coefficient index k of one limb row;
// consecutive lanes touch consecutive k, so every global access is a
// coalesced row segment of the limb-major [poly][limb][N] layout.  Batched
// kernels take the ciphertext index from blockIdx.z; per-ciphertext
// intermediates live in a workspace at base + z * stride (WsRef).
#include <type_traits>

#include "bconv_device.h"
#include "pft_device.h"
#include "pft_kernels.h"

#define PFT_MAX_ALPHA 12
#define PFT_MAX_K 12

namespace {

constexpr uint32_t TB = 256;

__device__ __forceinline__ uint64_t* ws_item(const WsRef& w) { return w.base + (size_t)blockIdx.z * w.stride; }
__device__ __forceinline__ size_t at(uint32_t row, uint32_t log_n, uint32_t k) { return ((size_t)row << log_n) + k; }

// ---- small elementwise kernels (key generation, encryption, HADD, ...) ----
__global__ __launch_bounds__(TB) void k_int_to_rns(const int64_t* __restrict__ x, SmallBatch out,
                                                   const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = out.first + limb;
    const uint64_t q = mods[sb_mod(out, row)].q;
    const int64_t v = x[((size_t)poly << log_n) + k];
    uint64_t r;
    if (v >= 0) {
        r = (uint64_t)v % q;
    } else {
        const uint64_t mag = (0ull - (uint64_t)v) % q;
        r = mag == 0 ? 0 : q - mag;
    }
    out.ptr[poly][at(row, log_n, k)] = r;
}

__global__ __launch_bounds__(TB) void k_ew(uint32_t op, SmallBatch out, SmallBatch a, SmallBatch b, SmallBatch c,
                                           const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = out.first + limb;
    const DevMod md = mods[sb_mod(out, row)];
    const uint64_t x = a.ptr[poly][at(a.first + limb, log_n, k)];
    uint64_t r = 0;
    switch (op) {
        case EW_ADD: r = add_mod(x, b.ptr[poly][at(b.first + limb, log_n, k)], md.q); break;
        case EW_SUB: r = sub_mod(x, b.ptr[poly][at(b.first + limb, log_n, k)], md.q); break;
        case EW_MUL: r = mul_barrett(x, b.ptr[poly][at(b.first + limb, log_n, k)], md); break;
        case EW_MULADD:
            r = add_mod(mul_barrett(x, b.ptr[poly][at(b.first + limb, log_n, k)], md),
                        c.ptr[poly][at(c.first + limb, log_n, k)], md.q);
            break;
        case EW_NEG_MULADD:
            r = sub_mod(c.ptr[poly][at(c.first + limb, log_n, k)],
                        mul_barrett(x, b.ptr[poly][at(b.first + limb, log_n, k)], md), md.q);
            break;
        default: r = x; break;
    }
    out.ptr[poly][at(row, log_n, k)] = r;
}

__global__ __launch_bounds__(TB) void k_mul_const(SmallBatch out, SmallBatch a, const TwPair* __restrict__ consts,
                                                  const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = out.first + limb;
    const uint64_t q = mods[sb_mod(out, row)].q;
    const TwPair w = consts[limb];
    const uint64_t x = a.ptr[poly][at(a.first + limb, log_n, k)];
    out.ptr[poly][at(row, log_n, k)] = shoup(x, w.w, w.wp, q);
}

// Switching-key storage form in place: rows whose modulus is below 2^50 hold
// the residue as an integer-valued double, the others residue * 2^64 mod m.
__global__ __launch_bounds__(TB) void k_key_form(SmallBatch out, const TwPair* __restrict__ to_mont,
                                                 const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = out.first + limb;
    const uint32_t mi = sb_mod(out, row);
    const DevMod md = mods[mi];
    uint64_t* p = out.ptr[poly] + at(row, log_n, k);
    const uint64_t x = *p;
    *p = md.fp ? fp_from_u64(x) : shoup(x, to_mont[mi].w, to_mont[mi].wp, md.q);
}

// ---- batched kernels of the homomorphic operations ------------------------

// HMUL tensor of ciphertexts a_z, b_z ([2][level][N] each): d0 = a0 b0,
// d1 = a0 b1 + a1 b0, d2 = a1 b1, written as [3][level][N] at ws_z + off_d.
__global__ __launch_bounds__(TB) void k_tensor_b(ItemPtrs a, ItemPtrs b, WsRef ws, uint64_t off_d, uint32_t level,
                                                 const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t i = blockIdx.y;
    const DevMod md = mods[i];
    const uint64_t* __restrict__ A = a.p[blockIdx.z];
    const uint64_t* __restrict__ B = b.p[blockIdx.z];
    uint64_t* __restrict__ d = ws_item(ws) + off_d;
    const size_t o0 = at(i, log_n, k), o1 = at(level + i, log_n, k);
    const uint64_t a0 = A[o0], a1 = A[o1], b0 = B[o0], b1 = B[o1];
    d[o0] = mul_barrett(a0, b0, md);
    d[o1] = add_mod(mul_barrett(a0, b1, md), mul_barrett(a1, b0, md), md.q);
    d[at(2 * level + i, log_n, k)] = mul_barrett(a1, b1, md);
}

// rows [0, gridDim.y) of src_z + src_off -> dst_z + dst_off
__global__ __launch_bounds__(TB) void k_copy_rows_b(ItemPtrs src, uint64_t src_off, ItemPtrs dst, uint64_t dst_off,
                                                    uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const size_t o = at(blockIdx.y, log_n, k);
    (dst.p[blockIdx.z] + dst_off)[o] = (src.p[blockIdx.z] + src_off)[o];
}

// NTT-domain X -> X^kappa on the `rows` rows of in_z, written to ws_z + off.
// Entry k holds the evaluation at psi^e with e = 2 brv(k) + 1; a(X^kappa)
// there equals a at psi^(e kappa mod 2N), stored at brv((e kappa mod 2N - 1)/2).
__global__ __launch_bounds__(TB) void k_automorphism_b(ItemPtrs in, WsRef ws, uint64_t off_out, uint64_t kappa,
                                                       uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const size_t base = (size_t)blockIdx.y << log_n;
    const uint64_t e = 2ull * brev_n(k, log_n) + 1;
    const uint64_t e2 = (e * kappa) & ((2ull << log_n) - 1);
    const uint32_t src = brev_n((uint32_t)((e2 - 1) >> 1), log_n);
    (ws_item(ws) + off_out)[base + k] = in.p[blockIdx.z][base + src];
}

// ModUp for digit j = blockIdx.y of item z at `level`: from d (coefficient
// form, [level][N] at off_d):
//   xt_i = d_i (D_j/q_i)^-1 mod q_i,  ext_j[t] = sum_i xt_i ((D_j/q_i) mod m_t)
// for every row t outside the digit (q-limbs then special primes); ext_j is
// [level+K][N] at off_ext + j (level+K) N.
__global__ __launch_bounds__(TB) void k_modup_b(WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level,
                                                KsConsts kc, const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t j = blockIdx.y;
    const uint32_t i0 = j * kc.alpha;
    const uint32_t i1 = min(i0 + kc.alpha, level);
    const uint32_t na = i1 - i0;
    const uint32_t rows = level + kc.K;
    const size_t cbase = ((size_t)(level - 1) * kc.dnum + j) * kc.alpha;
    const uint64_t* __restrict__ d = ws_item(ws) + off_d;
    uint64_t xt[PFT_MAX_ALPHA];
#pragma unroll
    for (uint32_t ii = 0; ii < PFT_MAX_ALPHA; ++ii) {
        if (ii < na) {
            const TwPair h = kc.modup_hatinv[cbase + ii];
            xt[ii] = shoup(d[at(i0 + ii, log_n, k)], h.w, h.wp, mods[i0 + ii].q);
        }
    }
    uint64_t* __restrict__ outj = ws_item(ws) + off_ext + ((size_t)j * rows << log_n);
    for (uint32_t t = 0; t < rows; ++t) {
        if (t >= i0 && t < i1) continue;
        const uint32_t mi = t < level ? t : kc.L + (t - level);
        const DevMod md = mods[mi];
        Acc128 acc = {0, 0};
#pragma unroll
        for (uint32_t ii = 0; ii < PFT_MAX_ALPHA; ++ii)
            if (ii < na) mac128(acc, xt[ii], kc.modup_c[(cbase + ii) * (kc.L + kc.K) + t]);
        outj[at(t, log_n, k)] = mont_redc(acc.lo, acc.hi, md.q, md.mont_neg_qinv);
    }
}

// ModUp on the matrix cores: same inputs and outputs as k_modup_b.  A wave
// converts 32 coefficients of digit j = blockIdx.y to every target row.  NKB
// = ceil(alpha' / 2) k-blocks of 16 for alpha' = min(alpha, level); a digit
// with fewer limbs has zero input digits in the unused k positions.
template <uint32_t NKB>
__global__ __launch_bounds__(TB) void k_modup_mfma_b(WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level,
                                                     KsConsts kc, const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t lane = threadIdx.x & 63u, half = lane >> 5;
    const uint32_t n = (blockIdx.x * (TB / 64) + (threadIdx.x >> 6)) * 32 + (lane & 31u);
    const uint32_t j = blockIdx.y;
    const uint32_t i0 = j * kc.alpha;
    const uint32_t na = min(i0 + kc.alpha, level) - i0;
    const uint32_t rows = level + kc.K, T = rows - na;
    const size_t cbase = ((size_t)(level - 1) * kc.dnum + j) * kc.alpha;
    const uint64_t* __restrict__ d = ws_item(ws) + off_d;
    long bop[NKB];
#pragma unroll
    for (uint32_t kb = 0; kb < NKB; ++kb) {
        const uint32_t ii = 2 * kb + half;
        uint64_t x = 0;
        if (ii < na) {
            const TwPair h = kc.modup_hatinv[cbase + ii];
            x = shoup(d[at(i0 + ii, log_n, n)], h.w, h.wp, mods[i0 + ii].q);
        }
        bop[kb] = split_digits(x);
    }
    const uint64_t* __restrict__ aop =
        kc.up_aop + ((size_t)(level - 1) * kc.dnum + j) * kc.up_rt * kc.up_kb * 64 + lane;
    uint64_t* __restrict__ outj = ws_item(ws) + off_ext + ((size_t)j * rows << log_n);
    __shared__ BconvRed s_red[64];
    stage_red(kc, s_red);
    // the constant digits of tile rt + 1 load while tile rt is folded
    long av[NKB];
#pragma unroll
    for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[kb * 64];
    for (uint32_t rt = 0; rt * 4 < T; ++rt) {
        const v16i zero = {};
        v16i acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[0], bop[0], zero, 0, 0, 0);
#pragma unroll
        for (uint32_t kb = 1; kb < NKB; ++kb) acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[kb], bop[kb], acc, 0, 0, 0);
        if ((rt + 1) * 4 < T) {
#pragma unroll
            for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[((rt + 1) * kc.up_kb + kb) * 64];
        }
        int z[8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 0) tile_digits<0>(acc, z); else tile_digits<1>(acc, z);
            const uint32_t tt = 4 * rt + 2 * half + u;
            if (tt < T) {
                const uint32_t t = tt < i0 ? tt : tt + na;
                const uint32_t mi = t < level ? t : kc.L + (t - level);
                outj[at(t, log_n, n)] = fold_digits(z, s_red[mi]);
            }
        }
    }
}

// ModDown conversion on the matrix cores: same inputs and outputs as
// k_moddown_conv_b (poly b = blockIdx.y); NKB = ceil(K / 2).
template <uint32_t NKB>
__global__ __launch_bounds__(TB) void k_moddown_mfma_b(WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                                                       KsConsts kc, const DevMod* __restrict__ mods,
                                                       uint32_t log_n) {
    const uint32_t lane = threadIdx.x & 63u, half = lane >> 5;
    const uint32_t n = (blockIdx.x * (TB / 64) + (threadIdx.x >> 6)) * 32 + (lane & 31u);
    const uint32_t b = blockIdx.y;
    const uint32_t rows = level + kc.K;
    const uint64_t* __restrict__ acc_in = ws_item(ws) + off_acc;
    long bop[NKB];
#pragma unroll
    for (uint32_t kb = 0; kb < NKB; ++kb) {
        const uint32_t k = 2 * kb + half;
        uint64_t x = 0;
        if (k < kc.K) {
            const TwPair h = kc.down_phatinv[k];
            x = shoup(acc_in[at(b * rows + level + k, log_n, n)], h.w, h.wp, mods[kc.L + k].q);
        }
        bop[kb] = split_digits(x);
    }
    const uint64_t* __restrict__ aop = kc.down_aop + lane;
    uint64_t* __restrict__ conv = ws_item(ws) + off_conv;
    __shared__ BconvRed s_red[64];
    stage_red(kc, s_red);
    long av[NKB];
#pragma unroll
    for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[kb * 64];
    for (uint32_t rt = 0; rt * 4 < level; ++rt) {
        const v16i zero = {};
        v16i acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[0], bop[0], zero, 0, 0, 0);
#pragma unroll
        for (uint32_t kb = 1; kb < NKB; ++kb) acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[kb], bop[kb], acc, 0, 0, 0);
        if ((rt + 1) * 4 < level) {
#pragma unroll
            for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[((rt + 1) * kc.down_kb + kb) * 64];
        }
        int z[8];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u == 0) tile_digits<0>(acc, z); else tile_digits<1>(acc, z);
            const uint32_t i = 4 * rt + 2 * half + u;
            if (i < level) conv[at(b * level + i, log_n, n)] = fold_digits(z, s_red[i]);
        }
    }
}

// acc_b[t] = sum_j x_j[t] key_{j,b}[row(t)], x_j = d (NTT domain, at off_d)
// on digit j's own rows and ext_j elsewhere; keys hold key * 2^64 mod m
// (Montgomery), so one REDC per output gives the plain residue.
__global__ __launch_bounds__(TB) void k_key_inner_b(WsRef ws, uint64_t off_d, uint64_t off_ext, uint64_t off_acc,
                                                    const uint64_t* __restrict__ key, uint32_t level, KsConsts kc,
                                                    const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t t = blockIdx.y;
    const uint32_t rows = level + kc.K;
    const uint32_t krow = t < level ? t : kc.L + (t - level);
    const DevMod md = mods[krow];
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    const uint32_t krows = kc.L + kc.K;
    const uint64_t* __restrict__ w = ws_item(ws);
    uint64_t* __restrict__ acc = ws_item(ws) + off_acc;
    if (md.fp) {
        // keys are integer-valued doubles; each term lies within 3q/4 and the
        // sums are brought back within q/2 every four terms (exact below 2^53)
        double s0 = 0.0, s1 = 0.0;
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t i0 = j * kc.alpha, i1 = min(i0 + kc.alpha, level);
            const uint64_t x = (t >= i0 && t < i1) ? w[off_d + at(t, log_n, k)]
                                                    : w[off_ext + at(j * rows + t, log_n, k)];
            const double xd = as_f(fp_from_u64(x));
            const double k0 = as_f(key[at((2 * j) * krows + krow, log_n, k)]);
            const double k1 = as_f(key[at((2 * j + 1) * krows + krow, log_n, k)]);
            s0 += fmulmod(xd, k0, k0 / md.qd, md.qd);
            s1 += fmulmod(xd, k1, k1 / md.qd, md.qd);
            if ((j & 3u) == 3u) {
                s0 = freduce(s0, md.qd, md.qinv);
                s1 = freduce(s1, md.qd, md.qinv);
            }
        }
        acc[at(t, log_n, k)] = fp_to_u64(as_u(s0), md.qd, md.qinv);
        acc[at(rows + t, log_n, k)] = fp_to_u64(as_u(s1), md.qd, md.qinv);
        return;
    }
    // 128-bit sums of at most 8 products stay below q 2^64 (8 q < 2^63)
    Acc128 a0 = {0, 0}, a1 = {0, 0};
    uint64_t r0 = 0, r1 = 0;
    for (uint32_t j = 0; j < beta; ++j) {
        const uint32_t i0 = j * kc.alpha, i1 = min(i0 + kc.alpha, level);
        const uint64_t x = (t >= i0 && t < i1) ? w[off_d + at(t, log_n, k)]
                                                : w[off_ext + at(j * rows + t, log_n, k)];
        mac128(a0, x, key[at((2 * j) * krows + krow, log_n, k)]);
        mac128(a1, x, key[at((2 * j + 1) * krows + krow, log_n, k)]);
        if ((j & 7u) == 7u || j + 1 == beta) {
            r0 = add_mod(r0, mont_redc(a0.lo, a0.hi, md.q, md.mont_neg_qinv), md.q);
            r1 = add_mod(r1, mont_redc(a1.lo, a1.hi, md.q, md.mont_neg_qinv), md.q);
            a0 = {0, 0};
            a1 = {0, 0};
        }
    }
    acc[at(t, log_n, k)] = r0;
    acc[at(rows + t, log_n, k)] = r1;
}

// The same inner product for all n_items ciphertexts of a launch, one thread
// per (coefficient, row): the 2 BETA key residues of the row are loaded once
// and reused for every item (the key is shared by the batch), then each item
// reads its BETA inputs and writes its two outputs.  The inputs of item z + 1
// are in flight while item z is computed.  Rows with q < 2^50 work in fp64
// (keys taken out of Montgomery form once per thread, each product by
// fmulmod: |term| < 3q/4, the sum of at most 8 terms stays exact); the others
// accumulate 128-bit products and finish with one REDC.
#define PFT_KEY_REGS 8
template <uint32_t BETA>
__global__ __launch_bounds__(TB) void k_key_inner_items(WsRef ws, uint32_t n_items, uint64_t off_d, uint64_t off_ext,
                                                        uint64_t off_acc, const uint64_t* __restrict__ key,
                                                        uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
                                                        uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t t = blockIdx.y;
    const uint32_t rows = level + kc.K;
    const uint32_t krow = t < level ? t : kc.L + (t - level);
    const DevMod md = mods[krow];
    const uint32_t krows = kc.L + kc.K;
    // word offset of digit j's input on this row within an item's workspace:
    // d itself on the digit's own rows, ext_j elsewhere
    uint64_t src[BETA];
#pragma unroll
    for (uint32_t j = 0; j < BETA; ++j) {
        const bool own = t >= j * kc.alpha && t < min(j * kc.alpha + kc.alpha, level);
        src[j] = own ? off_d + at(t, log_n, k) : off_ext + at(j * rows + t, log_n, k);
    }
    uint64_t k0[BETA], k1[BETA];
#pragma unroll
    for (uint32_t j = 0; j < BETA; ++j) {
        k0[j] = key[at((2 * j) * krows + krow, log_n, k)];
        k1[j] = key[at((2 * j + 1) * krows + krow, log_n, k)];
    }
    uint64_t xn[BETA];
#pragma unroll
    for (uint32_t j = 0; j < BETA; ++j) xn[j] = ws.base[src[j]];
    const uint64_t o0 = off_acc + at(t, log_n, k), o1 = off_acc + at(rows + t, log_n, k);
    if (md.fp) {
        double w0[BETA], p0[BETA], w1[BETA], p1[BETA];
#pragma unroll
        for (uint32_t j = 0; j < BETA; ++j) {
            w0[j] = as_f(k0[j]);
            w1[j] = as_f(k1[j]);
            p0[j] = w0[j] / md.qd;
            p1[j] = w1[j] / md.qd;
        }
        for (uint32_t z = 0; z < n_items; ++z) {
            uint64_t* __restrict__ w = ws.base + (size_t)z * ws.stride;
            double x[BETA];
#pragma unroll
            for (uint32_t j = 0; j < BETA; ++j) x[j] = as_f(fp_from_u64(xn[j]));
            if (z + 1 < n_items) {
#pragma unroll
                for (uint32_t j = 0; j < BETA; ++j) xn[j] = w[ws.stride + src[j]];
            }
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (uint32_t j = 0; j < BETA; ++j) {
                s0 += fmulmod(x[j], w0[j], p0[j], md.qd);
                s1 += fmulmod(x[j], w1[j], p1[j], md.qd);
            }
            w[o0] = fp_to_u64(as_u(s0), md.qd, md.qinv);
            w[o1] = fp_to_u64(as_u(s1), md.qd, md.qinv);
        }
    } else {
        for (uint32_t z = 0; z < n_items; ++z) {
            uint64_t* __restrict__ w = ws.base + (size_t)z * ws.stride;
            uint64_t x[BETA];
#pragma unroll
            for (uint32_t j = 0; j < BETA; ++j) x[j] = xn[j];
            if (z + 1 < n_items) {
#pragma unroll
                for (uint32_t j = 0; j < BETA; ++j) xn[j] = w[ws.stride + src[j]];
            }
            Acc128 a0 = {0, 0}, a1 = {0, 0};
#pragma unroll
            for (uint32_t j = 0; j < BETA; ++j) {
                mac128(a0, x[j], k0[j]);
                mac128(a1, x[j], k1[j]);
            }
            w[o0] = mont_redc(a0.lo, a0.hi, md.q, md.mont_neg_qinv);
            w[o1] = mont_redc(a1.lo, a1.hi, md.q, md.mont_neg_qinv);
        }
    }
}

// ModDown conversion of the K special rows (coefficient form) of acc_b:
// y_k = acc_b[level+k] (P/p_k)^-1 mod p_k; conv_b[i] = sum_k y_k ((P/p_k) mod q_i).
__global__ __launch_bounds__(TB) void k_moddown_conv_b(WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                                                       KsConsts kc, const DevMod* __restrict__ mods,
                                                       uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t b = blockIdx.y;
    const uint32_t rows = level + kc.K;
    const uint64_t* __restrict__ acc = ws_item(ws) + off_acc;
    uint64_t* __restrict__ conv = ws_item(ws) + off_conv;
    uint64_t y[PFT_MAX_K];
#pragma unroll
    for (uint32_t kk = 0; kk < PFT_MAX_K; ++kk) {
        if (kk < kc.K) {
            const TwPair h = kc.down_phatinv[kk];
            y[kk] = shoup(acc[at(b * rows + level + kk, log_n, k)], h.w, h.wp, mods[kc.L + kk].q);
        }
    }
    for (uint32_t i = 0; i < level; ++i) {
        const DevMod md = mods[i];
        Acc128 a = {0, 0};
#pragma unroll
        for (uint32_t kk = 0; kk < PFT_MAX_K; ++kk)
            if (kk < kc.K) mac128(a, y[kk], kc.down_c[kk * kc.L + i]);
        conv[at(b * level + i, log_n, k)] = mont_redc(a.lo, a.hi, md.q, md.mont_neg_qinv);
    }
}

// RESCALE, step 1: last_z ([2][N], coefficient form of limb level-1) ->
// tmp_z [2][level-1][N] with ((r + h) mod q_last) - h reduced mod q_k,
// h = (q_last - 1)/2 (mode 0, rounding) or 0 (mode 1, floor).
__global__ __launch_bounds__(TB) void k_rescale_expand_b(WsRef ws, uint64_t off_last, uint64_t off_tmp,
                                                         uint32_t level, uint32_t mode,
                                                         const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t nl = level - 1;
    const uint32_t b = blockIdx.y / nl, kq = blockIdx.y % nl;
    const uint64_t ql = mods[level - 1].q;
    const uint64_t h = mode == 0 ? (ql - 1) / 2 : 0;
    const uint64_t* __restrict__ w = ws_item(ws);
    uint64_t r = w[off_last + at(b, log_n, k)] + h;
    r = r >= ql ? r - ql : r;             // (c_last + h) mod q_last
    const uint64_t qk = mods[kq].q;       // q_last < q_k, so r - h lies in (-q_k, q_k)
    ws_item(ws)[off_tmp + at(b * nl + kq, log_n, k)] = r >= h ? r - h : r + qk - h;
}

// ws_z[off_out] = ws_z[off_a] + ws_z[off_b] over [2][level][N]
__global__ __launch_bounds__(TB) void k_add_ct_b(WsRef ws, uint64_t off_a, uint64_t off_b, uint64_t off_out,
                                                 uint32_t level, const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t row = blockIdx.y;
    const uint64_t q = mods[row % level].q;
    uint64_t* __restrict__ w = ws_item(ws);
    const size_t o = at(row, log_n, k);
    w[off_out + o] = add_mod(w[off_a + o], w[off_b + o], q);
}

// The inner sums of up to PT_GT giant steps at once: for g < n_g,
// acc_{z,g}[row] = sum_{j<J} baby_{z,j}[row] pt_{g,j}[row mod level], acc_{z,g}
// at ws_z + off_acc + g ct_words, pt_{g,j} at pt + (g J + j) level N; each
// baby residue is read once for all n_g giant steps (or outputs).  One thread
// per (item, row, coefficient); the items of one coefficient block are
// consecutive workgroups (items vary fastest), so the plaintext tiles they
// share are fetched about once per launch.  The plaintext rows hold
// plaintext * 2^64 mod q (Montgomery form); each 128-bit sum of full products
// is reduced every 8 terms, which keeps it below q 2^64.
constexpr uint32_t PT_GT = 8;
__global__ __launch_bounds__(TB) void k_pt_dot_multi_b(WsRef ws, uint32_t n_items, uint64_t off_baby,
                                                       uint64_t ct_words, const uint64_t* __restrict__ pt, uint32_t J,
                                                       uint32_t n_g, uint64_t off_acc, uint32_t level,
                                                       const DevMod* __restrict__ mods, uint32_t log_n) {
    using u128 = unsigned __int128;
    const uint32_t kblocks = (1u << log_n) / TB;
    const uint32_t z = blockIdx.x % n_items;
    const uint32_t rest = blockIdx.x / n_items;
    const uint32_t k = (rest % kblocks) * TB + threadIdx.x;
    const uint32_t row = rest / kblocks, i = row % level;
    const DevMod md = mods[i];
    uint64_t* __restrict__ w = ws.base + (size_t)z * ws.stride;
    const size_t o = at(row, log_n, k);
    const size_t pstep = ((size_t)J * level) << log_n;  // words between giant steps of pt
    u128 a[PT_GT];
    uint64_t res[PT_GT];
#pragma unroll
    for (uint32_t g = 0; g < PT_GT; ++g) {
        a[g] = 0;
        res[g] = 0;
    }
    auto fold = [&](uint32_t g) {
        res[g] = add_mod(res[g], mont_redc((uint64_t)a[g], (uint64_t)(a[g] >> 64), md.q, md.mont_neg_qinv), md.q);
        a[g] = 0;
    };
    for (uint32_t j = 0; j < J; ++j) {
        const uint64_t x = w[off_baby + j * ct_words + o];
        const uint64_t* __restrict__ pj = pt + at(j * level + i, log_n, k);
#pragma unroll
        for (uint32_t g = 0; g < PT_GT; ++g)
            if (g < n_g) a[g] += (u128)x * pj[g * pstep];
        if ((j & 7u) == 7u) {
#pragma unroll
            for (uint32_t g = 0; g < PT_GT; ++g)
                if (g < n_g) fold(g);
        }
    }
#pragma unroll
    for (uint32_t g = 0; g < PT_GT; ++g)
        if (g < n_g) {
            fold(g);
            w[off_acc + g * ct_words + o] = res[g];
        }
}

// out_z = in_z + c_z at X^0: in the evaluation domain the constant c_z[i]
// (mod q_i) is added to every entry of limb i of c0; c1 is copied.
__global__ __launch_bounds__(TB) void k_add_const_b(ItemPtrs in, ItemPtrs out, const TwPair* __restrict__ consts,
                                                    uint32_t level, const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t row = blockIdx.y;
    const size_t o = at(row, log_n, k);
    uint64_t v = in.p[blockIdx.z][o];
    if (row < level) v = add_mod(v, consts[(size_t)blockIdx.z * level + row].w, mods[row].q);
    out.p[blockIdx.z][o] = v;
}

// HMUL tensors of the encrypted-weight matrix-vector product, summed over the
// J diagonal terms of each of n_g <= CT_GT giant steps (Sec. 4.2, HMUL in
// place of HMULPLAIN): d0 = sum e0 x0, d1 = sum (e0 x1 + e1 x0), d2 = sum
// e1 x1.  Giant step g takes its diagonals from e.p[g J + j] and writes
// [3][level][N] at item g n_items + z of ws + off_d; each baby residue is read
// once for all of them.  The full 128-bit products are summed and brought
// back by a Montgomery reduction every 8 diagonal terms (at most 16 products
// below q^2 each: below q 2^64 for q < 2^60); the reductions' factor 2^-64
// is undone once at the end by a Shoup product with 2^64 mod q (to_mont).
constexpr uint32_t CT_GT = 4;
__global__ __launch_bounds__(TB) void k_ct_dot_multi_b(ItemPtrs e, uint32_t J, uint32_t n_g, WsRef xs, uint64_t off_x,
                                                       uint64_t ct_words, WsRef ws, uint32_t n_items, uint64_t off_d,
                                                       uint32_t level, const DevMod* __restrict__ mods,
                                                       const TwPair* __restrict__ to_mont, uint32_t log_n) {
    using u128 = unsigned __int128;
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t i = blockIdx.y;
    const DevMod md = mods[i];
    const uint64_t q = md.q;
    const uint64_t* __restrict__ x = xs.base + (size_t)blockIdx.z * xs.stride + off_x;
    const size_t o0 = at(i, log_n, k), o1 = at(level + i, log_n, k);
    u128 s[CT_GT][3];
    uint64_t d[CT_GT][3];
#pragma unroll
    for (uint32_t g = 0; g < CT_GT; ++g)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            s[g][t] = 0;
            d[g][t] = 0;
        }
    auto fold = [&](uint32_t g) {
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            d[g][t] = add_mod(d[g][t], mont_redc((uint64_t)s[g][t], (uint64_t)(s[g][t] >> 64), q, md.mont_neg_qinv), q);
            s[g][t] = 0;
        }
    };
    for (uint32_t j = 0; j < J; ++j) {
        const uint64_t x0 = x[j * ct_words + o0], x1 = x[j * ct_words + o1];
#pragma unroll
        for (uint32_t g = 0; g < CT_GT; ++g)
            if (g < n_g) {
                const uint64_t* __restrict__ E = e.p[g * J + j];
                const uint64_t e0 = E[o0], e1 = E[o1];
                s[g][0] += (u128)e0 * x0;
                s[g][1] += (u128)e0 * x1 + (u128)e1 * x0;
                s[g][2] += (u128)e1 * x1;
            }
        if ((j & 7u) == 7u) {
#pragma unroll
            for (uint32_t g = 0; g < CT_GT; ++g)
                if (g < n_g) fold(g);
        }
    }
    const TwPair r = to_mont[i];
#pragma unroll
    for (uint32_t g = 0; g < CT_GT; ++g)
        if (g < n_g) {
            fold(g);
            uint64_t* __restrict__ dd = ws.base + (size_t)(g * n_items + blockIdx.z) * ws.stride + off_d;
            dd[o0] = shoup(d[g][0], r.w, r.wp, q);
            dd[o1] = shoup(d[g][1], r.w, r.wp, q);
            dd[at(2 * level + i, log_n, k)] = shoup(d[g][2], r.w, r.wp, q);
        }
}

// out_z[b][i] = in_z[b][i] * c_z[i] (Shoup pairs, [n][level] on the device):
// multiplication by an integer constant polynomial.
__global__ __launch_bounds__(TB) void k_scale_const_b(ItemPtrs in, ItemPtrs out, const TwPair* __restrict__ consts,
                                                      uint32_t level, const DevMod* __restrict__ mods,
                                                      uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t row = blockIdx.y, i = row % level;
    const TwPair w = consts[(size_t)blockIdx.z * level + i];
    out.p[blockIdx.z][at(row, log_n, k)] = shoup(in.p[blockIdx.z][at(row, log_n, k)], w.w, w.wp, mods[i].q);
}

inline dim3 grid_nk(uint32_t log_n, uint32_t y, uint32_t z = 1) { return dim3((1u << log_n) / TB, y, z); }

}  // namespace

void launch_int_to_rns(const int64_t* x, const SmallBatch& out, const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_int_to_rns, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, x, out, t.mods,
                       log_n);
}

void launch_ew(EwOp op, const SmallBatch& out, const SmallBatch& a, const SmallBatch* b, const SmallBatch* c,
               const DevTables& t, uint32_t log_n, hipStream_t st) {
    SmallBatch bb = b ? *b : a, cc = c ? *c : a;
    hipLaunchKernelGGL(k_ew, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, (uint32_t)op, out, a, bb,
                       cc, t.mods, log_n);
}

void launch_key_form(const SmallBatch& rows, const TwPair* to_mont, const DevTables& t, uint32_t log_n,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_key_form, grid_nk(log_n, rows.n_polys * rows.n_limbs), dim3(TB), 0, st, rows, to_mont,
                       t.mods, log_n);
}

void launch_mul_const(const SmallBatch& out, const SmallBatch& a, const TwPair* consts, const DevTables& t,
                      uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_mul_const, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, out, a, consts,
                       t.mods, log_n);
}

void launch_tensor_b(uint32_t n, const ItemPtrs& a, const ItemPtrs& b, WsRef ws, uint64_t off_d, uint32_t level,
                     const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_tensor_b, grid_nk(log_n, level, n), dim3(TB), 0, st, a, b, ws, off_d, level, t.mods, log_n);
}

void launch_copy_rows_b(uint32_t n, const ItemPtrs& src, uint64_t src_off, const ItemPtrs& dst, uint64_t dst_off,
                        uint32_t rows, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_rows_b, grid_nk(log_n, rows, n), dim3(TB), 0, st, src, src_off, dst, dst_off, log_n);
}

void launch_automorphism_b(uint32_t n, const ItemPtrs& in, uint32_t rows, WsRef ws, uint64_t off_out, uint64_t kappa,
                           uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_automorphism_b, grid_nk(log_n, rows, n), dim3(TB), 0, st, in, ws, off_out, kappa, log_n);
}

// calls f(std::integral_constant<uint32_t, v>) for the runtime v in 1..MAX
template <uint32_t MAX, uint32_t V = 1, class F>
static void launch_kb(uint32_t v, F&& f) {
    if constexpr (V <= MAX) {
        if (v == V) f(std::integral_constant<uint32_t, V>{});
        else launch_kb<MAX, V + 1>(v, f);
    }
}

void launch_modup_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level, const KsConsts& kc,
                    const DevTables& t, uint32_t log_n, bool mfma, hipStream_t st) {
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    if (mfma)  // 32 coefficients per wave
        launch_kb<PFT_MAX_ALPHA / 2>((min(kc.alpha, level) + 1) / 2, [&](auto nkb) {
            hipLaunchKernelGGL(k_modup_mfma_b<decltype(nkb)::value>, dim3((1u << log_n) / (32 * (TB / 64)), beta, n),
                               dim3(TB), 0, st, ws, off_d, off_ext, level, kc, t.mods, log_n);
        });
    else
        hipLaunchKernelGGL(k_modup_b, grid_nk(log_n, beta, n), dim3(TB), 0, st, ws, off_d, off_ext, level, kc,
                           t.mods, log_n);
}

void launch_key_inner_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint64_t off_acc, const uint64_t* key,
                        uint32_t level, const KsConsts& kc, const DevTables& t, uint32_t log_n, hipStream_t st) {
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    if (beta <= PFT_KEY_REGS)
        launch_kb<PFT_KEY_REGS>(beta, [&](auto bc) {
            hipLaunchKernelGGL(k_key_inner_items<decltype(bc)::value>, grid_nk(log_n, level + kc.K, 1), dim3(TB), 0,
                               st, ws, n, off_d, off_ext, off_acc, key, level, kc, t.mods, log_n);
        });
    else
        hipLaunchKernelGGL(k_key_inner_b, grid_nk(log_n, level + kc.K, n), dim3(TB), 0, st, ws, off_d, off_ext,
                           off_acc, key, level, kc, t.mods, log_n);
}

void launch_moddown_conv_b(uint32_t n, WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                           const KsConsts& kc, const DevTables& t, uint32_t log_n, bool mfma, hipStream_t st) {
    if (mfma)
        launch_kb<PFT_MAX_K / 2>((kc.K + 1) / 2, [&](auto nkb) {
            hipLaunchKernelGGL(k_moddown_mfma_b<decltype(nkb)::value>, dim3((1u << log_n) / (32 * (TB / 64)), 2, n),
                               dim3(TB), 0, st, ws, off_acc, off_conv, level, kc, t.mods, log_n);
        });
    else
        hipLaunchKernelGGL(k_moddown_conv_b, grid_nk(log_n, 2, n), dim3(TB), 0, st, ws, off_acc, off_conv, level,
                           kc, t.mods, log_n);
}

void launch_rescale_expand_b(uint32_t n, WsRef ws, uint64_t off_last, uint64_t off_tmp, uint32_t level, uint32_t mode,
                             const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_rescale_expand_b, grid_nk(log_n, 2 * (level - 1), n), dim3(TB), 0, st, ws, off_last,
                       off_tmp, level, mode, t.mods, log_n);
}

void launch_add_ct_b(uint32_t n, WsRef ws, uint64_t off_a, uint64_t off_b, uint64_t off_out, uint32_t level,
                     const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_ct_b, grid_nk(log_n, 2 * level, n), dim3(TB), 0, st, ws, off_a, off_b, off_out, level,
                       t.mods, log_n);
}

uint32_t pt_dot_multi_steps() { return PT_GT; }

void launch_pt_dot_multi_b(uint32_t n, WsRef ws, uint64_t off_baby, uint64_t ct_words, const uint64_t* pt, uint32_t J,
                           uint32_t n_g, uint64_t off_acc, uint32_t level, const DevTables& t, uint32_t log_n,
                           hipStream_t st) {
    const uint64_t blocks = (uint64_t)n * ((1u << log_n) / TB) * 2 * level;
    hipLaunchKernelGGL(k_pt_dot_multi_b, dim3((uint32_t)blocks), dim3(TB), 0, st, ws, n, off_baby, ct_words, pt, J, n_g,
                       off_acc, level, t.mods, log_n);
}

void launch_add_const_b(uint32_t n, const ItemPtrs& in, const ItemPtrs& out, const TwPair* consts, uint32_t level,
                        const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_add_const_b, grid_nk(log_n, 2 * level, n), dim3(TB), 0, st, in, out, consts, level, t.mods,
                       log_n);
}

uint32_t ct_dot_multi_steps() { return CT_GT; }

void launch_ct_dot_multi_b(uint32_t n, const ItemPtrs& e, uint32_t J, uint32_t n_g, WsRef xs, uint64_t off_x,
                           uint64_t ct_words, WsRef ws, uint64_t off_d, uint32_t level, const TwPair* to_mont,
                           const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_ct_dot_multi_b, grid_nk(log_n, level, n), dim3(TB), 0, st, e, J, n_g, xs, off_x, ct_words, ws,
                       n, off_d, level, t.mods, to_mont, log_n);
}

void launch_scale_const_b(uint32_t n, const ItemPtrs& in, const ItemPtrs& out, const TwPair* consts, uint32_t level,
                          const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_const_b, grid_nk(log_n, 2 * level, n), dim3(TB), 0, st, in, out, consts, level,
                       t.mods, log_n);
}
