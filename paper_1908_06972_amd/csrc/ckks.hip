// ckks.hip -- limb-parallel kernels of the CKKS homomorphic operations
// (Sec. 3.4 HADD/HMUL/HMULPLAIN/ROTATE, Sec. 5.1 RESCALE) and of hybrid key
// switching (ModUp base conversion, key inner product, ModDown).
//
// Every kernel maps one thread to one coefficient index k of one limb row;
// consecutive lanes touch consecutive k, so every global access is a
// coalesced row segment of the limb-major [poly][limb][N] layout.
#include "pft_device.h"
#include "pft_kernels.h"

#define PFT_MAX_ALPHA 12
#define PFT_MAX_K 12

namespace {

constexpr uint32_t TB = 256;

__global__ __launch_bounds__(TB) void k_int_to_rns(const int64_t* __restrict__ x, PolyBatch out,
                                                   const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = pb_row(out, limb);
    const uint64_t q = mods[pb_mod(out, row)].q;
    const int64_t v = x[((size_t)poly << log_n) + k];
    uint64_t r;
    if (v >= 0) {
        r = (uint64_t)v % q;
    } else {
        const uint64_t mag = (0ull - (uint64_t)v) % q;
        r = mag == 0 ? 0 : q - mag;
    }
    out.ptr[poly][((size_t)row << log_n) + k] = r;
}

__global__ __launch_bounds__(TB) void k_ew(uint32_t op, PolyBatch out, PolyBatch a, PolyBatch b, PolyBatch c,
                                           const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = pb_row(out, limb);
    const DevMod md = mods[pb_mod(out, row)];
    const size_t oa = ((size_t)pb_row(a, limb) << log_n) + k;
    const uint64_t x = a.ptr[poly][oa];
    uint64_t r = 0;
    switch (op) {
        case EW_ADD: r = add_mod(x, b.ptr[poly][((size_t)pb_row(b, limb) << log_n) + k], md.q); break;
        case EW_SUB: r = sub_mod(x, b.ptr[poly][((size_t)pb_row(b, limb) << log_n) + k], md.q); break;
        case EW_MUL: r = mul_barrett(x, b.ptr[poly][((size_t)pb_row(b, limb) << log_n) + k], md); break;
        case EW_MULADD:
            r = add_mod(mul_barrett(x, b.ptr[poly][((size_t)pb_row(b, limb) << log_n) + k], md),
                        c.ptr[poly][((size_t)pb_row(c, limb) << log_n) + k], md.q);
            break;
        case EW_NEG_MULADD:
            r = sub_mod(c.ptr[poly][((size_t)pb_row(c, limb) << log_n) + k],
                        mul_barrett(x, b.ptr[poly][((size_t)pb_row(b, limb) << log_n) + k], md), md.q);
            break;
        default: r = x; break;
    }
    out.ptr[poly][((size_t)row << log_n) + k] = r;
}

__global__ __launch_bounds__(TB) void k_mul_const(PolyBatch out, PolyBatch a, const TwPair* __restrict__ consts,
                                                  const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t limb = blockIdx.y / out.n_polys, poly = blockIdx.y % out.n_polys;
    const uint32_t row = pb_row(out, limb);
    const uint64_t q = mods[pb_mod(out, row)].q;
    const TwPair w = consts[limb];
    const uint64_t x = a.ptr[poly][((size_t)pb_row(a, limb) << log_n) + k];
    out.ptr[poly][((size_t)row << log_n) + k] = shoup(x, w.w, w.wp, q);
}

__global__ __launch_bounds__(TB) void k_tensor(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                               uint64_t* __restrict__ d0, uint64_t* __restrict__ d1,
                                               uint64_t* __restrict__ d2, uint32_t level,
                                               const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t i = blockIdx.y;
    const DevMod md = mods[i];
    const size_t o0 = ((size_t)i << log_n) + k, o1 = ((size_t)(level + i) << log_n) + k;
    const uint64_t a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
    d0[o0] = mul_barrett(a0, b0, md);
    d1[o0] = add_mod(mul_barrett(a0, b1, md), mul_barrett(a1, b0, md), md.q);
    d2[o0] = mul_barrett(a1, b1, md);
}

// NTT-domain X -> X^kappa.  Entry k holds the evaluation at psi^e with
// e = 2 brv(k) + 1; a(X^kappa) there equals a at psi^(e kappa mod 2N), which
// is stored at brv((e kappa mod 2N - 1) / 2).
__global__ __launch_bounds__(TB) void k_automorphism(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                     uint64_t kappa, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const size_t base = (size_t)blockIdx.y << log_n;
    const uint64_t e = 2ull * brev_n(k, log_n) + 1;
    const uint64_t e2 = (e * kappa) & ((2ull << log_n) - 1);
    const uint32_t src = brev_n((uint32_t)((e2 - 1) >> 1), log_n);
    out[base + k] = in[base + src];
}

// ModUp: for digit j = blockIdx.y of a ciphertext at `level`:
// xt_i = d_i * (D_j/q_i)^-1 mod q_i, ext_j[t] = sum_i xt_i ((D_j/q_i) mod m_t)
// for every row t outside the digit (q-limbs then special primes).
__global__ __launch_bounds__(TB) void k_modup(const uint64_t* __restrict__ d, uint64_t* __restrict__ ext,
                                              uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
                                              uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t j = blockIdx.y;
    const uint32_t i0 = j * kc.alpha;
    const uint32_t i1 = min(i0 + kc.alpha, level);
    const uint32_t na = i1 - i0;
    const uint32_t rows = level + kc.K;
    const size_t cbase = ((size_t)(level - 1) * kc.dnum + j) * kc.alpha;
    uint64_t xt[PFT_MAX_ALPHA];
#pragma unroll
    for (uint32_t ii = 0; ii < PFT_MAX_ALPHA; ++ii) {
        if (ii < na) {
            const TwPair h = kc.modup_hatinv[cbase + ii];
            xt[ii] = shoup(d[((size_t)(i0 + ii) << log_n) + k], h.w, h.wp, mods[i0 + ii].q);
        }
    }
    uint64_t* __restrict__ outj = ext + ((size_t)j * rows << log_n);
    for (uint32_t t = 0; t < rows; ++t) {
        if (t >= i0 && t < i1) continue;
        const uint32_t mi = t < level ? t : kc.L + (t - level);
        const DevMod md = mods[mi];
        Acc128 acc = {0, 0};
#pragma unroll
        for (uint32_t ii = 0; ii < PFT_MAX_ALPHA; ++ii)
            if (ii < na) mac128(acc, xt[ii], kc.modup_c[(cbase + ii) * (kc.L + kc.K) + t]);
        outj[((size_t)t << log_n) + k] = mont_redc(acc.lo, acc.hi, md.q, md.mont_neg_qinv);
    }
}

// acc_b[t] = sum_j x_j[t] key_{j,b}[row(t)], x_j = d (NTT) on digit j's own
// rows and ext_j elsewhere; keys are stored times 2^64 (Montgomery).
__global__ __launch_bounds__(TB) void k_key_inner(const uint64_t* __restrict__ d, const uint64_t* __restrict__ ext,
                                                  const uint64_t* __restrict__ key, uint64_t* __restrict__ acc,
                                                  uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
                                                  uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t t = blockIdx.y;
    const uint32_t rows = level + kc.K;
    const uint32_t krow = t < level ? t : kc.L + (t - level);
    const DevMod md = mods[krow];
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    const uint32_t krows = kc.L + kc.K;
    Acc128 a0 = {0, 0}, a1 = {0, 0};
    for (uint32_t j = 0; j < beta; ++j) {
        const uint32_t i0 = j * kc.alpha, i1 = min(i0 + kc.alpha, level);
        const uint64_t x = (t >= i0 && t < i1) ? d[((size_t)t << log_n) + k]
                                                : ext[((size_t)(j * rows + t) << log_n) + k];
        const uint64_t kb = key[((size_t)((2 * j) * krows + krow) << log_n) + k];
        const uint64_t ka = key[((size_t)((2 * j + 1) * krows + krow) << log_n) + k];
        mac128(a0, x, kb);
        mac128(a1, x, ka);
    }
    acc[((size_t)t << log_n) + k] = mont_redc(a0.lo, a0.hi, md.q, md.mont_neg_qinv);
    acc[((size_t)(rows + t) << log_n) + k] = mont_redc(a1.lo, a1.hi, md.q, md.mont_neg_qinv);
}

// ModDown conversion of the K special rows (coefficient form) of acc_b:
// y_k = acc_b[level+k] * (P/p_k)^-1 mod p_k; conv_b[i] = sum_k y_k ((P/p_k) mod q_i).
__global__ __launch_bounds__(TB) void k_moddown_conv(const uint64_t* __restrict__ acc, uint64_t* __restrict__ conv,
                                                     uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
                                                     uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t b = blockIdx.y;
    const uint32_t rows = level + kc.K;
    uint64_t y[PFT_MAX_K];
#pragma unroll
    for (uint32_t kk = 0; kk < PFT_MAX_K; ++kk) {
        if (kk < kc.K) {
            const TwPair h = kc.down_phatinv[kk];
            y[kk] = shoup(acc[((size_t)(b * rows + level + kk) << log_n) + k], h.w, h.wp, mods[kc.L + kk].q);
        }
    }
    for (uint32_t i = 0; i < level; ++i) {
        const DevMod md = mods[i];
        Acc128 a = {0, 0};
#pragma unroll
        for (uint32_t kk = 0; kk < PFT_MAX_K; ++kk)
            if (kk < kc.K) mac128(a, y[kk], kc.down_c[kk * kc.L + i]);
        conv[((size_t)(b * level + i) << log_n) + k] = mont_redc(a.lo, a.hi, md.q, md.mont_neg_qinv);
    }
}

__global__ __launch_bounds__(TB) void k_moddown_final(const uint64_t* __restrict__ acc,
                                                      const uint64_t* __restrict__ conv,
                                                      const uint64_t* __restrict__ add0,
                                                      const uint64_t* __restrict__ add1, uint64_t* __restrict__ out,
                                                      uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
                                                      uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t b = blockIdx.y / level, i = blockIdx.y % level;
    const uint32_t rows = level + kc.K;
    const uint64_t q = mods[i].q;
    const uint64_t x = acc[((size_t)(b * rows + i) << log_n) + k];
    const uint64_t c = conv[((size_t)(b * level + i) << log_n) + k];
    const TwPair w = kc.down_pinv[i];
    uint64_t r = shoup(x + q - c, w.w, w.wp, q);
    const uint64_t* add = b == 0 ? add0 : add1;
    if (add) r = add_mod(r, add[((size_t)i << log_n) + k], q);
    out[((size_t)(b * level + i) << log_n) + k] = r;
}

__global__ __launch_bounds__(TB) void k_rescale_expand(const uint64_t* __restrict__ last, uint64_t* __restrict__ tmp,
                                                       uint32_t level, uint32_t mode,
                                                       const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t nl = level - 1;
    const uint32_t b = blockIdx.y / nl, kq = blockIdx.y % nl;
    const uint64_t ql = mods[level - 1].q;
    const uint64_t h = mode == 0 ? (ql - 1) / 2 : 0;
    uint64_t r = last[((size_t)b << log_n) + k] + h;
    r = r >= ql ? r - ql : r;             // (c_last + h) mod q_last
    const uint64_t qk = mods[kq].q;       // q_last < q_k: r - h lies in (-q_k, q_k)
    const uint64_t v = r >= h ? r - h : r + qk - h;
    tmp[((size_t)(b * nl + kq) << log_n) + k] = v;
}

__global__ __launch_bounds__(TB) void k_rescale_final(const uint64_t* __restrict__ c, const uint64_t* __restrict__ tmp,
                                                      uint64_t* __restrict__ out, uint32_t level,
                                                      const TwPair* __restrict__ qinv,
                                                      const DevMod* __restrict__ mods, uint32_t log_n) {
    const uint32_t k = blockIdx.x * TB + threadIdx.x;
    const uint32_t nl = level - 1;
    const uint32_t b = blockIdx.y / nl, kq = blockIdx.y % nl;
    const uint64_t q = mods[kq].q;
    const uint64_t x = c[((size_t)(b * level + kq) << log_n) + k];
    const uint64_t t = tmp[((size_t)(b * nl + kq) << log_n) + k];
    const TwPair w = qinv[kq];
    out[((size_t)(b * nl + kq) << log_n) + k] = shoup(x + q - t, w.w, w.wp, q);
}

inline dim3 grid_nk(uint32_t log_n, uint32_t y) { return dim3((1u << log_n) / TB, y); }

}  // namespace

void launch_int_to_rns(const int64_t* x, const PolyBatch& out, const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_int_to_rns, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, x, out, t.mods,
                       log_n);
}

void launch_ew(EwOp op, const PolyBatch& out, const PolyBatch& a, const PolyBatch* b, const PolyBatch* c,
               const DevTables& t, uint32_t log_n, hipStream_t st) {
    PolyBatch bb = b ? *b : a, cc = c ? *c : a;
    hipLaunchKernelGGL(k_ew, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, (uint32_t)op, out, a, bb,
                       cc, t.mods, log_n);
}

void launch_mul_const(const PolyBatch& out, const PolyBatch& a, const TwPair* consts, const DevTables& t,
                      uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_mul_const, grid_nk(log_n, out.n_polys * out.n_limbs), dim3(TB), 0, st, out, a, consts,
                       t.mods, log_n);
}

void launch_tensor(const uint64_t* a, const uint64_t* b, uint64_t* d0, uint64_t* d1, uint64_t* d2, uint32_t level,
                   const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_tensor, grid_nk(log_n, level), dim3(TB), 0, st, a, b, d0, d1, d2, level, t.mods, log_n);
}

void launch_automorphism(const uint64_t* in, uint64_t* out, uint32_t n_polys, uint32_t level, uint64_t kappa,
                         uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_automorphism, grid_nk(log_n, n_polys * level), dim3(TB), 0, st, in, out, kappa, log_n);
}

void launch_modup(const uint64_t* d_coef, uint64_t* ext, uint32_t level, const KsConsts& kc, const DevTables& t,
                  uint32_t log_n, hipStream_t st) {
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    hipLaunchKernelGGL(k_modup, grid_nk(log_n, beta), dim3(TB), 0, st, d_coef, ext, level, kc, t.mods, log_n);
}

void launch_key_inner(const uint64_t* d_ntt, const uint64_t* ext, const uint64_t* key, uint64_t* acc, uint32_t level,
                      const KsConsts& kc, const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_key_inner, grid_nk(log_n, level + kc.K), dim3(TB), 0, st, d_ntt, ext, key, acc, level, kc,
                       t.mods, log_n);
}

void launch_moddown_conv(const uint64_t* acc, uint64_t* conv, uint32_t level, const KsConsts& kc, const DevTables& t,
                         uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_moddown_conv, grid_nk(log_n, 2), dim3(TB), 0, st, acc, conv, level, kc, t.mods, log_n);
}

void launch_moddown_final(const uint64_t* acc, const uint64_t* conv, const uint64_t* add0, const uint64_t* add1,
                          uint64_t* out, uint32_t level, const KsConsts& kc, const DevTables& t, uint32_t log_n,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_moddown_final, grid_nk(log_n, 2 * level), dim3(TB), 0, st, acc, conv, add0, add1, out, level,
                       kc, t.mods, log_n);
}

void launch_rescale_expand(const uint64_t* last, uint64_t* tmp, uint32_t level, uint32_t mode, const DevTables& t,
                           uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_rescale_expand, grid_nk(log_n, 2 * (level - 1)), dim3(TB), 0, st, last, tmp, level, mode,
                       t.mods, log_n);
}

void launch_rescale_final(const uint64_t* c, const uint64_t* tmp, uint64_t* out, uint32_t level,
                          const TwPair* qinv, const DevTables& t, uint32_t log_n, hipStream_t st) {
    hipLaunchKernelGGL(k_rescale_final, grid_nk(log_n, 2 * (level - 1)), dim3(TB), 0, st, c, tmp, out, level, qinv,
                       t.mods, log_n);
}
