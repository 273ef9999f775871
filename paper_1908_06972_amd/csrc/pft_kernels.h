// pft_kernels.h -- host-side launchers of the HIP kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pft_device.h"

// Device-resident per-parameter-set tables.
struct DevTables {
    DevMod* mods;     // [L+K]: q_0..q_{L-1}, p_0..p_{K-1}
    TwPair* tw_fwd;   // [L+K][N]: psi^brv(k)
    TwPair* tw_inv;   // [L+K][N]: psi^-brv(k)
};

bool ntt_supported(uint32_t log_n);
void launch_ntt(const PolyBatch& b, const DevTables& t, uint32_t log_n, bool inverse, hipStream_t st);

// ---- elementwise kernels (ckks.hip) --------------------------------------
// Signed small/integer polynomial x ([N] int64, device) reduced into every
// limb of `out`.
void launch_int_to_rns(const int64_t* x, const PolyBatch& out, const DevTables& t, uint32_t log_n, hipStream_t st);

// Limb-wise ops on NTT-domain data.  Each operand is a PolyBatch with the
// same shape; modulus mapping taken from `out`.
enum EwOp : uint32_t {
    EW_ADD = 0,       // out = a + b
    EW_SUB = 1,       // out = a - b
    EW_MUL = 2,       // out = a * b
    EW_MULADD = 3,    // out = a * b + c
    EW_NEG_MULADD = 4,  // out = -(a * b) + c
    EW_COPY = 5,      // out = a
};
void launch_ew(EwOp op, const PolyBatch& out, const PolyBatch& a, const PolyBatch* b, const PolyBatch* c,
               const DevTables& t, uint32_t log_n, hipStream_t st);
// out = a * const_r (Shoup) per limb, consts indexed by limb: (w, w') pairs on device
void launch_mul_const(const PolyBatch& out, const PolyBatch& a, const TwPair* consts, const DevTables& t,
                      uint32_t log_n, hipStream_t st);

// HMUL tensor: d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 over `level` limbs.
void launch_tensor(const uint64_t* a, const uint64_t* b, uint64_t* d0, uint64_t* d1, uint64_t* d2, uint32_t level,
                   const DevTables& t, uint32_t log_n, hipStream_t st);

// NTT-domain automorphism X -> X^kappa: out[k] = in[perm(k)] for n_limbs of
// n_polys polynomials of a [n_polys][level][N] array.
void launch_automorphism(const uint64_t* in, uint64_t* out, uint32_t n_polys, uint32_t level, uint64_t kappa,
                         uint32_t log_n, hipStream_t st);

// Key switching pieces.
struct KsConsts {
    const TwPair* modup_hatinv;   // [L][dnum][alpha]   indexed by (level-1, j, ii)
    const uint64_t* modup_c;      // [L][dnum][alpha][L+K] Montgomery form, row = target row
    const TwPair* down_phatinv;   // [K]
    const uint64_t* down_c;       // [K][L] Montgomery form
    const TwPair* down_pinv;      // [L]
    uint32_t L, K, dnum, alpha;
};
// ModUp base conversion: d_coef [level][N] -> ext [beta][level+K][N]
// (coefficient form; rows inside digit j of ext_j are left untouched).
void launch_modup(const uint64_t* d_coef, uint64_t* ext, uint32_t level, const KsConsts& kc, const DevTables& t,
                  uint32_t log_n, hipStream_t st);
// acc [2][level+K][N] = sum_j ext_j (or d_ntt on digit rows) * key_j (Montgomery)
void launch_key_inner(const uint64_t* d_ntt, const uint64_t* ext, const uint64_t* key, uint64_t* acc, uint32_t level,
                      const KsConsts& kc, const DevTables& t, uint32_t log_n, hipStream_t st);
// ModDown conversion: acc special rows (coefficient form) -> conv [2][level][N] coefficient form
void launch_moddown_conv(const uint64_t* acc, uint64_t* conv, uint32_t level, const KsConsts& kc, const DevTables& t,
                         uint32_t log_n, hipStream_t st);
// out_b[i] = (acc_b[i] - conv_b[i]) P^-1 + add_b[i]   (add may be null; add1 null -> no add on poly 1)
void launch_moddown_final(const uint64_t* acc, const uint64_t* conv, const uint64_t* add0, const uint64_t* add1,
                          uint64_t* out, uint32_t level, const KsConsts& kc, const DevTables& t, uint32_t log_n,
                          hipStream_t st);

// Rescale: last (coefficient form, [2][N]) -> tmp [2][level-1][N] holding
// ((r + h) mod q_last) - h reduced mod q_k (h = (q_last-1)/2 or 0).
void launch_rescale_expand(const uint64_t* last, uint64_t* tmp, uint32_t level, uint32_t mode, const DevTables& t,
                           uint32_t log_n, hipStream_t st);
// out_b[k] = (c_b[k] - tmp_b[k]) * q_last^-1 (consts [level-1] pairs)
void launch_rescale_final(const uint64_t* c, const uint64_t* tmp, uint64_t* out, uint32_t level,
                          const TwPair* qinv, const DevTables& t, uint32_t log_n, hipStream_t st);
