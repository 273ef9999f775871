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

// Optional per-launch timing: begin/end bracket one kernel launch with HIP
// events on the launch stream and record its algorithmic traffic and work.
enum ProfKernel : int {
    PK_NTT_FWD = 0, PK_NTT_INV = 1, PK_MODUP = 2, PK_KEY_INNER = 3, PK_MODDOWN_CONV = 4,
    PK_MODDOWN_FINAL = 5, PK_TENSOR = 6, PK_AUTOMORPHISM = 7, PK_RESCALE = 8, PK_ELEMENTWISE = 9, PK_COUNT = 10
};
// variant: which instantiation of the family ran (0 for single-kernel
// families; NTT passes: 1 + (radix | col << 5 | final << 6 | staged << 7)).
struct ProfHook {
    // st: the stream the bracketed launch goes to (null: the context stream)
    virtual void begin(int kid, hipStream_t st = nullptr) = 0;
    virtual void end(int kid, double bytes, double ops, uint32_t variant = 0, hipStream_t st = nullptr) = 0;
    virtual ~ProfHook() {}
};

// An NTT pass schedule: the radices (log2 of the stage windows) in forward
// order, summing to log2 N, and flags.
enum : uint32_t {
    NTT_DIRECT_ROWS = 1,  // row pass reads/writes its strided side directly
    NTT_E8 = 2            // 8 residues per thread (512-thread workgroups) instead of 16
};
struct NttSchedule {
    uint32_t n_passes;
    uint8_t radix[4];
    uint32_t flags;
};
// Epilogue of a forward transform's final pass that finishes ModDown in
// place of storing the transform: for transformed row i of polynomial p =
// 2 z + b (z the item, b in {0, 1}) it writes
//   out_z[b][i] = (acc - conv) P^-1 mod q_i (+ add) (+ add2)
// where conv is the transformed value and acc / add / add2 sit at word
// offsets d_acc[b] / d_add[b] / d_add2[b] from it (PFT_EPI_NO_ADD: no
// addend), or acc is row i of polynomial b of an item's own ciphertext
// (PFT_EPI_ITEM_ACC; RESCALE uses this with P^-1 replaced by q_last^-1).  out
// may coincide with an addend (each element is read before it is written).
#define PFT_EPI_NO_ADD INT64_MIN
#define PFT_EPI_ITEM_ACC (INT64_MIN + 1)
struct NttEpilogue {
    int64_t d_acc[2];   // or PFT_EPI_ITEM_ACC: acc of item z at acc_item[z] + (b acc_level + i) N
    int64_t d_add[2];
    int64_t d_add2[2];  // a second addend, or PFT_EPI_NO_ADD
    uint64_t* out[PFT_MAX_POLYS / 2];  // per item of the launch: [2][level][N]
    const uint64_t* acc_item[PFT_MAX_POLYS / 2];
    uint32_t acc_level;
    const TwPair* pinv;                // [L]: P^-1 mod q_i (Shoup pairs)
    const TwPair* pinv_fp;             // [L]: the same as (w, w/q) doubles, used where q_i < 2^50
    uint32_t level;
    // X -> X^kappa (kappa = 0: none) folded into a row pass: the first pass
    // of an inverse transform reads row i of polynomial p from perm_src[p]
    // + i N through the permutation; a forward epilogue adds, for the first
    // polynomial of item z, row i of perm_src[z] through the permutation.
    // kappa_inv = kappa^-1 mod 2N.
    const uint64_t* perm_src[PFT_MAX_POLYS / 2];
    uint64_t kappa, kappa_inv;
};
bool ntt_supported(uint32_t log_n);
int ntt_candidates(uint32_t log_n, NttSchedule* out, int max_out);
bool ntt_schedule_valid(uint32_t log_n, const NttSchedule& s);
// epi, forward: finish ModDown in the final pass instead of storing (and
// add the permuted addend when epi->kappa is set); inverse: only
// epi->kappa / perm_src are used, by the first pass.
// first: a forward transform starts at pass `first` of the schedule (the
// earlier passes already applied, e.g. by launch_modup_col_b); an inverse
// transform stops before pass `first` (the remaining passes applied by the
// consumer, e.g. launch_modup_col_b with ifuse).
void launch_ntt(const PolyBatch& b, const DevTables& t, uint32_t log_n, bool inverse, const NttSchedule& s,
                hipStream_t st, ProfHook* prof = nullptr, const NttEpilogue* epi = nullptr, uint32_t first = 0);

// ---- elementwise kernels (ckks.hip) --------------------------------------
// Signed integer polynomials x ([n_polys][N] int64, device) reduced into
// every limb of `out` (polynomial p from x + p N).
void launch_int_to_rns(const int64_t* x, const SmallBatch& out, const DevTables& t, uint32_t log_n, hipStream_t st);

// Limb-wise ops on NTT-domain data.  Operands share the shape of `out`; the
// modulus mapping is taken from `out`.
enum EwOp : uint32_t {
    EW_ADD = 0,         // out = a + b
    EW_SUB = 1,         // out = a - b
    EW_MUL = 2,         // out = a * b
    EW_MULADD = 3,      // out = a * b + c
    EW_NEG_MULADD = 4,  // out = -(a * b) + c
    EW_COPY = 5,        // out = a
};
void launch_ew(EwOp op, const SmallBatch& out, const SmallBatch& a, const SmallBatch* b, const SmallBatch* c,
               const DevTables& t, uint32_t log_n, hipStream_t st);
// Switching-key storage form, in place on the rows of `rows` (plain residues
// in): rows whose modulus is below 2^50 hold each residue as an
// integer-valued double (the inner product's fp64 products read it
// directly), the other rows residue * 2^64 mod m (Montgomery form: one REDC
// per 128-bit sum of products).  to_mont: [L+K] Shoup pairs of 2^64 mod m.
void launch_key_form(const SmallBatch& rows, const TwPair* to_mont, const DevTables& t, uint32_t log_n,
                     hipStream_t st);
// out = a * consts[limb] (Shoup pairs on the device)
void launch_mul_const(const SmallBatch& out, const SmallBatch& a, const TwPair* consts, const DevTables& t,
                      uint32_t log_n, hipStream_t st);

// ---- batched kernels: item z uses pointers [z] and workspace base + z*stride
struct WsRef {
    uint64_t* base;
    uint64_t stride;  // words
};
#define PFT_NO_OFFSET (~0ull)

// Per-target constants of the digit fold (sum_b 256^b Z_b mod m).
struct BconvRed {
    uint64_t m;
    uint64_t negm;  // 2^64 - m                      (m >= 2^50)
    uint64_t cq0;   // 2^30 m mod 2^64               (m >= 2^50)
    double md;      // m                             (m < 2^50)
    double minv;    // 1 / m
    double c32;     // 2^32 mod m                    (m < 2^50)
    double c32q;    // (2^32 mod m) / m              (m < 2^50)
    uint32_t fp;    // 1 when m < 2^50
    uint32_t pad;
};
static_assert(sizeof(BconvRed) == 64, "BconvRed is staged into LDS as 8 words");

struct KsConsts {
    const TwPair* modup_hatinv;   // [L][dnum][alpha]   indexed by (level-1, j, ii)
    const uint64_t* modup_c;      // [L][dnum][alpha][L+K] Montgomery form, row = target row
    const TwPair* down_phatinv;   // [K]
    const uint64_t* down_c;       // [K][L] Montgomery form
    const TwPair* down_pinv;      // [2L]: Shoup pairs, then fp64 pairs
    // MFMA base conversion: int8 digit operands, one 64-bit word per lane
    // ModUp:   [L][dnum][up_rt][up_kb][64]   (level-1, digit, row tile, k block, lane)
    // ModDown: [down_rt][down_kb][64]
    const uint64_t* up_aop;
    const uint64_t* down_aop;
    const BconvRed* red;          // [L+K] by modulus index
    uint32_t up_rt, up_kb, down_rt, down_kb;
    uint32_t L, K, dnum, alpha;
};

// d [3][level][N] at ws_z + off_d from ciphertexts a_z, b_z.
void launch_tensor_b(uint32_t n, const ItemPtrs& a, const ItemPtrs& b, WsRef ws, uint64_t off_d, uint32_t level,
                     const DevTables& t, uint32_t log_n, hipStream_t st);
void launch_copy_rows_b(uint32_t n, const ItemPtrs& src, uint64_t src_off, const ItemPtrs& dst, uint64_t dst_off,
                        uint32_t rows, uint32_t log_n, hipStream_t st);
// NTT-domain X -> X^kappa of `rows` rows of in_z into ws_z + off_out.
void launch_automorphism_b(uint32_t n, const ItemPtrs& in, uint32_t rows, WsRef ws, uint64_t off_out, uint64_t kappa,
                           uint32_t log_n, hipStream_t st);
// ModUp base conversion: d (coefficient form) -> ext [beta][level+K][N].
// mfma: the contraction on the matrix cores (int8 digits), else 128-bit VALU MACs.
void launch_modup_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level, const KsConsts& kc,
                    const DevTables& t, uint32_t log_n, bool mfma, hipStream_t st);
// ModUp on the matrix cores fused with the first pass of the forward
// transform (a radix-16 column pass, stages 0-3) of every converted row:
// ext holds the output of that pass; the transform continues at pass 1 of a
// schedule whose first radix is 4 (ntt.hip).  Needs log_n >= 8.  ifuse: d
// comes from an inverse transform of such a schedule that stopped before its
// final (radix-16 column) pass; the kernel applies that pass to its inputs.
void launch_modup_col_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level, const KsConsts& kc,
                        const DevTables& t, uint32_t log_n, bool ifuse, hipStream_t st);
// ModDown's conversion (conv_b = base conversion of the K special rows of
// acc_b to the q-limbs 0..level-1) fused the same way: conv holds the output
// of the first transform pass.
void launch_moddown_col_b(uint32_t n, WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                          const KsConsts& kc, const DevTables& t, uint32_t log_n, bool ifuse, hipStream_t st);
// RESCALE's expansion of last_z [2][N] into tmp_z [2][level-1][N] fused the
// same way: tmp holds the output of the first transform pass.
void launch_rescale_col_b(uint32_t n, WsRef ws, uint64_t off_last, uint64_t off_tmp, uint32_t level, uint32_t mode,
                          const DevTables& t, uint32_t log_n, hipStream_t st);
// The key inner product fused with the remaining (row) pass of the forward
// transform of ModUp's rows, for the items of a batch (ntt.hip): ext holds
// the rows after the first pass of a (4, log_n - 4) schedule (as
// launch_modup_col_b leaves them), d the NTT-domain input; writes
// acc [2][level+K][N].  Needs row_inner_supported(log_n) and at most 8
// digits; fp_rows[m] (host, by modulus index) is 1 where modulus m runs
// fp64 arithmetic (one launch per kind).  kappa != 0: d is not read; its
// own rows are the X -> X^kappa image of the rows of perm_src[z] (host
// array of n device pointers, item z's input polynomial [level][N], NTT
// domain), taken through the permutation as they are loaded.  pair_digits:
// the fp64 rows take two digits through each row pass together (same
// results).  prof: each launch (one per arithmetic kind) is timed as a
// PK_KEY_INNER variant 1024 + (log_n - 4) (+ 64 fp64 rows, + 128 digit pairs).
#define PFT_ROW_LIST 64
struct RowInner {
    uint64_t* base;  // item z's workspace at base + z stride
    uint64_t stride;
    uint64_t off_d, off_ext, off_acc;
    const uint64_t* key;  // [dnum][2][L+K][N] in the storage form of launch_key_form
    uint32_t n_items, level, rows, alpha, beta, L, krows, tiles;
    uint32_t n_rows;              // rows of this launch
    uint16_t row[PFT_ROW_LIST];   // their indices (0..level+K-1)
    const uint64_t* perm_src[PFT_MAX_ITEMS];
    uint64_t kappa, kappa_inv;
};
bool row_inner_supported(uint32_t log_n);
// at most 8 digits (ceil(level / alpha) <= 8; aborts otherwise).  rows:
// which rows this call launches, ROW_INNER_FP (those with q < 2^50),
// ROW_INNER_INT (the others) or both.
enum : uint32_t { ROW_INNER_INT = 1, ROW_INNER_FP = 2, ROW_INNER_ALL = 3 };
void launch_row_inner(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint64_t off_acc, const uint64_t* key,
                      uint32_t level, const KsConsts& kc, const DevTables& t, const uint32_t* fp_rows,
                      uint32_t log_n, const uint64_t* const* perm_src, uint64_t kappa, uint64_t kappa_inv,
                      bool pair_digits, hipStream_t st, ProfHook* prof = nullptr, uint32_t rows = ROW_INNER_ALL);
// acc [2][level+K][N] = sum_j x_j * key_j  (key: [dnum][2][L+K][N], Montgomery form)
void launch_key_inner_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint64_t off_acc, const uint64_t* key,
                        uint32_t level, const KsConsts& kc, const DevTables& t, uint32_t log_n, hipStream_t st);
// acc special rows (coefficient form) -> conv [2][level][N] (coefficient form)
void launch_moddown_conv_b(uint32_t n, WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                           const KsConsts& kc, const DevTables& t, uint32_t log_n, bool mfma, hipStream_t st);
// RESCALE pieces (see ckks.hip)
void launch_rescale_expand_b(uint32_t n, WsRef ws, uint64_t off_last, uint64_t off_tmp, uint32_t level, uint32_t mode,
                             const DevTables& t, uint32_t log_n, hipStream_t st);
// ws_z[off_out] = ws_z[off_a] + ws_z[off_b] over [2][level][N]
void launch_add_ct_b(uint32_t n, WsRef ws, uint64_t off_a, uint64_t off_b, uint64_t off_out, uint32_t level,
                     const DevTables& t, uint32_t log_n, hipStream_t st);
// PtMatVec inner sums of n_g <= pt_dot_multi_steps() giant steps (or
// outputs) at once: acc_{z,g} (at off_acc + g ct_words) = sum_j baby_{z,j} *
// pt_{g,j}, pt_{g,j} at pt + (g J + j) level N in Montgomery form; each
// baby_{z,j} is read once for all of them
uint32_t pt_dot_multi_steps();
void launch_pt_dot_multi_b(uint32_t n, WsRef ws, uint64_t off_baby, uint64_t ct_words, const uint64_t* pt, uint32_t J,
                           uint32_t n_g, uint64_t off_acc, uint32_t level, const DevTables& t, uint32_t log_n,
                           hipStream_t st);
// out_z = in_z * consts[z][limb] (integer constant polynomial)
void launch_scale_const_b(uint32_t n, const ItemPtrs& in, const ItemPtrs& out, const TwPair* consts, uint32_t level,
                          const DevTables& t, uint32_t log_n, hipStream_t st);
// out_z = (in_z.c0 + consts[z][limb].w, in_z.c1): HADDPLAIN of a constant
void launch_add_const_b(uint32_t n, const ItemPtrs& in, const ItemPtrs& out, const TwPair* consts, uint32_t level,
                        const DevTables& t, uint32_t log_n, hipStream_t st);
// Encrypted-weight products of n_g <= ct_dot_multi_steps() giant steps (n_g
// J <= PFT_MAX_ITEMS): for item z and giant step g, the HMUL tensor sum_j
// E_{g,j} (x) X_{z,j} into ws item g n + z at off_d as [3][level][N], with
// E_{g,j} = e.p[g J + j] (ciphertexts shared by all items, [2][level][N]) and
// X_{z,j} at xs_z + off_x + j ct_words; each X_{z,j} is read once for all of
// them.  to_mont: [L+K] 2^64 mod q as Shoup pairs.
uint32_t ct_dot_multi_steps();
void launch_ct_dot_multi_b(uint32_t n, const ItemPtrs& e, uint32_t J, uint32_t n_g, WsRef xs, uint64_t off_x,
                           uint64_t ct_words, WsRef ws, uint64_t off_d, uint32_t level, const TwPair* to_mont,
                           const DevTables& t, uint32_t log_n, hipStream_t st);

// The fixed scratch of the allocation-free entry point (noalloc.hip): a
// file-scope device array of PFT_NOALLOC_SCRATCH_BYTES per GPU.  Resolves
// (once per device, with `device` current) and returns its device address;
// 0 on success, -1 if the device is not current or the symbol lookup fails.
#define PFT_NOALLOC_SCRATCH_BYTES (64ull << 20)
#define PFT_NOALLOC_MAX_DEVICES 64
int noalloc_scratch_init(int device, uint64_t** out);

// Seeded draws (sampler.hip): Philox4x64-10 streams keyed by (k0, k1).
#define PFT_GAUSS_BOUND 19  // the discrete Gaussian's support is -19..19
struct SampleModuli {
    uint64_t q[64];  // modulus of output row i
};
struct GaussianCdt {
    uint64_t t[2 * PFT_GAUSS_BOUND];  // floor(2^64 F(k)), k = -B .. B-1
    uint32_t count;
};
// The thresholds of the discrete Gaussian of sigma 3.2; returns their count
// (2 PFT_GAUSS_BOUND) or -1 if capacity is too small.  Host only.
int gaussian_cdt_host(uint64_t* t, uint32_t capacity);
// out[i][j], i < rows, j < n: uniform residues mod mods.q[i]
void launch_sample_uniform(uint64_t k0, uint64_t k1, const SampleModuli& mods, uint32_t rows, uint64_t* out,
                           uint32_t n, hipStream_t st);
// out[j], j < n: kind 0 ternary, kind 1 discrete Gaussian
void launch_sample_small(uint32_t kind, uint64_t k0, uint64_t k1, const GaussianCdt& cdt, int64_t* out, uint32_t n,
                         hipStream_t st);
