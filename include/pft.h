/*
 * pft.h -- C ABI of libpft: RNS-CKKS primitives of PrivFT (arXiv:1908.06972)
 * as HIP kernels for AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every int-returning call returns PFT_OK (0) or a negative PFT_E*
 *   code; pft_last_error() then returns a message (thread-local, owned by
 *   the library, valid until the next failing call on that thread).
 * Ring: R_q = Z_q[X]/(X^N+1), N = 2^log_n, residues are uint64 < q < 2^60
 *   (Sec. 3.4, the CKKS levelled scheme).  The chain q_0 > q_1 > ... > q_{L-1}
 *   is strictly descending so that the prime dropped by RESCALE is the
 *   smallest (Sec. 5.1, the paragraph before Eq. (1)); K special primes
 *   p_0..p_{K-1} follow for key switching.
 * Level: a ciphertext at level l uses q_0..q_{l-1} (1 <= l <= L).
 * Device layout: a ciphertext is [2][level][N] uint64 in device memory, limb
 *   i of both polynomials reduced mod q_i, in the NTT domain: entry k of a
 *   limb holds the evaluation at psi^(2*brv(k)+1), psi the primitive 2N-th
 *   root g^((q-1)/2N) with g the smallest quadratic non-residue.  Host-side
 *   import/export and decrypt outputs use coefficient form.
 * Memory: ciphertext and plaintext storage is caller-owned device memory
 *   (e.g. torch tensors); the library never frees it.  Keys, tables and
 *   scratch are library-owned and freed with their context.
 * Streams: a context enqueues all work on the HIP stream given at creation;
 *   calls that return host data synchronize that stream.  A context is not
 *   thread-safe; use one per host thread/stream.
 * Randomness: KEYGEN and ENC either take their random polynomials as
 *   arguments (ternary secret, Gaussian errors, uniform masks) or, in the
 *   seeded entry points pft_keygen and pft_encrypt_seeded, draw them on the
 *   device from a counter-based generator keyed by a seed; either way results
 *   are a pure function of the inputs.
 */
#ifndef PFT_H
#define PFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PFT_OK = 0,
    PFT_EINVAL = -1,  /* bad pointer, size or shape */
    PFT_EPARAM = -2,  /* parameter set unsupported or primes not found */
    PFT_ELEVEL = -3,  /* level mismatch or level out of range */
    PFT_ESCALE = -4,  /* scales differ by more than 2^-40 (relative) */
    PFT_ENOKEY = -5,  /* missing public/relinearisation/rotation key */
    PFT_ENOMEM = -6,  /* device allocation failed */
    PFT_EHIP = -7     /* a HIP runtime call failed; message has the HIP error */
};

typedef struct pft_params pft_params; /* opaque, host */
typedef struct pft_ctx pft_ctx;       /* opaque, owns device tables and keys */

/* SETUP (Sec. 3.4; parameter guidance Sec. 6.4).  Primes are the largest
 * primes = 1 mod 2N of the given bit sizes: q_0 has q0_bits bits, q_1..q_{L-1}
 * the next L-1 largest with q_bits bits (descending), the K special primes
 * the largest unused with p_bits bits.  Bit sizes must be in 20..60.
 * 12 <= log_n <= 16, 1 <= n_q <= 64, 1 <= n_p <= 12, 1 <= dnum <= n_q,
 * alpha = ceil(n_q / dnum) <= 12.  rescale_mode: the mode RESCALE uses when
 * called with PFT_RESCALE_DEFAULT (0 rounds, the RESCALE of Sec. 3.4; 1
 * floors, Alg. 3 as printed).  PFT_EPARAM otherwise. */
typedef struct pft_param_spec {
    uint32_t log_n;
    uint32_t n_q;     /* L */
    uint32_t q0_bits;
    uint32_t q_bits;
    uint32_t n_p;     /* K */
    uint32_t p_bits;
    uint32_t dnum;    /* digits of hybrid key switching, alpha = ceil(L/dnum) */
    uint32_t rescale_mode;
    double scale;     /* default encoding scale Delta */
} pft_param_spec;

int pft_params_create(const pft_param_spec* spec, pft_params** out);
/* SETUP with the caller's prime chain (the moduli of Sec. 3.4 given
 * explicitly): q: host [n_q], the ciphertext primes, strictly descending
 * (RESCALE drops the last and smallest, Sec. 5.1); p: host [n_p], the
 * special primes.  Every modulus must be prime, = 1 mod 2N, in (2^20, 2^60)
 * and distinct from every other; PFT_EPARAM names the first that is not
 * (nothing is created).  Other fields and limits as pft_param_spec; the
 * arrays are copied. */
typedef struct pft_param_primes {
    uint32_t log_n;
    uint32_t n_q;
    const uint64_t* q;
    const uint64_t* p;
    uint32_t n_p;
    uint32_t dnum;
    uint32_t rescale_mode;
    uint32_t reserved;
    double scale;
} pft_param_primes;
int pft_params_create_primes(const pft_param_primes* spec, pft_params** out);
void pft_params_destroy(pft_params* params);
/* The parameter set's rescale_mode (host, *mode receives 0 or 1). */
int pft_params_rescale_mode(const pft_params* params, uint32_t* mode);
/* Copies q_0..q_{L-1} and p_0..p_{K-1} (host arrays of L and K entries). */
int pft_params_moduli(const pft_params* params, uint64_t* q, uint64_t* p);
/* N, L, K, dnum, alpha in that order (host array of 5). */
int pft_params_dims(const pft_params* params, uint32_t* dims);

const char* pft_last_error(void);

/* One context per device and stream.  stream may be NULL (the null stream).
 * Every call enqueues its work on that stream; within a call the library may
 * fork work onto a helper stream of its own (created with the context) and
 * always joins it back into the context stream before the call returns, so
 * the context stream's order (and a graph captured from it) covers it. */
int pft_ctx_create(const pft_params* params, int device, void* hip_stream, pft_ctx** out);
void pft_ctx_destroy(pft_ctx* ctx);
int pft_ctx_synchronize(pft_ctx* ctx);

/* Device memory of the library's own buffers (tables, keys, plaintext
 * matrices, per-operation scratch; never the caller's ciphertexts).
 * alloc/free: the caller's allocator (e.g. a framework's caching allocator),
 * both or neither (NULL: hipMalloc/hipFree); alloc(user, bytes, device)
 * returns device memory aligned to 256 bytes or NULL, free(user, ptr) takes
 * back what alloc returned; both are called on the host thread that calls
 * the library.  budget_bytes (0: none): an allocation that would take the
 * context's live bytes past it fails with PFT_ENOMEM, and so does the call
 * that needed it (an admission controller can size work by this).
 * pft_ctx_create_alloc: pft_ctx_create with that allocator and budget (NULL:
 * defaults); PFT_ENOMEM if the parameter set's tables already exceed it.
 * pft_ctx_set_budget changes the budget later (PFT_ENOMEM, unchanged, if the
 * context already holds more).  pft_ctx_memory writes {bytes of tables and
 * keys, bytes of scratch and other buffers, budget} to out[3]. */
typedef struct pft_allocator {
    void* (*alloc)(void* user, uint64_t bytes, int device);
    void (*free)(void* user, void* ptr);
    void* user;
    uint64_t budget_bytes;
} pft_allocator;
int pft_ctx_create_alloc(const pft_params* params, int device, void* hip_stream, const pft_allocator* alloc,
                         pft_ctx** out);
int pft_ctx_set_budget(pft_ctx* ctx, uint64_t budget_bytes);
int pft_ctx_memory(const pft_ctx* ctx, uint64_t* out);

/* ---- ciphertexts ------------------------------------------------------- */
typedef struct pft_ct {
    uint64_t* data;   /* device, >= 2*level*N uint64, layout [2][level][N], NTT domain */
    uint32_t level;
    uint32_t reserved;
    double scale;
} pft_ct;

/* Plaintext already in the NTT domain on the device: [level][N]. */
typedef struct pft_pt {
    uint64_t* data;
    uint32_t level;
    uint32_t reserved;
    double scale;
} pft_pt;

/* ---- KEYGEN (Sec. 3.4), randomness supplied by the caller (host memory) --
 * s: ternary secret, N int64 in {-1,0,1}.  Must be called first.  Setting a
 * secret (here or through pft_keygen) drops every key derived from an
 * earlier one -- public, relinearisation and rotation keys -- so until they
 * are generated again the calls that need them return PFT_ENOKEY.
 * Synchronizes the context stream. */
int pft_set_secret(pft_ctx* ctx, const int64_t* s);
/* Public key b = -a s + e over q_0..q_{L-1}.  a: [L][N] uniform residues in
 * coefficient form (a[i][k] < q_i); e: [N] small errors. */
int pft_gen_public_key(pft_ctx* ctx, const uint64_t* a, const int64_t* e);
/* Switching keys of hybrid key switching (the paper cites key switching for
 * relinearisation and rotation, Sec. 3.4 and its footnote).  For each digit
 * j < dnum: a[j]: [L+K][N] uniform residues in coefficient form (rows 0..L-1
 * mod q_i, rows L..L+K-1 mod p_k), e[j]: [N] errors.  The key is
 * b_j = -a_j s + e_j + [limb in digit j] (P mod q_limb) s' on all L+K limbs,
 * with s' = s^2 (relinearisation) or s(X^kappa), kappa = 5^step mod 2N
 * (rotation of the slots by `step` to the left).  Keys stay in device memory. */
int pft_gen_relin_key(pft_ctx* ctx, const uint64_t* a, const int64_t* e);
int pft_gen_rotation_key(pft_ctx* ctx, int32_t step, const uint64_t* a, const int64_t* e);
/* Rotation-key cache (keys beyond the HBM budget; Sec. 6.5 notes that at
 * logN = 16 the rotation keys were kept in host memory and migrated per
 * use).  max_resident = 0 (default): every rotation key stays in device
 * memory.  max_resident = k > 0: each rotation key generated afterwards
 * keeps a pinned host copy, and at most k keys occupy device slots; using a
 * non-resident key copies it into a slot on a copy stream of the library's
 * (the context stream waits for the copy through an event).  A slot is
 * refilled only after every stream that read it has reached the point where
 * the refill was decided (events; no device-wide synchronisation, so other
 * contexts' streams keep running).  Victim: the resident key whose next use
 * in the plan set by pft_key_cache_plan lies farthest ahead (keys the plan
 * does not use first; the optimal offline choice for a known order), or,
 * without a plan, the least recently used key.  With a plan, each rotation
 * also starts the copy of the plan's next key if it is not resident, so the
 * transfer overlaps the rotation.  Must be set before the first rotation
 * key is generated (PFT_EINVAL otherwise).  With a limited cache, rotations
 * are refused during graph capture (PFT_EINVAL: a replay would read
 * whatever key then occupies the slot).  The relinearisation key is never
 * cached.  pft_key_cache_stats writes {max_resident, slots allocated, hits,
 * misses, bytes copied to the device, keys copied ahead of use} to out[6]
 * (a use that finds its key resident is a hit, also after a copy ahead). */
/* The expected order of rotation steps, repeated cyclically (e.g. the
 * rotations of one inference): steps[n_steps] (host, copied), any sign, each
 * non-zero mod N/2 (PFT_EINVAL otherwise); n_steps = 0 clears the plan.  A
 * rotation by a step of the plan moves the plan position past its next
 * occurrence; steps outside the plan leave it.  Only affects which key is
 * evicted and copied ahead, never results. */
int pft_key_cache_plan(pft_ctx* ctx, const int32_t* steps, uint32_t n_steps);
/* Seeded KEYGEN (Sec. 3.4; X_key, the uniform masks and X_err of SETUP, sigma
 * = 3.2 from Sec. 6.4, CKKS parameter selection): the secret, public key, relinearisation key and one
 * rotation key per listed step, every draw taken on the device from the
 * Philox4x64-10 counter-based generator (Salmon et al., SC 2011).  Stream
 * key (seed, purpose 2^56 + key_id 2^8 + digit), counter (coefficient j,
 * limb i, 0, 0); purposes 1 secret, 2/3 public-key mask/error, 4/5
 * switching-key masks/errors (key_id 0 relinearisation, 1 + (step mod N/2)
 * rotation), 6/7/8 ENC v/e0/e1.  From a block's words w0, w1: ternary
 * (w0 mod 3) - 1; uniform floor((w1 2^64 + w0) q / 2^128); discrete Gaussian
 * -19 + #{k : T_k <= w0} with T from pft_gaussian_cdt.  The result equals the
 * caller-draws entry points above fed with the same draws.  A step that is 0
 * mod N/2 is refused (PFT_EINVAL) before any key changes.  Every key of an
 * earlier secret is dropped first (rotation keys for steps missing from
 * rot_steps then return PFT_ENOKEY); the key-cache setting applies as above.
 * Synchronizes the context stream. */
int pft_keygen(pft_ctx* ctx, uint64_t seed, const int32_t* rot_steps, uint32_t n_steps);
/* The 38 thresholds T_k = floor(2^64 F(k)), k = -19..18, of the cumulative
 * distribution F of the discrete Gaussian of sigma 3.2 on -19..19, in
 * increasing order.  Host only; table needs capacity >= 38 (PFT_EINVAL
 * otherwise); *count receives 38. */
int pft_gaussian_cdt(uint64_t* table, uint32_t capacity, uint32_t* count);
int pft_set_key_cache(pft_ctx* ctx, uint32_t max_resident);
int pft_key_cache_stats(const pft_ctx* ctx, uint64_t* out);
/* Number of device bytes held by keys and tables. */
int pft_ctx_device_bytes(const pft_ctx* ctx, uint64_t* bytes);

/* ---- ENC / DEC (Sec. 3.4) ---------------------------------------------
 * ENC of the integer plaintext m ([N] int64, host) at `level`:
 * (b v + e0 + m, a v + e1) with v ternary, e0/e1 errors ([N] int64, host).
 * out->data must be caller-allocated device memory of 2*level*N uint64;
 * the call sets out->level and out->scale. */
int pft_encrypt(pft_ctx* ctx, const int64_t* m, uint32_t level, double scale,
                const int64_t* v, const int64_t* e0, const int64_t* e1, pft_ct* out);
/* ENC with v, e0, e1 drawn on the device from the streams of `seed`
 * (purposes 6, 7, 8 of pft_keygen).  A seed must not be reused for two
 * encryptions under one key (the masks would repeat).  Synchronizes. */
int pft_encrypt_seeded(pft_ctx* ctx, const int64_t* m, uint32_t level, double scale, uint64_t seed, pft_ct* out);
/* DEC: c0 + c1 s mod q_i, written to host memory [level][N] in coefficient
 * form.  Synchronizes the context stream. */
int pft_decrypt(pft_ctx* ctx, const pft_ct* ct, uint64_t* out);
/* Coefficient-form transfer of a whole ciphertext, host [2][level][N].
 * export synchronizes; import sets ct->level/scale from the arguments. */
int pft_ct_export(pft_ctx* ctx, const pft_ct* ct, uint64_t* host);
int pft_ct_import(pft_ctx* ctx, const uint64_t* host, uint32_t level, double scale, pft_ct* ct);
/* Integer plaintext polynomial m ([N] int64, host) to an NTT-domain
 * plaintext at `level` (pt->data: caller device memory of level*N). */
int pft_pt_from_coeffs(pft_ctx* ctx, const int64_t* m, uint32_t level, double scale, pft_pt* pt);

/* ---- homomorphic operations (Sec. 3.4), all asynchronous ----------------
 * Batched forms take arrays of n descriptors; every element is independent.
 * Elements of equal level are processed together, up to 64 per launch, so
 * that one launch fills the GPU and reads each key once per batch.
 * out may alias an input for add, add_plain, mul_plain, mod_drop and
 * total_sum, not for mul_relin, rescale or rotate. */
int pft_add(pft_ctx* ctx, const pft_ct* a, const pft_ct* b, pft_ct* out);           /* HADD */
int pft_add_plain(pft_ctx* ctx, const pft_ct* a, const pft_pt* p, pft_ct* out);     /* HADDPLAIN */
int pft_mul_plain(pft_ctx* ctx, const pft_ct* a, const pft_pt* p, pft_ct* out);     /* HMULPLAIN */
/* HMUL followed by relinearisation (Table 2's HMUL+REL), no rescale. */
int pft_mul_relin(pft_ctx* ctx, const pft_ct* a, const pft_ct* b, pft_ct* out);
int pft_mul_relin_batch(pft_ctx* ctx, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out);
/* pft_mul_relin_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, with the key-switching
 * workspace in a fixed device scratch of 64 MiB per GPU (a file-scope device
 * array that each GPU holds until the process ends) instead of the
 * context's growable workspace.  No hipMalloc, hipFree or other allocation
 * happens in the call; the NTT autotuner is not run for new batch classes
 * (their default schedule is used; results do not depend on it).  Each
 * level group of the batch needs n_group * (3 level + level + beta (level +
 * K) + 2 (level + K) + 2 level) * N * 8 bytes, beta = ceil(level / alpha);
 * a batch with a group above 64 MiB is refused with PFT_ENOMEM before
 * anything is enqueued (e.g. one ciphertext at N = 2^15 and 16 limbs fits;
 * one at N = 2^16 and 24 limbs does not).  Calls on one GPU share its
 * scratch: calls that overlap in time on different streams of the same GPU
 * race and must be ordered by the caller.  The scratch needs no clearing
 * (every word a call reads it has written first).  PFT_EHIP if the scratch's
 * device address could not be resolved when the context was created. */
int pft_mul_relin_batch_noalloc(pft_ctx* ctx, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out);
/* RESCALE by q_{level-1} (Sec. 5.1, Eq. (1) and Alg. 3).  mode 0 rounds
 * (adds (q-1)/2 before the exact division, the RESCALE of Sec. 3.4), mode 1
 * floors (Alg. 3 as printed), PFT_RESCALE_DEFAULT takes the parameter set's
 * rescale_mode.  out->data needs 2*(level-1)*N uint64 and must
 * not alias in.  (Where the forward schedule starts with a radix-16 column
 * pass, the expansion of the last limb applies that pass itself.) */
#define PFT_RESCALE_DEFAULT 2u
int pft_rescale(pft_ctx* ctx, const pft_ct* in, uint32_t mode, pft_ct* out);
int pft_rescale_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, uint32_t mode, pft_ct* out);
/* Keep limbs 0..level-1 (exact).  out may alias in. */
int pft_mod_drop(pft_ctx* ctx, const pft_ct* in, uint32_t level, pft_ct* out);
/* ROTATE (Sec. 3.4): X -> X^kappa, kappa = 5^step mod 2N, then key switching
 * with the rotation key of `step` (PFT_ENOKEY if absent).  Slot j of the
 * result holds slot j+step of the input.  A step that is a multiple of N/2
 * leaves every slot in place (kappa = 1): out is a copy of in, no key is
 * needed or used. */
int pft_rotate(pft_ctx* ctx, const pft_ct* in, int32_t step, pft_ct* out);
int pft_rotate_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, int32_t step, pft_ct* out);
/* ROTATE by any step from power-of-two keys (the paper's cost model for
 * ROTATE, Sec. 6.5: one automorphism and key switch per set bit of the step,
 * so ROTATE_LHW is one key switch and ROTATE_HHW up to log2(N/2)): with
 * r = step mod N/2, for every set bit k of r in ascending order the
 * ciphertext is rotated by 2^k with the key for 2^k.  Same slots as a direct
 * rotation by step (the residues differ: different key switches).  in and out
 * may alias.  PFT_ENOKEY names the first missing power-of-two key. */
int pft_rotate_pow2(pft_ctx* ctx, const pft_ct* in, int32_t step, pft_ct* out);
int pft_rotate_pow2_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, int32_t step, pft_ct* out);
/* TotalSum (Sec. 4.1, Alg. 2): ct += ROTATE(ct, 2^i) for i < log2(n_slots);
 * needs the rotation keys 1, 2, 4, ..., n_slots/2.  out may alias in. */
int pft_total_sum(pft_ctx* ctx, const pft_ct* in, uint32_t n_slots, pft_ct* out);
int pft_total_sum_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, uint32_t n_slots, pft_ct* out);

/* ---- constant multiplication -------------------------------------------
 * out = in * m with the integer constant m = round(value * q_{level-1})
 * (half away from zero), i.e. HMULPLAIN by the constant plaintext whose
 * slots all equal `value` at scale q_{level-1}; out->scale = in->scale *
 * q_{level-1}, so a following RESCALE restores in->scale.  |value| < 4.
 * Used for the 1/w average of Sec. 4.1.  Synchronizes (per-call constants). */
int pft_mul_const(pft_ctx* ctx, const pft_ct* in, double value, pft_ct* out);
int pft_mul_const_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, const double* values, pft_ct* out);
/* HADDPLAIN of a constant (Sec. 3.4): out = in + m at X^0 with the integer
 * m = round(value * in->scale) (half away from zero), i.e. every slot gains
 * `value` at the ciphertext's own scale; out->scale = in->scale, level
 * unchanged.  PFT_EINVAL if |value * scale| >= 2^62.  out may alias in.
 * Used by the softmax approximation of Sec. 4.2.  Synchronizes (per-call
 * constants); not capturable. */
int pft_add_const(pft_ctx* ctx, const pft_ct* in, double value, pft_ct* out);
int pft_add_const_batch(pft_ctx* ctx, uint32_t n, const pft_ct* in, const double* values, pft_ct* out);

/* ---- PtMatVec: plaintext matrix x encrypted vector (Sec. 4.1, v H and h O)
 * Matrix M (n_o x n_in*n_i, row-major doubles) acting on an input split over
 * n_in ciphertexts (1 <= n_in <= 4096) whose t = N/2 slots hold a vector periodic with period
 * n_i (n_o | n_i | t, powers of two).  Diagonal method, baby-step/giant-step
 * form with b baby steps and G = n_o/b giant steps, b the power of two that
 * minimises the rotations n_in (b - 1) + (G - 1) of one product (the larger
 * b on ties; b = 2^ceil(log2(n_o)/2) for n_in = 1):
 *   D^c_i[k] = M[k mod n_o][c n_i + (k+i) mod n_i],   i = g b + r,
 *   P^c_{g,r} = D^c_{gb+r} rotated right by g b (pre-rotated, encoded at
 *               scale q_{level-1}),
 *   u = sum_g ROTATE(sum_c sum_r P^c_{g,r} * ROTATE(v_c, r), g b),
 *   y = u + ROTATE(u, n_o) + ... (steps n_o 2^s while n_o 2^s < n_i),
 * so slot k of y holds (M v)_{k mod n_o}.  Rotation keys for 1..b-1, g b and
 * n_o 2^s must exist.  No rescale: y->scale = v->scale * pt_scale.
 * pft_ptmat_create encodes the pre-rotated diagonals on the host (encoder of
 * pft_encode) at scale q_{level-1}; pft_ptmat_create_from_coeffs takes the
 * integer plaintexts P^c_{g,r} directly, layout [n_in][G][b][N] int64.
 * The matrix lives in device memory of its context until the context is
 * destroyed. */
typedef struct pft_ptmat pft_ptmat;
int pft_ptmat_create(pft_ctx* ctx, const double* M, uint32_t n_o, uint32_t n_i, uint32_t n_in, uint32_t level,
                     pft_ptmat** out);
int pft_ptmat_create_from_coeffs(pft_ctx* ctx, const int64_t* coeffs, uint32_t n_o, uint32_t n_i, uint32_t n_in,
                                 uint32_t level, double pt_scale, pft_ptmat** out);
/* Client side (host only): the integer plaintexts of the pre-rotated
 * diagonals P^c_{g,r} of M (same plan and layout as above), encoded with
 * pft_encode at `scale`, written to out [n_in][G][b][N] (caller memory).
 * Used to encrypt a model's diagonals for pft_ctmatvec (Sec. 4.2). */
int pft_diagonals_encode(const pft_params* params, const double* M, uint32_t n_o, uint32_t n_i, uint32_t n_in,
                         double scale, int64_t* out);
/* n_o, n_i, n_in, level, b, G (host array of 6). */
int pft_ptmat_info(const pft_ptmat* m, uint32_t* info);
void pft_ptmat_destroy(pft_ptmat* m);
/* in: n_docs * n_in ciphertexts, document-major, all at the matrix level;
 * out: n_docs ciphertexts (caller memory, 2*level*N each).  Scratch: the
 * context's auxiliary device buffer grows to n_docs (n_in b + G + 1)
 * ciphertexts at the matrix level (PFT_ENOMEM if it cannot, or if it would
 * have to grow during graph capture). */
int pft_ptmatvec(pft_ctx* ctx, const pft_ptmat* m, uint32_t n_docs, const pft_ct* in, pft_ct* out);

/* ---- plaintext dot products with TotalSum (Sec. 4.1, column packing) -----
 * The paper's own packing of the inference: H packed vertically (plaintext
 * H_{c,j} = rows c t .. c t + t - 1 of column j), one TotalSum per column
 * (Alg. 2), and O packed horizontally (plaintext O_j = row j of O in slots
 * 0 .. c-1).  A pft_ptdot holds n_out groups of J plaintexts P_{k,j}:
 *   out[z][k] = TotalSum_{n_sum}( sum_j in[z][j] * P_{k,j} )
 * (HMULPLAIN and HADD; TotalSum adds ROTATE by 1, 2, ..., n_sum/2, so with
 * n_sum = t every slot holds the sum over all slots; n_sum = 1: no
 * rotation).  Stage 1: n_out = n columns, J = ceil(m/t), n_sum = t; stage 2:
 * n_out = 1, J = n, n_sum = 1.
 * pft_ptdot_create encodes slot vectors [n_out][J][t] (doubles) with the
 * encoder of pft_encode at scale q_{level-1}; ..._from_coeffs takes integer
 * plaintexts [n_out][J][N] at pt_scale.  Device memory of the context,
 * freed with it.
 * pft_ptdot_apply: in n_docs * J ciphertexts (document-major) at the
 * plaintexts' level with equal scales; out n_docs * n_out ciphertexts
 * (caller memory); out scale = in scale * pt_scale, no rescale; needs the
 * rotation keys 1, 2, ..., n_sum/2.  PFT_EINVAL if n_sum is not a power of
 * two <= N/2. */
typedef struct pft_ptdot pft_ptdot;
int pft_ptdot_create(pft_ctx* ctx, const double* slots, uint32_t n_out, uint32_t J, uint32_t level,
                     pft_ptdot** out);
int pft_ptdot_create_from_coeffs(pft_ctx* ctx, const int64_t* coeffs, uint32_t n_out, uint32_t J, uint32_t level,
                                 double pt_scale, pft_ptdot** out);
void pft_ptdot_destroy(pft_ptdot* m);
int pft_ptdot_apply(pft_ctx* ctx, const pft_ptdot* m, uint32_t n_docs, const pft_ct* in, uint32_t n_sum,
                    pft_ct* out);

/* ---- CtMatVec: encrypted matrix x encrypted vector (Sec. 4.2) ------------
 * The predict step of training with encrypted weights: the PtMatVec above
 * with the pre-rotated diagonals E^c_{g,r} given as ciphertexts (so each
 * diagonal product is HMUL instead of HMULPLAIN):
 *   u = sum_g ROTATE(Relin(sum_c sum_r E^c_{g,r} (x) ROTATE(v_c, r)), g b),
 *   y = u + ROTATE(u, n_o) + ... (steps n_o 2^s while n_o 2^s < n_i),
 * where (x) is the HMUL tensor and the tensors of one giant step are summed
 * before a single relinearisation.  Same plan rule and rotation keys as
 * PtMatVec, plus the relinearisation key.  diags: n_in * G * b ciphertexts,
 * layout [n_in][G][b], all at one level and scale (the caller's encrypted
 * model, read only); in: n_docs * n_in ciphertexts, document-major, at the
 * diagonals' level and of equal scales; out: n_docs ciphertexts (caller
 * memory, 2*level*N each), out->scale = in scale * diagonal scale, no
 * rescale.  PFT_EINVAL if n_in * b > 64. */
int pft_ctmatvec(pft_ctx* ctx, uint32_t n_o, uint32_t n_i, uint32_t n_in, const pft_ct* diags, uint32_t n_docs,
                 const pft_ct* in, pft_ct* out);

/* ---- transforms on raw RNS polynomials ---------------------------------
 * data: device [n_polys][n_limbs][N], limb i of every polynomial mod q_i
 * (n_limbs <= L).  Forward maps coefficient form to the NTT domain of the
 * header comment, inverse maps back.  In place. */
int pft_ntt_forward(pft_ctx* ctx, uint64_t* data, uint32_t n_polys, uint32_t n_limbs);
int pft_ntt_inverse(pft_ctx* ctx, uint64_t* data, uint32_t n_polys, uint32_t n_limbs);

/* ---- NTT pass schedules (autotuner) --------------------------------------
 * A transform of length N = 2^log_n runs as one or two passes over windows of
 * consecutive stages.  A schedule crosses this boundary as four uint32 words:
 * the window sizes (radices, log2 of each window's stage count) in forward
 * order, zero-filled to three entries and summing to log_n, then a flags word
 * (bit 0: the last window's pass accesses the side of its data that is not
 * coalesced directly, 16 bytes per lane, instead of staging it through LDS;
 * bit 1: 8 residues per thread in 512-thread workgroups instead of 16 in 256,
 * for more waves in flight).
 * Every schedule computes the same transform bit for bit; the choice only
 * changes speed.
 * pft_ntt_candidates writes the candidates for the ring of p (default first)
 * as scheds[4 i .. 4 i + 3] for i < max_count and returns how many exist
 * (scheds may be NULL to count them).
 * pft_ntt_autotune(ctx, 1) (the default): the first transform of a direction
 * and batch-size class (up to 2^k limbs, k <= 10) times every candidate on
 * library-allocated scratch (zeroed, <= 2^10 limbs cycling through all
 * moduli) on the context stream and keeps the fastest; while a graph capture
 * is open the default schedule is used instead.  pft_ntt_autotune(ctx, 0)
 * forgets tuned choices and uses the default.  pft_ntt_set_schedule pins a
 * candidate (4 words) for one direction (inverse 0/1) and every batch size
 * (NULL unpins); PFT_EINVAL if it is not a candidate.  pft_ntt_get_schedule
 * writes the schedule a transform of n_limbs limbs would use (tuning first if
 * enabled). */
int pft_ntt_candidates(const pft_params* p, uint32_t* scheds, uint32_t max_count);
int pft_ntt_autotune(pft_ctx* ctx, int enable);
int pft_ntt_set_schedule(pft_ctx* ctx, int inverse, const uint32_t* sched);
int pft_ntt_get_schedule(pft_ctx* ctx, int inverse, uint64_t n_limbs, uint32_t* sched);
/* The tuned table as entries of six words (inverse 0/1, batch-size class
 * 0..10, or 32 + class for a choice restricted to schedules whose first
 * radix is 4 (made for the fused conversions), the four schedule words): export writes up to max_count entries and
 * returns how many exist; import validates every entry (PFT_EINVAL, nothing
 * changed) and then sets them, so a later run can reuse earlier choices. */
int pft_ntt_tuning_export(pft_ctx* ctx, uint32_t* entries, uint32_t max_count);
int pft_ntt_tuning_import(pft_ctx* ctx, const uint32_t* entries, uint32_t count);

/* ---- base conversion on the matrix cores ---------------------------------
 * The ModUp and ModDown base conversions (sums of alpha or K products of
 * residues below 2^60 by per-prime constants) run by default on MFMA: both
 * operands are split into signed base-256 digits, the int8 x int8 products
 * are summed exactly in int32 by v_mfma_i32_32x32x16_i8, and each target's
 * 8 digit sums are folded back into a residue on the VALU.  mode 0 selects the
 * 128-bit VALU multiply-accumulate kernels instead, 1 the matrix cores, 2 the
 * matrix cores with each conversion (ModUp and ModDown) fused
 * with the first pass of the forward transform of its output rows (used
 * where that transform's schedule starts with a radix-16 column pass and
 * N >= 256; otherwise as mode 1): each converted row is written once, already
 * through stages 0-3.  In mode 2 the inverse transform of the conversion's
 * inputs also stops before its final radix-16 column pass (its schedule is
 * then chosen among those ending with one) and the conversion applies that
 * pass while loading.  Mode 3 (the default) is mode 2 with the key inner
 * product fused into the remaining (row) pass of the forward transform of
 * ModUp's rows: where that transform's schedule is (4, log_n - 4), log_n in
 * {12, 13, 14, 16}, and at most 8 digits are active, one kernel takes each
 * extended row through its row pass and accumulates its products with the
 * key, so the extended digits are read once and only the accumulators are
 * written (otherwise as mode 2); its rows below 2^50 take two digits through
 * each row pass together (one twiddle load and one LDS barrier serve both).
 * Mode 4 is mode 3 with one digit per row pass.  The results are identical
 * in every mode.  PFT_EINVAL for any other mode. */
int pft_bconv_mode(pft_ctx* ctx, int mode);

/* ---- op-list executor ---------------------------------------------------
 * pft_exec_batch runs n_ops operations on the ciphertexts cts[0..n_cts) with
 * the result of issuing them one at a time, in list order, through the
 * single-op calls (bit for bit; the descriptors' level and scale of every
 * output are updated as those calls would).  op.a / op.b / op.out index cts:
 *   PFT_OP_NTT, PFT_OP_INTT   forward / inverse transform of both polynomials
 *                             of cts[a] in place (raw RNS polynomials, as
 *                             pft_ntt_forward/inverse); b, out unused
 *   PFT_OP_ADD                cts[out] = cts[a] + cts[b]            (pft_add)
 *   PFT_OP_MUL_RELIN          cts[out] = HMUL+relin(cts[a], cts[b]) (out distinct)
 *   PFT_OP_RESCALE            cts[out] = RESCALE(cts[a]), op.mode as pft_rescale
 *   PFT_OP_ROTATE             cts[out] = ROTATE(cts[a], op.step)    (out distinct)
 * Output buffers are caller-owned and sized for their level.  The list is
 * split into dependency waves (an op waits for every earlier op that writes
 * what it touches or reads what it writes); inside a wave, ops of equal kind,
 * input level and step/mode run as one batched call, and the groups of a wave
 * run concurrently on side streams forked from the context stream (joined
 * before the next wave), each with its own library workspace, so ciphertexts
 * of different levels share the device.  Captured between pft_graph_begin and
 * pft_graph_end, the list becomes one graph with a branch per group (run it
 * once eagerly first so the workspaces exist).  Errors: PFT_EINVAL (bad
 * index, kind, aliasing, timing enabled), PFT_ELEVEL (operand levels), any
 * error of the single-op calls; work of earlier waves may have been issued. */
enum { PFT_OP_NTT = 1, PFT_OP_INTT = 2, PFT_OP_ADD = 3, PFT_OP_MUL_RELIN = 4, PFT_OP_RESCALE = 5, PFT_OP_ROTATE = 6 };
typedef struct pft_op {
    uint32_t kind;
    uint32_t a, b, out;
    int32_t step;   /* PFT_OP_ROTATE */
    uint32_t mode;  /* PFT_OP_RESCALE */
} pft_op;
int pft_exec_batch(pft_ctx* ctx, pft_ct* cts, uint32_t n_cts, const pft_op* ops, uint32_t n_ops);
/* The plan pft_exec_batch would follow, on the host only: for input levels
 * levels[0..n_cts), writes each op's wave and its group index within the
 * wave (either array may be NULL) and returns the number of waves, or the
 * error pft_exec_batch would return for the list. */
int pft_exec_plan(const pft_op* ops, uint32_t n_ops, const uint32_t* levels, uint32_t n_cts, uint32_t* wave,
                  uint32_t* group);
/* The plan of PtMatVec (Sec. 4.1) as an op list another implementation can
 * replay: the operations pft_ptmatvec applies to one document, in its order,
 * over a register file of ciphertexts.  Registers 0..n_in-1 hold the inputs
 * v_c; the baby-step rotations of input c by r go to n_in + c (b - 1) + r - 1;
 * then come the registers PROD, ACC, TMP and TOT (next four indices), the
 * result is TOT (the out of the last op).  Kinds:
 *   PFT_OP_ROTATE     R[out] = ROTATE(R[a], step)
 *   PFT_OP_MUL_PLAIN  R[out] = HMULPLAIN(R[a], P_b), P_b the pre-rotated
 *                     diagonal b of the [n_in][G][b] layout above
 *   PFT_OP_ADD        R[out] = R[a] + R[b]
 * (the plan's own kinds: pft_exec_batch does not take PFT_OP_MUL_PLAIN).
 * pft_ptmat_plan: for the shape alone (host only; PFT_EINVAL unless n_o and
 * n_i are powers of two with n_o <= n_i and 1 <= n_in <= 4096).
 * pft_ptmat_plan_export: for a matrix, and (diag_coeffs not NULL) its
 * integer plaintexts P_b, [n_in][G][b][N] int64, as pft_ptmatvec multiplies
 * by them (times q_{level-1} scale, see pft_ptmat_create).
 * Both write min(max_ops, count) ops (ops may be NULL) and the count to
 * *n_ops. */
enum { PFT_OP_MUL_PLAIN = 7 };
int pft_ptmat_plan(uint32_t n_o, uint32_t n_i, uint32_t n_in, pft_op* ops, uint32_t max_ops, uint32_t* n_ops);
int pft_ptmat_plan_export(const pft_ptmat* m, pft_op* ops, uint32_t max_ops, uint32_t* n_ops, int64_t* diag_coeffs);

/* ---- HIP graphs ----------------------------------------------------------
 * pft_graph_begin starts a capture on the context stream (which must not be
 * the null stream); every following call on the context is recorded instead
 * of run, until pft_graph_end, which instantiates the graph.  pft_graph_launch
 * replays it on the context stream: same kernels, same device buffers (the
 * descriptors' data pointers and levels are baked in).  Calls that move host
 * data, synchronize, or would grow the library scratch fail with PFT_EINVAL /
 * PFT_ENOMEM while a capture is open; pft_ctx_reserve sizes the scratch
 * (bytes of the per-operation workspace and of the composite-operation
 * buffers) beforehand.  A graph must be destroyed before its context. */
typedef struct pft_graph pft_graph;
int pft_ctx_reserve(pft_ctx* ctx, uint64_t ws_bytes, uint64_t aux_bytes);
int pft_graph_begin(pft_ctx* ctx);
int pft_graph_end(pft_ctx* ctx, pft_graph** out);
int pft_graph_launch(pft_ctx* ctx, pft_graph* graph);
void pft_graph_destroy(pft_graph* graph);

/* ---- per-kernel timing ------------------------------------------------
 * pft_prof_enable brackets every launch of the selected kernel families
 * (bit k of mask = family k; 0 turns timing off) with HIP events recorded on
 * the context stream, and clears previous records.  pft_prof_read
 * synchronizes and returns, for family `kid`, the summed event time, the
 * number of launches, and the summed algorithmic HBM bytes and algorithmic
 * operations (butterflies for the transforms, 64-bit modular multiply-adds
 * otherwise) of those launches.  Algorithmic bytes are the method's: the
 * operands a launch reads and the results it writes, 8 bytes per residue;
 * the words a transform leaves between two of its passes are the layout's
 * cost and are not counted (a pass that neither starts nor ends its
 * transform counts none).  Families: 0 forward NTT pass, 1 inverse NTT
 * pass, 2 ModUp base conversion, 3 key inner product, 4 ModDown base
 * conversion, 5 ModDown final scaling (kept as an index; it now runs as
 * the epilogue of the forward NTT pass that produces it, family 0), 6 HMUL
 * tensor, 7 automorphism, 8 rescale (the spreading of the last limb; the
 * final scaling runs as the epilogue of the forward NTT pass, family 0),
 * 9 other elementwise. */
int pft_prof_enable(pft_ctx* ctx, uint32_t mask);
int pft_prof_read(pft_ctx* ctx, uint32_t kid, double* total_ms, uint64_t* launches, double* bytes, double* ops);
/* Per-instantiation totals of family kid since pft_prof_enable, largest total
 * time first: up to max_count entries of (variant, ms, launches, algorithmic
 * bytes, ops); returns the number of distinct variants.  variant 0: the
 * family's single kernel; NTT passes (families 0 and 1): 1 + (radix | 32 if a
 * column pass | 64 if the transform's final pass | 128 if staged | 256 if 8
 * residues per thread | 512 if the pass finishes ModDown | 1024 if X^kappa
 * is folded into it), naming k_ntt_pass<radix, log2 residues per thread,
 * inverse, column, final, staged, ModDown epilogue[, true]>; base
 * conversions on the matrix cores (families 2 and 4): the number of 16-deep
 * k-blocks, naming k_modup_mfma_b<kb> and k_moddown_mfma_b<kb>, or 64 + kb
 * (+ 16 with the inverse pass folded in) for the conversions fused with
 * transform passes, naming k_bconv_col_b<kb, ModDown, inverse pass>; the key
 * inner product (family 3): the number of digits beta, naming
 * k_key_inner_items<beta>, or 1024 + the radix of the row pass it is fused
 * with, naming k_row_inner<radix, 3>.  Any output may be NULL. */
int pft_prof_read_variants(pft_ctx* ctx, uint32_t kid, uint32_t max_count, uint32_t* variants, double* total_ms,
                           uint64_t* launches, double* bytes, double* ops);

/* ---- client-side ENCODE / DECODE on the host (Sec. 3.4; CPU per Sec. 5.1)
 * encode: slots z_j = re[j] + i im[j], j < n_slots <= N/2, to the integer
 * polynomial round((2 scale/N) Re sum_j z_j zeta^(-(5^j) k)), zeta = e^{i pi/N};
 * PFT_EINVAL if a coefficient would exceed 2^62 in magnitude.
 * decode: residues [level][N] (coefficient form, e.g. from pft_decrypt),
 * centred CRT lift, then z_j = (1/scale) sum_k mu_k zeta^((5^j) k). */
int pft_encode(const pft_params* params, const double* re, const double* im, uint32_t n_slots,
               double scale, int64_t* out);
int pft_decode(const pft_params* params, const uint64_t* residues, uint32_t level, double scale,
               uint32_t n_slots, double* re, double* im);

#ifdef __cplusplus
}
#endif
#endif /* PFT_H */
