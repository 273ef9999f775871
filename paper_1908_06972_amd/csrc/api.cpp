// api.cpp -- the extern "C" boundary of libpft (declared in include/pft.h):
// parameter setup, device tables, key generation, encryption, and the
// homomorphic operations as sequences of HIP kernel launches on the
// context's stream.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/pft.h"
#include "host_math.h"
#include "pft_kernels.h"

using namespace pft;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCK(expr)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(PFT_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

extern "C" const char* pft_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// parameters (SETUP, Sec. 3.4)
// ---------------------------------------------------------------------------
struct pft_params {
    uint32_t log_n, n, L, K, dnum, alpha;
    uint32_t rescale_mode = 0;  // mode of pft_rescale's PFT_RESCALE_DEFAULT
    double scale;
    std::vector<uint64_t> q, p, mods;  // mods = q then p
    std::vector<uint64_t> psi;         // per modulus
};

static bool largest_primes(uint64_t two_n, uint32_t bits, uint32_t count, const std::vector<uint64_t>& exclude,
                           std::vector<uint64_t>& out) {
    uint64_t top = (bits >= 64) ? ~0ull : ((1ull << bits) - 1);
    uint64_t k = (top - 1) / two_n;
    uint64_t lo = 1ull << (bits - 1);
    while (count) {
        if (k == 0) return false;
        uint64_t c = k * two_n + 1;
        if (c < lo) return false;
        if (std::find(exclude.begin(), exclude.end(), c) == exclude.end() &&
            std::find(out.begin(), out.end(), c) == out.end() && is_prime_u64(c)) {
            out.push_back(c);
            --count;
        }
        --k;
    }
    return true;
}

static uint64_t primitive_2n_root(uint64_t q, uint64_t n) {
    uint64_t g = 2;
    while (powmod(g, (q - 1) / 2, q) != q - 1) ++g;  // smallest quadratic non-residue
    return powmod(g, (q - 1) / (2 * n), q);
}

// Limits shared by both forms of SETUP.
static int check_shape(uint32_t log_n, uint32_t n_q, uint32_t n_p, uint32_t dnum, uint32_t rescale_mode) {
    if (!ntt_supported(log_n)) return fail(PFT_EPARAM, "log_n %u unsupported (12..16)", log_n);
    if (n_q < 1 || n_q > 64) return fail(PFT_EPARAM, "n_q must be in 1..64");
    if (n_p < 1 || n_p > 12) return fail(PFT_EPARAM, "n_p must be in 1..12");
    if (dnum < 1 || dnum > n_q) return fail(PFT_EPARAM, "dnum must be in 1..n_q");
    if ((n_q + dnum - 1) / dnum > 12) return fail(PFT_EPARAM, "alpha = ceil(L/dnum) must be <= 12");
    if ((n_q + n_p) * 2 > 128) return fail(PFT_EPARAM, "too many primes");
    if (rescale_mode > 1) return fail(PFT_EPARAM, "rescale_mode must be 0 (round) or 1 (floor)");
    return PFT_OK;
}

// The rest of SETUP once the primes are fixed: moduli list and roots.
static pft_params* finish_params(pft_params* P) {
    P->mods = P->q;
    P->mods.insert(P->mods.end(), P->p.begin(), P->p.end());
    for (uint64_t m : P->mods) P->psi.push_back(primitive_2n_root(m, P->n));
    return P;
}

extern "C" int pft_params_create_primes(const pft_param_primes* s, pft_params** out) {
    if (!s || !out || !s->q || !s->p) return fail(PFT_EINVAL, "null argument");
    int r;
    if ((r = check_shape(s->log_n, s->n_q, s->n_p, s->dnum, s->rescale_mode))) return r;
    const uint64_t two_n = 2ull << s->log_n;
    std::vector<uint64_t> all;
    for (uint32_t i = 0; i < s->n_q + s->n_p; ++i) {
        const bool is_q = i < s->n_q;
        const uint64_t m = is_q ? s->q[i] : s->p[i - s->n_q];
        const char* kind = is_q ? "q" : "p";
        const uint32_t idx = is_q ? i : i - s->n_q;
        if (m <= (1ull << 20) || m >= (1ull << 60))
            return fail(PFT_EPARAM, "%s[%u] = %llu is not in (2^20, 2^60)", kind, idx, (unsigned long long)m);
        if (m % two_n != 1) return fail(PFT_EPARAM, "%s[%u] = %llu is not 1 mod 2N", kind, idx, (unsigned long long)m);
        if (!is_prime_u64(m)) return fail(PFT_EPARAM, "%s[%u] = %llu is not prime", kind, idx, (unsigned long long)m);
        if (std::find(all.begin(), all.end(), m) != all.end())
            return fail(PFT_EPARAM, "%s[%u] = %llu appears twice", kind, idx, (unsigned long long)m);
        if (is_q && i > 0 && !(s->q[i - 1] > m))
            return fail(PFT_EPARAM, "q must be strictly descending (q[%u] <= q[%u])", i - 1, i);
        all.push_back(m);
    }
    auto* P = new pft_params();
    P->log_n = s->log_n;
    P->n = 1u << s->log_n;
    P->L = s->n_q;
    P->K = s->n_p;
    P->dnum = s->dnum;
    P->alpha = (s->n_q + s->dnum - 1) / s->dnum;
    P->rescale_mode = s->rescale_mode;
    P->scale = s->scale;
    P->q.assign(s->q, s->q + s->n_q);
    P->p.assign(s->p, s->p + s->n_p);
    *out = finish_params(P);
    return PFT_OK;
}

extern "C" int pft_params_create(const pft_param_spec* s, pft_params** out) {
    if (!s || !out) return fail(PFT_EINVAL, "null argument");
    int r0;
    if ((r0 = check_shape(s->log_n, s->n_q, s->n_p, s->dnum, s->rescale_mode))) return r0;
    uint32_t alpha = (s->n_q + s->dnum - 1) / s->dnum;
    for (uint32_t b : {s->q0_bits, s->q_bits, s->p_bits})
        if (b < 20 || b > 60) return fail(PFT_EPARAM, "prime bit sizes must be in 20..60");
    if (s->q0_bits < s->q_bits) return fail(PFT_EPARAM, "q0_bits must be >= q_bits (descending chain)");
    auto* P = new pft_params();
    P->log_n = s->log_n;
    P->n = 1u << s->log_n;
    P->L = s->n_q;
    P->K = s->n_p;
    P->dnum = s->dnum;
    P->alpha = alpha;
    P->rescale_mode = s->rescale_mode;
    P->scale = s->scale;
    const uint64_t two_n = 2ull * P->n;
    std::vector<uint64_t> none;
    if (!largest_primes(two_n, s->q0_bits, 1, none, P->q) ||
        !largest_primes(two_n, s->q_bits, s->n_q - 1, P->q, P->q) ||
        !largest_primes(two_n, s->p_bits, s->n_p, P->q, P->p)) {
        delete P;
        return fail(PFT_EPARAM, "not enough primes = 1 mod 2N of the requested sizes");
    }
    for (uint32_t i = 1; i < P->L; ++i)
        if (!(P->q[i - 1] > P->q[i])) {
            delete P;
            return fail(PFT_EPARAM, "prime chain is not strictly descending");
        }
    *out = finish_params(P);
    return PFT_OK;
}

extern "C" void pft_params_destroy(pft_params* P) { delete P; }

extern "C" int pft_params_rescale_mode(const pft_params* P, uint32_t* mode) {
    if (!P || !mode) return fail(PFT_EINVAL, "null argument");
    *mode = P->rescale_mode;
    return PFT_OK;
}

extern "C" int pft_params_moduli(const pft_params* P, uint64_t* q, uint64_t* p) {
    if (!P || !q || !p) return fail(PFT_EINVAL, "null argument");
    memcpy(q, P->q.data(), P->L * 8);
    memcpy(p, P->p.data(), P->K * 8);
    return PFT_OK;
}

extern "C" int pft_params_dims(const pft_params* P, uint32_t* d) {
    if (!P || !d) return fail(PFT_EINVAL, "null argument");
    d[0] = P->n;
    d[1] = P->L;
    d[2] = P->K;
    d[3] = P->dnum;
    d[4] = P->alpha;
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// context: device tables, keys, scratch
// ---------------------------------------------------------------------------
struct SwitchKeyDev {
    uint64_t* data = nullptr;  // [dnum][2][L+K][N], NTT domain, times 2^64 mod m
    // rotation keys under a limited key cache: pinned host copy, and the
    // cache slot that holds data while the key is resident
    uint64_t* host = nullptr;
    int slot = -1;
    uint64_t last_use = 0;
};

// HIP-event bracketing of kernel families on the context stream.  The
// events only time work and are read after a stream synchronisation, so they
// skip the system-scope fence (a cache writeback and invalidation each time
// one is recorded) that the default event performs.
struct EventProf : ProfHook {
    hipStream_t st = nullptr;
    uint32_t mask = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec {
        int kid;
        uint32_t variant;
        hipEvent_t a, b;
        double bytes, ops;
    };
    std::vector<Rec> recs;
    hipEvent_t open[PK_COUNT] = {};
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    bool on(int kid) const { return (mask >> kid) & 1u; }
    void begin(int kid, hipStream_t s) override {
        if (!on(kid)) return;
        open[kid] = get();
        if (open[kid]) (void)hipEventRecord(open[kid], s ? s : st);
    }
    void end(int kid, double bytes, double ops, uint32_t variant, hipStream_t s) override {
        if (!on(kid) || !open[kid]) return;
        hipEvent_t b = get();
        if (!b) return;
        (void)hipEventRecord(b, s ? s : st);
        recs.push_back(Rec{kid, variant, open[kid], b, bytes, ops});
        open[kid] = nullptr;
    }
    void reset() {
        recs.clear();
        used = 0;
    }
    ~EventProf() override {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct pft_ctx {
    EventProf prof;
    const pft_params* P = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    DevTables tabs{};
    KsConsts kc{};
    TwPair* rescale_qinv = nullptr;  // [2][L][L]: row l-1 holds q_{l-1}^-1 mod q_k (Shoup pairs, then fp64 pairs)
    TwPair* gadget = nullptr;        // [L]: (P mod q_i) as Shoup pairs
    TwPair* to_mont = nullptr;       // [L+K]: 2^64 mod m as Shoup pairs
    std::vector<void*> allocs;
    uint64_t device_bytes = 0;
    uint64_t* s = nullptr;        // [L+K][N] secret, NTT domain
    uint64_t* s_prime = nullptr;  // [L+K][N] scratch for s^2 / s(X^kappa) during key generation
    uint64_t* pk = nullptr;  // [2][L][N] (b, a), NTT domain
    SwitchKeyDev rlk;
    // pk and rlk hold keys of the current secret (false after the secret
    // changed and until they are generated again)
    bool pk_ok = false, rlk_ok = false;
    std::vector<uint64_t*> key_pool;  // device memory of dropped switching keys, reused by new ones
    std::map<int32_t, SwitchKeyDev> rot;  // keyed by step mod N/2
    // rotation-key cache (0 = every key resident): at most rot_cache_max keys
    // in device slots, all keys in pinned host memory.  A slot is refilled
    // only after every stream that read it has passed that point (events, no
    // device-wide synchronisation); keys are copied in on a copy stream of
    // their own.  Victim: the resident key whose next use in the caller's
    // cyclic plan lies farthest ahead (keys outside the plan first), else
    // the least recently used.  With a plan, the next key of the plan is
    // copied in while the current rotation runs.
    uint32_t rot_cache_max = 0;
    std::vector<uint64_t*> rot_slots;
    std::vector<int32_t> rot_slot_owner;  // normalised step, or -1
    struct SlotSync {
        std::vector<hipStream_t> readers;  // streams with queued reads since the last fill
        hipEvent_t ready = nullptr;        // recorded on the copy stream after the last fill
        bool ready_pending = false;        // a copy-stream fill the readers must still wait for
    };
    std::vector<SlotSync> rot_sync;
    std::map<hipStream_t, hipEvent_t> stream_ev;  // one event per stream, recorded at each slot refill
    hipStream_t copy_st = nullptr;
    std::vector<int32_t> rot_plan;  // normalised steps, cyclic
    size_t rot_plan_pos = 0;
    uint64_t rot_clock = 0, rot_hits = 0, rot_misses = 0, rot_bytes_in = 0, rot_prefetches = 0;
    uint64_t* scratch = nullptr;  // this device's fixed scratch (noalloc.hip), resolved at creation
    uint64_t* ws = nullptr;  // scratch of one operation (key switching etc.)
    size_t ws_bytes = 0;
    uint64_t* aux = nullptr;  // buffers of composite operations (PtMatVec) that call other operations
    size_t aux_bytes = 0;
    TwPair* cbuf = nullptr;  // per-call constants (e.g. 1/w per document)
    size_t cbuf_n = 0;
    bool capturing = false;  // a HIP graph capture is open on the stream
    int live_graphs = 0;     // graphs may reference ws/aux: grow by retiring, never free
    std::vector<void*> retired;
    // NTT pass schedules: pinned per direction, else tuned per (direction,
    // batch-size class) on first use when ntt_tune is set
    bool bconv_mfma = true;  // base conversions on the matrix cores
    bool bconv_fuse = true;  // conversions fused with the adjacent transform passes (MFMA only)
    bool inner_fuse = true;  // key inner product fused with the row pass of ModUp's rows (needs bconv_fuse)
    bool inner_pairs = true;  // the fused inner product takes two digits through each row pass
    std::vector<uint32_t> fp_rows;  // [L+K]: 1 where the modulus runs fp64 arithmetic (below 2^50)
    bool ntt_tune = true;
    NttSchedule ntt_pinned[2] = {};
    std::map<uint32_t, NttSchedule> ntt_tuned;
    // the stream the context was created with, and a helper stream beside
    // it: the fused inner product's 60-bit rows run there concurrently with
    // its fp64 rows (forked from and joined back into the context stream)
    hipStream_t home = nullptr;
    hipStream_t inner_st = nullptr;
    hipEvent_t inner_fork = nullptr, inner_join = nullptr;
    // op-list executor: side streams and their workspaces (branch k > 0;
    // branch 0 is the context stream with ws)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_ev;
    std::vector<std::pair<uint64_t*, size_t>> side_ws;
    // device memory of the library's own buffers: the caller's allocator (or
    // hipMalloc/hipFree), the bytes of every live allocation, and the budget
    // (0: none) that new allocations must fit under
    pft_allocator alloc{};
    std::unordered_map<void*, size_t> live;
    uint64_t live_bytes = 0;
};

// Every device allocation of the library goes through here: refused with
// PFT_ENOMEM (and a message naming `what`) if it would take the context's
// live bytes past its budget or if the allocator fails.
static int dev_alloc(pft_ctx* c, void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (c->alloc.budget_bytes && c->live_bytes + bytes > c->alloc.budget_bytes)
        return fail(PFT_ENOMEM, "%s of %zu bytes exceeds the context's device-memory budget (%llu of %llu bytes in use)",
                    what, bytes, (unsigned long long)c->live_bytes, (unsigned long long)c->alloc.budget_bytes);
    if (c->alloc.alloc) {
        *p = c->alloc.alloc(c->alloc.user, bytes, c->device);
        if (!*p) return fail(PFT_ENOMEM, "%s: the caller's allocator returned no memory for %zu bytes", what, bytes);
    } else {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            return fail(PFT_ENOMEM, "%s: hipMalloc(%zu): %s", what, bytes, hipGetErrorString(e));
        }
    }
    c->live[*p] = bytes;
    c->live_bytes += bytes;
    return PFT_OK;
}

static void dev_free(pft_ctx* c, void* p) {
    if (!p) return;
    auto it = c->live.find(p);
    if (it != c->live.end()) {
        c->live_bytes -= it->second;
        c->live.erase(it);
    }
    if (c->alloc.free)
        c->alloc.free(c->alloc.user, p);
    else
        (void)hipFree(p);
}

template <typename T>
static int dalloc(pft_ctx* c, T** p, size_t bytes) {
    void* v = nullptr;
    int r = dev_alloc(c, &v, bytes, "table or key storage");
    if (r) return r;
    c->allocs.push_back(v);
    c->device_bytes += bytes;
    *p = (T*)v;
    return PFT_OK;
}

template <typename T>
static int upload(pft_ctx* c, T** dst, const std::vector<T>& src) {
    int r = dalloc(c, dst, src.size() * sizeof(T));
    if (r) return r;
    HIPCK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return PFT_OK;
}

static int ensure_ws(pft_ctx* c, size_t bytes) {
    if (c->ws_bytes >= bytes) return PFT_OK;
    if (c->capturing)
        return fail(PFT_ENOMEM, "workspace of %zu bytes needed during graph capture; call pft_ctx_reserve first",
                    bytes);
    if (c->ws) {
        HIPCK(hipStreamSynchronize(c->stream));
        if (c->live_graphs)
            c->retired.push_back(c->ws);
        else
            dev_free(c, c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    void* v = nullptr;
    int r = dev_alloc(c, &v, bytes, "workspace");
    if (r) return r;
    c->ws = (uint64_t*)v;
    c->ws_bytes = bytes;
    return PFT_OK;
}

static int ensure_aux(pft_ctx* c, size_t bytes) {
    if (c->aux_bytes >= bytes) return PFT_OK;
    if (c->capturing)
        return fail(PFT_ENOMEM, "aux buffer of %zu bytes needed during graph capture; call pft_ctx_reserve first",
                    bytes);
    if (c->aux) {
        HIPCK(hipStreamSynchronize(c->stream));
        if (c->live_graphs)
            c->retired.push_back(c->aux);
        else
            dev_free(c, c->aux);
        c->aux = nullptr;
        c->aux_bytes = 0;
    }
    void* v = nullptr;
    int r = dev_alloc(c, &v, bytes, "aux buffer");
    if (r) return r;
    c->aux = (uint64_t*)v;
    c->aux_bytes = bytes;
    return PFT_OK;
}

// Limbs whose NTT runs in fp64 (exact for q < 2^50).
static bool ntt_fp(uint64_t q) { return bit_length(q) <= 50; }
static uint64_t dbits(double v) {
    uint64_t u;
    memcpy(&u, &v, sizeof u);
    return u;
}
static TwPair pair(uint64_t w, uint64_t q) { return TwPair{w, shoup_companion(w, q)}; }
// NTT twiddle in the form the limb's butterflies use.
static TwPair twiddle(uint64_t w, uint64_t q) {
    if (ntt_fp(q)) return TwPair{dbits((double)w), dbits((double)w / (double)q)};
    return pair(w, q);
}

static int build_tables(pft_ctx* c) {
    const pft_params* P = c->P;
    const uint32_t n = P->n, lg = P->log_n, M = P->L + P->K;
    std::vector<DevMod> mods(M);
    std::vector<TwPair> fw((size_t)M * n), iw((size_t)M * n);
    std::vector<uint64_t> pw(n), ipw(n);
    for (uint32_t m = 0; m < M; ++m) {
        const uint64_t q = P->mods[m], psi = P->psi[m], psi_inv = invmod(psi, q);
        pw[0] = ipw[0] = 1;
        for (uint32_t j = 1; j < n; ++j) {
            pw[j] = mulmod(pw[j - 1], psi, q);
            ipw[j] = mulmod(ipw[j - 1], psi_inv, q);
        }
        for (uint32_t k = 0; k < n; ++k) {
            const uint32_t r = bitrev(k, lg);
            fw[(size_t)m * n + k] = twiddle(pw[r], q);
            iw[(size_t)m * n + k] = twiddle(ipw[r], q);
        }
        DevMod& d = mods[m];
        d.q = q;
        d.two_q = 2 * q;
        d.bits = bit_length(q);
        d.mu = (uint64_t)(((u128)1 << (2 * d.bits)) / q);
        uint64_t inv = 1;  // q^-1 mod 2^64 by Newton iteration
        for (int i = 0; i < 7; ++i) inv *= 2 - q * inv;
        d.mont_neg_qinv = 0 - inv;
        d.n_inv = invmod(n % q, q);
        d.n_inv_sh = shoup_companion(d.n_inv, q);
        d.last_inv = mulmod(ipw[n / 2], d.n_inv, q);  // psi^-brv(1) = psi^-(N/2)
        d.last_inv_sh = shoup_companion(d.last_inv, q);
        d.fp = ntt_fp(q) ? 1u : 0u;
        d.qd = (double)q;
        d.qinv = 1.0 / (double)q;
        d.n_inv_d = (double)d.n_inv;
        d.n_inv_q = (double)d.n_inv / (double)q;
        d.last_inv_d = (double)d.last_inv;
        d.last_inv_q = (double)d.last_inv / (double)q;
    }
    int r;
    if ((r = upload(c, &c->tabs.mods, mods)) || (r = upload(c, &c->tabs.tw_fwd, fw)) ||
        (r = upload(c, &c->tabs.tw_inv, iw)))
        return r;

    // ---- hybrid key switching constants
    const uint32_t L = P->L, K = P->K, dnum = P->dnum, A = P->alpha;
    std::vector<TwPair> hatinv((size_t)L * dnum * A, TwPair{0, 0});
    std::vector<uint64_t> cmat((size_t)L * dnum * A * (L + K), 0);
    for (uint32_t lvl = 1; lvl <= L; ++lvl) {
        const uint32_t beta = (lvl + A - 1) / A;
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t i0 = j * A, i1 = std::min(i0 + A, lvl);
            for (uint32_t i = i0; i < i1; ++i) {
                const size_t ci = ((size_t)(lvl - 1) * dnum + j) * A + (i - i0);
                uint64_t h = 1;  // (D_j / q_i) mod q_i
                for (uint32_t o = i0; o < i1; ++o)
                    if (o != i) h = mulmod(h, P->q[o] % P->q[i], P->q[i]);
                hatinv[ci] = pair(invmod(h, P->q[i]), P->q[i]);
                for (uint32_t t = 0; t < lvl + K; ++t) {
                    const uint64_t m = t < lvl ? P->q[t] : P->p[t - lvl];
                    uint64_t ht = 1;  // (D_j / q_i) mod m_t
                    for (uint32_t o = i0; o < i1; ++o)
                        if (o != i) ht = mulmod(ht, P->q[o] % m, m);
                    cmat[ci * (L + K) + t] = to_mont(ht, m);
                }
            }
        }
    }
    std::vector<TwPair> phatinv(K), pinv(2 * L), gadget(L), tomont(L + K);
    std::vector<uint64_t> downc((size_t)K * L);
    for (uint32_t k = 0; k < K; ++k) {
        uint64_t h = 1;
        for (uint32_t o = 0; o < K; ++o)
            if (o != k) h = mulmod(h, P->p[o] % P->p[k], P->p[k]);
        phatinv[k] = pair(invmod(h, P->p[k]), P->p[k]);
        for (uint32_t i = 0; i < L; ++i) {
            uint64_t hi = 1;
            for (uint32_t o = 0; o < K; ++o)
                if (o != k) hi = mulmod(hi, P->p[o] % P->q[i], P->q[i]);
            downc[(size_t)k * L + i] = to_mont(hi, P->q[i]);
        }
    }
    for (uint32_t i = 0; i < L; ++i) {
        uint64_t pm = 1;
        for (uint32_t o = 0; o < K; ++o) pm = mulmod(pm, P->p[o] % P->q[i], P->q[i]);
        pinv[i] = pair(invmod(pm, P->q[i]), P->q[i]);
        pinv[L + i] = twiddle(invmod(pm, P->q[i]), P->q[i]);  // fp64 form for q < 2^50
        gadget[i] = pair(pm, P->q[i]);
    }
    for (uint32_t m = 0; m < L + K; ++m) tomont[m] = pair(to_mont(1, P->mods[m]), P->mods[m]);
    std::vector<TwPair> rq(2 * (size_t)L * L, TwPair{0, 0});
    for (uint32_t lvl = 2; lvl <= L; ++lvl)
        for (uint32_t k = 0; k + 1 < lvl; ++k) {
            const uint64_t v = invmod(P->q[lvl - 1] % P->q[k], P->q[k]);
            rq[(size_t)(lvl - 1) * L + k] = pair(v, P->q[k]);
            rq[(size_t)L * L + (size_t)(lvl - 1) * L + k] = twiddle(v, P->q[k]);  // fp64 form for q < 2^50
        }

    // ---- MFMA base conversion operands (v_mfma_i32_32x32x16_i8).
    // The contraction y_t = sum_i x_i h_{i,t} mod m_t is evaluated with both
    // operands in signed base-256 digits: x_i = sum_a x_{i,a} 256^a and
    // V_{(i,a),t} = 256^a h_{i,t} mod m_t = sum_b v_{(i,a),t,b} 256^b, so
    // y_t = sum_b 256^b Z_{t,b} mod m_t with Z_{t,b} = sum_{i,a} x_{i,a}
    // v_{(i,a),t,b}: exact int8 x int8 products summed in int32 (|Z| <=
    // 12 * 8 * 128^2 < 2^21).  A 32 x 32 output tile holds 4 targets x 8 digit
    // rows; row r is target (r/8)%2 + 2 ((r%8)/4), digit 4 (r/16) + r%4, so
    // each lane receives all 8 digits of two targets.  Lane l of the A
    // operand holds row l%32 and k = 8 (l/32) .. +7, k = 8 i_local + a.
    auto digits = [](uint64_t v) { return v + 0x8080808080808080ull; };  // balanced digits, biased by 128
    auto digit = [&](uint64_t v, uint32_t b) { return (int)((digits(v) >> (8 * b)) & 255u) - 128; };
    auto row_t = [](uint32_t r) { return ((r / 8) % 2) + 2 * ((r % 8) / 4); };
    auto row_b = [](uint32_t r) { return 4 * (r / 16) + (r % 4); };
    auto pack_lane = [&](uint32_t lane, auto&& vmat /* (i_local, t_local, a) -> V or ~0 */) {
        uint64_t w = 0;
        const uint32_t r = lane % 32, half = lane / 32;
        for (uint32_t a = 0; a < 8; ++a) {
            const uint64_t v = vmat(half, row_t(r), a);
            const int d = v == ~0ull ? 0 : digit(v, row_b(r));
            w |= (uint64_t)(uint8_t)(int8_t)d << (8 * a);
        }
        return w;
    };
    const uint32_t up_rt = (L + K + 3) / 4, up_kb = (A + 1) / 2;
    const uint32_t dn_rt = (L + 3) / 4, dn_kb = (K + 1) / 2;
    std::vector<uint64_t> upa((size_t)L * dnum * up_rt * up_kb * 64, 0), dna((size_t)dn_rt * dn_kb * 64, 0);
    std::vector<uint64_t> pw8(8);
    for (uint32_t lvl = 1; lvl <= L; ++lvl) {
        const uint32_t beta = (lvl + A - 1) / A;
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t i0 = j * A, na = std::min(i0 + A, lvl) - i0, T = lvl + K - na;
            for (uint32_t rt = 0; rt < (T + 3) / 4; ++rt)
                for (uint32_t kb = 0; kb < (na + 1) / 2; ++kb)
                    for (uint32_t lane = 0; lane < 64; ++lane) {
                        auto vm = [&](uint32_t half, uint32_t tl, uint32_t a) -> uint64_t {
                            const uint32_t ii = 2 * kb + half, tt = 4 * rt + tl;
                            if (ii >= na || tt >= T) return ~0ull;
                            const uint32_t t = tt < i0 ? tt : tt + na;
                            const uint64_t m = t < lvl ? P->q[t] : P->p[t - lvl];
                            uint64_t h = 1;  // (D_j / q_{i0+ii}) mod m
                            for (uint32_t o = i0; o < i0 + na; ++o)
                                if (o != i0 + ii) h = mulmod(h, P->q[o] % m, m);
                            return mulmod(h, powmod(2 % m, 8 * a, m), m);
                        };
                        upa[((((size_t)(lvl - 1) * dnum + j) * up_rt + rt) * up_kb + kb) * 64 + lane] =
                            pack_lane(lane, vm);
                    }
        }
    }
    for (uint32_t rt = 0; rt < dn_rt; ++rt)
        for (uint32_t kb = 0; kb < dn_kb; ++kb)
            for (uint32_t lane = 0; lane < 64; ++lane) {
                auto vm = [&](uint32_t half, uint32_t tl, uint32_t a) -> uint64_t {
                    const uint32_t k = 2 * kb + half, i = 4 * rt + tl;
                    if (k >= K || i >= L) return ~0ull;
                    const uint64_t m = P->q[i];
                    uint64_t h = 1;  // (P / p_k) mod q_i
                    for (uint32_t o = 0; o < K; ++o)
                        if (o != k) h = mulmod(h, P->p[o] % m, m);
                    return mulmod(h, powmod(2 % m, 8 * a, m), m);
                };
                dna[((size_t)rt * dn_kb + kb) * 64 + lane] = pack_lane(lane, vm);
            }
    std::vector<BconvRed> red(L + K);
    for (uint32_t mi = 0; mi < L + K; ++mi) {
        const uint64_t m = P->mods[mi];
        const uint64_t c32 = powmod(2 % m, 32, m);
        red[mi].m = m;
        red[mi].negm = 0 - m;
        red[mi].cq0 = m << 30;
        red[mi].md = (double)m;
        red[mi].minv = 1.0 / (double)m;
        red[mi].c32 = (double)c32;
        red[mi].c32q = (double)c32 / (double)m;
        red[mi].fp = ntt_fp(m) ? 1u : 0u;
        red[mi].pad = 0;
    }

    TwPair *d_hatinv, *d_phatinv, *d_pinv;
    uint64_t *d_cmat, *d_downc, *d_upa, *d_dna;
    BconvRed* d_red;
    if ((r = upload(c, &d_upa, upa)) || (r = upload(c, &d_dna, dna)) || (r = upload(c, &d_red, red))) return r;
    if ((r = upload(c, &d_hatinv, hatinv)) || (r = upload(c, &d_cmat, cmat)) || (r = upload(c, &d_phatinv, phatinv)) ||
        (r = upload(c, &d_downc, downc)) || (r = upload(c, &d_pinv, pinv)) || (r = upload(c, &c->rescale_qinv, rq)) ||
        (r = upload(c, &c->gadget, gadget)) || (r = upload(c, &c->to_mont, tomont)))
        return r;
    c->kc = KsConsts{d_hatinv, d_cmat, d_phatinv, d_downc, d_pinv, d_upa, d_dna, d_red,
                     up_rt,    up_kb,  dn_rt,       dn_kb,   L,      K,     dnum,  A};
    return PFT_OK;
}

extern "C" int pft_ctx_create(const pft_params* P, int device, void* stream, pft_ctx** out) {
    return pft_ctx_create_alloc(P, device, stream, nullptr, out);
}

extern "C" int pft_ctx_create_alloc(const pft_params* P, int device, void* stream, const pft_allocator* alloc,
                                    pft_ctx** out) {
    if (!P || !out) return fail(PFT_EINVAL, "null argument");
    if (alloc && (!alloc->alloc) != (!alloc->free)) return fail(PFT_EINVAL, "allocator needs both alloc and free");
    HIPCK(hipSetDevice(device));
    auto* c = new pft_ctx();
    if (alloc) c->alloc = *alloc;
    c->P = P;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->home = c->stream;
    c->prof.st = c->stream;
    // the inner product's helper stream (default priority); without it the
    // two kinds of rows run one after the other on the context stream
    if (hipStreamCreateWithFlags(&c->inner_st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->inner_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->inner_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (c->inner_st) (void)hipStreamDestroy(c->inner_st);
        if (c->inner_fork) (void)hipEventDestroy(c->inner_fork);
        if (c->inner_join) (void)hipEventDestroy(c->inner_join);
        c->inner_st = nullptr;
        c->inner_fork = c->inner_join = nullptr;
    }
    for (uint64_t m : P->mods) c->fp_rows.push_back(ntt_fp(m) ? 1u : 0u);
    // the device address of this GPU's fixed scratch (null if unavailable:
    // then only the allocation-free entry point refuses)
    if (noalloc_scratch_init(device, &c->scratch)) c->scratch = nullptr;
    int r = build_tables(c);
    if (r) {
        pft_ctx_destroy(c);
        return r;
    }
    *out = c;
    return PFT_OK;
}

extern "C" void pft_ctx_destroy(pft_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (hipStream_t st : c->side) (void)hipStreamSynchronize(st);
    if (c->copy_st) (void)hipStreamSynchronize(c->copy_st);
    if (c->inner_st) (void)hipStreamSynchronize(c->inner_st);
    for (void* p : c->allocs) dev_free(c, p);
    dev_free(c, c->ws);
    dev_free(c, c->aux);
    dev_free(c, c->cbuf);
    for (void* p : c->retired) dev_free(c, p);
    if (c->copy_st) (void)hipStreamDestroy(c->copy_st);
    for (auto& ss : c->rot_sync)
        if (ss.ready) (void)hipEventDestroy(ss.ready);
    for (auto& kv : c->stream_ev)
        if (kv.second) (void)hipEventDestroy(kv.second);
    for (auto& kv : c->rot)
        if (kv.second.host) (void)hipHostFree(kv.second.host);
    for (hipStream_t st : c->side) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    for (hipEvent_t e : c->side_ev) (void)hipEventDestroy(e);
    for (auto& w : c->side_ws) dev_free(c, w.first);
    if (c->inner_st) (void)hipStreamDestroy(c->inner_st);
    if (c->inner_fork) (void)hipEventDestroy(c->inner_fork);
    if (c->inner_join) (void)hipEventDestroy(c->inner_join);
    delete c;
}

extern "C" int pft_ctx_synchronize(pft_ctx* c) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (c->capturing) return fail(PFT_EINVAL, "cannot synchronize during graph capture");
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ctx_set_budget(pft_ctx* c, uint64_t budget_bytes) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (budget_bytes && c->live_bytes > budget_bytes)
        return fail(PFT_ENOMEM, "the context already holds %llu bytes, more than a budget of %llu",
                    (unsigned long long)c->live_bytes, (unsigned long long)budget_bytes);
    c->alloc.budget_bytes = budget_bytes;
    return PFT_OK;
}

extern "C" int pft_ctx_memory(const pft_ctx* c, uint64_t* out) {
    if (!c || !out) return fail(PFT_EINVAL, "null argument");
    out[0] = c->device_bytes;
    out[1] = c->live_bytes - c->device_bytes;
    out[2] = c->alloc.budget_bytes;
    return PFT_OK;
}

extern "C" int pft_ctx_device_bytes(const pft_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return fail(PFT_EINVAL, "null argument");
    *bytes = c->device_bytes;
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// launch descriptors
// ---------------------------------------------------------------------------
// Up to eight polynomials of n_limbs rows starting at row `first`; rows below
// `split` are q-limbs, the others special limbs.
static SmallBatch sb(const pft_params* P, std::initializer_list<uint64_t*> ptrs, uint32_t n_limbs, uint32_t first = 0,
                     uint32_t split = ~0u) {
    SmallBatch b{};
    uint32_t i = 0;
    for (uint64_t* p : ptrs) b.ptr[i++] = p;
    b.n_polys = i;
    b.n_limbs = n_limbs;
    b.first = first;
    b.split = split;
    b.off0 = 0;
    b.off1 = P->L;
    return b;
}

// n_polys consecutive [rows_per_poly][N] blocks starting at base.
static SmallBatch sb_rows(const pft_params* P, uint64_t* base, uint32_t n_polys, uint32_t rows_per_poly,
                          uint32_t n_limbs, uint32_t split = ~0u) {
    SmallBatch b{};
    for (uint32_t i = 0; i < n_polys; ++i) b.ptr[i] = base + ((size_t)i * rows_per_poly << P->log_n);
    b.n_polys = n_polys;
    b.n_limbs = n_limbs;
    b.first = 0;
    b.split = split;
    b.off0 = 0;
    b.off1 = P->L;
    return b;
}

static ProfHook* hook(pft_ctx* c) { return c->prof.mask ? &c->prof : nullptr; }

// One transform job: a polynomial whose n_limbs limbs sit at rows
// i + (i >= gap_at ? gap_len : 0) of ptr.
struct NttJob {
    uint64_t* ptr;
    uint32_t gap_at, gap_len;
};

// ---- NTT schedule selection (autotuner) -----------------------------------
// Transforms of up to 2^k limbs share a class (k <= 10); every candidate
// schedule gives the same result, so the choice only affects speed.
static uint32_t ntt_class(uint64_t limbs) {
    uint32_t k = 0;
    while (k < 10 && (1ull << k) < limbs) ++k;
    return k;
}

static NttSchedule ntt_default(const pft_params* P) {
    NttSchedule s[1];
    ntt_candidates(P->log_n, s, 1);
    return s[0];
}

// Times every candidate on zeroed scratch of min(limbs, 2^class) limbs that
// cycle through all L + K moduli (fp64 and integer limbs in the chain's
// proportion): the median of five runs each.  The earliest candidate within
// 2% of the fastest wins, so near-ties resolve the same way run to run.
// col16: only candidates whose first radix is 4 (a radix-16 column pass at
// the start of a forward / the end of an inverse transform, the pass the
// fused conversion kernels apply themselves).
static NttSchedule ntt_tune(pft_ctx* c, bool inverse, uint32_t cls, bool col16 = false) {
    const pft_params* P = c->P;
    NttSchedule all[32], cand[32];
    const int na = ntt_candidates(P->log_n, all, 32);
    int nc = 0;
    for (int k = 0; k < na; ++k)
        if (!col16 || (all[k].n_passes >= 2 && all[k].radix[0] == 4)) cand[nc++] = all[k];
    if (nc == 0) return all[0];
    if (nc <= 1) return cand[0];
    const uint32_t rows = P->L + P->K;
    const uint64_t want = 1ull << cls;
    uint32_t np = (uint32_t)std::min<uint64_t>((want + rows - 1) / rows, PFT_MAX_POLYS);
    if (np == 0) np = 1;
    const uint32_t nl = (uint32_t)std::min<uint64_t>(want, rows);
    const size_t bytes = (size_t)np * rows * P->n * 8;
    void* buf = nullptr;
    if (dev_alloc(c, &buf, bytes, "autotuner scratch") != PFT_OK) {
        (void)hipGetLastError();
        return cand[0];
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) {
        dev_free(c, buf);
        return cand[0];
    }
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        dev_free(c, buf);
        return cand[0];
    }
    std::vector<float> med(nc, 1e30f);
    bool ok = hipMemsetAsync(buf, 0, bytes, c->stream) == hipSuccess;
    PolyBatch b{};
    for (uint32_t i = 0; i < np; ++i) {
        b.ptr[i] = (uint64_t*)buf + ((size_t)i * rows << P->log_n);
        b.gap_at[i] = 255;
        b.gap_len[i] = 0;
    }
    b.n_polys = np;
    b.n_limbs = nl;
    b.split = P->L;
    b.off0 = 0;
    b.off1 = P->L;
    for (int k = 0; ok && k < nc; ++k) {
        launch_ntt(b, c->tabs, P->log_n, inverse, cand[k], c->stream, nullptr);
        float t[5];
        for (int r = 0; ok && r < 5; ++r) {
            ok = hipEventRecord(e0, c->stream) == hipSuccess;
            launch_ntt(b, c->tabs, P->log_n, inverse, cand[k], c->stream, nullptr);
            ok = ok && hipEventRecord(e1, c->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&t[r], e0, e1) == hipSuccess;
        }
        if (ok) {
            std::sort(t, t + 5);
            med[k] = t[2];
        }
    }
    NttSchedule best = cand[0];
    if (ok) {
        const float fastest = *std::min_element(med.begin(), med.end());
        for (int k = 0; k < nc; ++k)
            if (med[k] <= 1.02f * fastest) {
                best = cand[k];
                break;
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    dev_free(c, buf);
    return best;
}

// Tuned choices are keyed by direction (64), restriction to first radix 4
// (32) and class.
static NttSchedule ntt_schedule(pft_ctx* c, bool inverse, uint64_t limbs, bool col16 = false) {
    if (c->ntt_pinned[inverse].n_passes) return c->ntt_pinned[inverse];
    const uint32_t key = (inverse ? 64u : 0u) + (col16 ? 32u : 0u) + ntt_class(limbs);
    auto it = c->ntt_tuned.find(key);
    if (it != c->ntt_tuned.end()) return it->second;
    if (!c->ntt_tune || c->capturing) {  // no timing inside a capture
        if (!col16) return ntt_default(c->P);
        NttSchedule all[32];
        const int na = ntt_candidates(c->P->log_n, all, 32);
        for (int k = 0; k < na; ++k)
            if (all[k].n_passes >= 2 && all[k].radix[0] == 4) return all[k];
        return ntt_default(c->P);
    }
    const NttSchedule s = ntt_tune(c, inverse, ntt_class(limbs), col16);
    c->ntt_tuned[key] = s;
    return s;
}

// epi: forward transforms of (item, b) polynomial pairs whose final pass
// finishes ModDown; epi->out lists every item, a launch gets its share.
static void ntt_jobs(pft_ctx* c, const std::vector<NttJob>& jobs, uint32_t n_limbs, uint32_t split, bool inverse,
                     uint32_t off0 = 0, const NttEpilogue* epi = nullptr, int64_t src_delta = 0, uint32_t first = 0,
                     bool col16 = false) {
    const pft_params* P = c->P;
    const NttSchedule sched = ntt_schedule(c, inverse, (uint64_t)jobs.size() * n_limbs, col16);
    for (size_t s = 0; s < jobs.size(); s += PFT_MAX_POLYS) {
        PolyBatch b{};
        const uint32_t np = (uint32_t)std::min<size_t>(PFT_MAX_POLYS, jobs.size() - s);
        for (uint32_t i = 0; i < np; ++i) {
            b.ptr[i] = jobs[s + i].ptr;
            b.gap_at[i] = (uint8_t)std::min<uint32_t>(jobs[s + i].gap_at, 255u);
            b.gap_len[i] = (uint8_t)jobs[s + i].gap_len;
        }
        b.n_polys = np;
        b.n_limbs = n_limbs;
        b.split = split;
        b.off0 = off0;
        b.off1 = P->L;
        b.src_delta = src_delta;
        if (epi) {
            NttEpilogue e = *epi;
            for (uint32_t i = 0; i < PFT_MAX_POLYS / 2; ++i) {
                e.out[i] = s / 2 + i < PFT_MAX_POLYS / 2 ? epi->out[s / 2 + i] : nullptr;
                e.acc_item[i] = s / 2 + i < PFT_MAX_POLYS / 2 ? epi->acc_item[s / 2 + i] : nullptr;
                // perm_src is per item for a forward epilogue, per polynomial for an inverse transform
                const size_t pi = inverse ? s + i : s / 2 + i;
                e.perm_src[i] = pi < PFT_MAX_POLYS / 2 ? epi->perm_src[pi] : nullptr;
            }
            launch_ntt(b, c->tabs, P->log_n, inverse, sched, c->stream, hook(c), &e, first);
        } else {
            launch_ntt(b, c->tabs, P->log_n, inverse, sched, c->stream, hook(c), nullptr, first);
        }
    }
}

// Transform of n_polys consecutive [rows_per_poly][N] blocks, limbs 0..n_limbs-1.
static void ntt_rows(pft_ctx* c, uint64_t* base, uint32_t n_polys, uint32_t rows_per_poly, uint32_t n_limbs,
                     bool inverse, uint32_t split = ~0u) {
    std::vector<NttJob> jobs;
    for (uint32_t i = 0; i < n_polys; ++i)
        jobs.push_back(NttJob{base + ((size_t)i * rows_per_poly << c->P->log_n), 255u, 0u});
    ntt_jobs(c, jobs, n_limbs, split, inverse);
}

// Runs f (one kernel launch) bracketed by profiling events when enabled.
template <typename F>
static void timed(pft_ctx* c, int kid, double bytes, double ops, F&& f, uint32_t variant = 0) {
    ProfHook* h = hook(c);
    if (h) h->begin(kid);
    f();
    if (h) h->end(kid, bytes, ops, variant);
}

// ---------------------------------------------------------------------------
// KEYGEN (Sec. 3.4)
// ---------------------------------------------------------------------------
static int upload_i64(pft_ctx* c, int64_t* dst, const int64_t* src, size_t count) {
    HIPCK(hipMemcpyAsync(dst, src, count * 8, hipMemcpyHostToDevice, c->stream));
    return PFT_OK;
}
static int upload_u64(pft_ctx* c, uint64_t* dst, const uint64_t* src, size_t count) {
    HIPCK(hipMemcpyAsync(dst, src, count * 8, hipMemcpyHostToDevice, c->stream));
    return PFT_OK;
}

static bool check_ternary(const int64_t* s, uint32_t n) {
    for (uint32_t i = 0; i < n; ++i)
        if (s[i] < -1 || s[i] > 1) return false;
    return true;
}

static bool check_uniform(const uint64_t* a, const std::vector<uint64_t>& mods, uint32_t rows, uint32_t n) {
    for (uint32_t r = 0; r < rows; ++r)
        for (uint32_t k = 0; k < n; ++k)
            if (a[(size_t)r * n + k] >= mods[r]) return false;
    return true;
}

// Where KEYGEN and ENC take their random draws: caller arrays in host memory,
// or the Philox4x64-10 streams of a seed (sampler.hip), keyed by
// (seed, purpose 2^56 + key_id 2^8 + digit).
enum : uint64_t {
    DRAW_SECRET = 1, DRAW_PK_A = 2, DRAW_PK_E = 3, DRAW_KS_A = 4, DRAW_KS_E = 5, DRAW_ENC_V = 6, DRAW_ENC_E0 = 7,
    DRAW_ENC_E1 = 8
};
struct Draws {
    bool seeded;
    uint64_t seed;
    uint64_t key_id;     // switching keys: 0 relinearisation, 1 + step for rotation by step
    const uint64_t* a;   // host masks (not seeded)
    const int64_t* e;    // host errors (not seeded)
};
static Draws host_draws(const uint64_t* a, const int64_t* e) { return Draws{false, 0, 0, a, e}; }
static Draws seeded_draws(uint64_t seed, uint64_t key_id) { return Draws{true, seed, key_id, nullptr, nullptr}; }
static uint64_t stream_k1(uint64_t purpose, uint64_t key_id, uint32_t digit) {
    return (purpose << 56) | (key_id << 8) | digit;
}
static const GaussianCdt& gaussian_cdt() {
    static const GaussianCdt t = [] {
        GaussianCdt g{};
        const int k = gaussian_cdt_host(g.t, 2 * PFT_GAUSS_BOUND);
        g.count = k > 0 ? (uint32_t)k : 0u;  // the kernel reads t[0 .. count)
        return g;
    }();
    return t;
}
// rows x N uniform residues of stream (seed, purpose, key_id, digit) into dev
static void sample_uniform(pft_ctx* c, const Draws& d, uint64_t purpose, uint32_t digit, const uint64_t* mods,
                           uint32_t rows, uint64_t* dev) {
    SampleModuli sm{};
    for (uint32_t i = 0; i < rows; ++i) sm.q[i] = mods[i];
    launch_sample_uniform(d.seed, stream_k1(purpose, d.key_id, digit), sm, rows, dev, c->P->n, c->stream);
}
// N ternary (kind 0) or discrete-Gaussian (kind 1) coefficients into dev
static void sample_small(pft_ctx* c, const Draws& d, uint32_t kind, uint64_t purpose, uint32_t digit, int64_t* dev) {
    launch_sample_small(kind, d.seed, stream_k1(purpose, d.key_id, digit), gaussian_cdt(), dev, c->P->n, c->stream);
}

extern "C" int pft_gaussian_cdt(uint64_t* table, uint32_t capacity, uint32_t* count) {
    if (!table || !count) return fail(PFT_EINVAL, "null argument");
    const int k = gaussian_cdt_host(table, capacity);
    if (k < 0) return fail(PFT_EINVAL, "capacity below %u", 2u * PFT_GAUSS_BOUND);
    *count = (uint32_t)k;
    return PFT_OK;
}

// Every key derived from the secret (public, relinearisation and rotation
// keys) is dropped when the secret changes, so that no key of an earlier
// secret stays usable; the device memory of dropped rotation keys is reused
// by the keys generated next.  Queued work may still read the old keys, so
// the stream is drained first.
static int drop_derived_keys(pft_ctx* c) {
    HIPCK(hipStreamSynchronize(c->stream));
    if (c->copy_st) HIPCK(hipStreamSynchronize(c->copy_st));  // no key copy still reads a host copy
    c->pk_ok = false;
    c->rlk_ok = false;
    for (auto& kv : c->rot) {
        SwitchKeyDev& k = kv.second;
        if (k.slot < 0 && k.data) c->key_pool.push_back(k.data);
        if (k.host) (void)hipHostFree(k.host);
    }
    c->rot.clear();
    for (auto& o : c->rot_slot_owner) o = -1;
    for (auto& ss : c->rot_sync) {
        ss.readers.clear();
        ss.ready_pending = false;
    }
    return PFT_OK;
}

static int set_secret_core(pft_ctx* c, const int64_t* s, const Draws& d) {
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    int r;
    if (!c->s && (r = dalloc(c, &c->s, (size_t)R * P->n * 8))) return r;
    if ((r = ensure_ws(c, (size_t)P->n * 8))) return r;
    if (d.seeded)
        sample_small(c, d, 0, DRAW_SECRET, 0, (int64_t*)c->ws);
    else if ((r = upload_i64(c, (int64_t*)c->ws, s, P->n)))
        return r;
    launch_int_to_rns((const int64_t*)c->ws, sb(P, {c->s}, R, 0, P->L), c->tabs, P->log_n, c->stream);
    ntt_rows(c, c->s, 1, R, R, false, P->L);
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_set_secret(pft_ctx* c, const int64_t* s) {
    if (!c || !s) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    if (!check_ternary(s, c->P->n)) return fail(PFT_EINVAL, "secret must be ternary");
    int r;
    if ((r = drop_derived_keys(c))) return r;
    return set_secret_core(c, s, host_draws(nullptr, nullptr));
}

static int gen_public_key_core(pft_ctx* c, const Draws& d) {
    const pft_params* P = c->P;
    int r;
    const size_t nL = (size_t)P->L * P->n;
    if (!c->pk && (r = dalloc(c, &c->pk, 2 * nL * 8))) return r;
    if ((r = ensure_ws(c, (nL + P->n) * 8))) return r;
    uint64_t* e_rns = c->ws;
    int64_t* e_raw = (int64_t*)(c->ws + nL);
    uint64_t* pa = c->pk + nL;
    if (d.seeded) {
        sample_uniform(c, d, DRAW_PK_A, 0, P->q.data(), P->L, pa);
        sample_small(c, d, 1, DRAW_PK_E, 0, e_raw);
    } else if ((r = upload_u64(c, pa, d.a, nL)) || (r = upload_i64(c, e_raw, d.e, P->n))) {
        return r;
    }
    ntt_rows(c, pa, 1, P->L, P->L, false);
    launch_int_to_rns(e_raw, sb(P, {e_rns}, P->L), c->tabs, P->log_n, c->stream);
    ntt_rows(c, e_rns, 1, P->L, P->L, false);
    // b = -(a s) + e
    SmallBatch A = sb(P, {pa}, P->L), S = sb(P, {c->s}, P->L), E = sb(P, {e_rns}, P->L), B = sb(P, {c->pk}, P->L);
    launch_ew(EW_NEG_MULADD, B, A, &S, &E, c->tabs, P->log_n, c->stream);
    HIPCK(hipStreamSynchronize(c->stream));
    c->pk_ok = true;
    return PFT_OK;
}

extern "C" int pft_gen_public_key(pft_ctx* c, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    if (!check_uniform(a, c->P->q, c->P->L, c->P->n)) return fail(PFT_EINVAL, "mask residues must be < q_i");
    return gen_public_key_core(c, host_draws(a, e));
}

// s_prime: [L+K][N] NTT domain (device).  Builds the switching key into *dst.
static size_t key_bytes(const pft_params* P) { return (size_t)P->dnum * 2 * (P->L + P->K) * P->n * 8; }

// Distance from the cache's plan position to the next use of rotation step
// `ns` in the cyclic plan (0: the next rotation), or SIZE_MAX if the plan
// does not use it (or there is no plan).
static size_t plan_next_use(const pft_ctx* c, int32_t ns) {
    const size_t n = c->rot_plan.size();
    for (size_t d = 0; d < n; ++d)
        if (c->rot_plan[(c->rot_plan_pos + d) % n] == ns) return d;
    return SIZE_MAX;
}

// Makes `fill` wait until every queued read of slot `idx` has run: each
// stream that read the slot since its last fill records its event now (its
// reads were enqueued earlier) and `fill` waits for it; a fill still in
// flight on the copy stream is waited for too.  Clears the reader list.
static int slot_wait_readers(pft_ctx* c, int idx, hipStream_t fill) {
    pft_ctx::SlotSync& ss = c->rot_sync[idx];
    for (hipStream_t rs : ss.readers) {
        if (rs == fill) continue;  // stream order suffices
        hipEvent_t& ev = c->stream_ev[rs];
        if (!ev) HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCK(hipEventRecord(ev, rs));
        HIPCK(hipStreamWaitEvent(fill, ev, 0));
    }
    ss.readers.clear();
    if (ss.ready_pending && fill != c->copy_st) HIPCK(hipStreamWaitEvent(fill, ss.ready, 0));
    return PFT_OK;
}

// A device slot for rotation key `step` under the limited key cache: a free
// slot, a new one below the limit, else a victim's (the resident key whose
// next use in the plan is farthest ahead, without a plan the least recently
// used; never `keep`).  The victim becomes non-resident; the slot is not
// filled here (the caller orders the fill after the slot's readers with
// slot_wait_readers).  Sets the key's data and slot; *idx_out = the slot, or
// -1 if every slot holds `keep`.
static int key_slot(pft_ctx* c, int32_t step, int32_t keep, int* idx_out) {
    int idx = -1;
    *idx_out = -1;
    for (size_t i = 0; i < c->rot_slot_owner.size(); ++i)
        if (c->rot_slot_owner[i] < 0) {
            idx = (int)i;
            break;
        }
    if (idx < 0 && c->rot_slots.size() < c->rot_cache_max) {
        uint64_t* p = nullptr;
        int r;
        if ((r = dalloc(c, &p, key_bytes(c->P)))) return r;
        c->rot_slots.push_back(p);
        c->rot_slot_owner.push_back(-1);
        c->rot_sync.emplace_back();
        HIPCK(hipEventCreateWithFlags(&c->rot_sync.back().ready, hipEventDisableTiming));
        idx = (int)c->rot_slots.size() - 1;
    }
    if (idx < 0) {
        size_t far = 0;
        uint64_t oldest = ~0ull;
        for (size_t i = 0; i < c->rot_slots.size(); ++i) {
            const int32_t owner = c->rot_slot_owner[i];
            if (owner == keep) continue;
            const SwitchKeyDev& o = c->rot[owner];
            const size_t d = plan_next_use(c, owner);
            if (idx < 0 || d > far || (d == far && o.last_use < oldest)) {
                far = d;
                oldest = o.last_use;
                idx = (int)i;
            }
        }
        if (idx < 0) return PFT_OK;
        SwitchKeyDev& victim = c->rot[c->rot_slot_owner[idx]];
        victim.data = nullptr;
        victim.slot = -1;
    }
    SwitchKeyDev& k = c->rot[step];
    c->rot_slot_owner[idx] = step;
    k.data = c->rot_slots[idx];
    k.slot = idx;
    k.last_use = ++c->rot_clock;
    *idx_out = idx;
    return PFT_OK;
}

// Copies the pinned host copy of rotation key `ns` into a slot on the copy
// stream (after the slot's readers); readers wait for the slot's `ready`
// event.  `keep` is never evicted.  *copied = false if no slot could be
// freed.
static int key_fill(pft_ctx* c, int32_t ns, int32_t keep, bool* copied) {
    *copied = false;
    int r, idx;
    if ((r = key_slot(c, ns, keep, &idx))) return r;
    if (idx < 0) return PFT_OK;
    if (!c->copy_st) HIPCK(hipStreamCreateWithFlags(&c->copy_st, hipStreamNonBlocking));
    if ((r = slot_wait_readers(c, idx, c->copy_st))) return r;
    SwitchKeyDev& k = c->rot[ns];
    const size_t bytes = key_bytes(c->P);
    HIPCK(hipMemcpyAsync(k.data, k.host, bytes, hipMemcpyHostToDevice, c->copy_st));
    pft_ctx::SlotSync& ss = c->rot_sync[idx];
    HIPCK(hipEventRecord(ss.ready, c->copy_st));
    ss.ready_pending = true;
    c->rot_bytes_in += bytes;
    *copied = true;
    return PFT_OK;
}

static int check_switch_draws(const pft_params* P, const uint64_t* a) {
    const uint32_t R = P->L + P->K;
    const size_t nR = (size_t)R * P->n;
    for (uint32_t j = 0; j < P->dnum; ++j)
        if (!check_uniform(a + (size_t)j * nR, P->mods, R, P->n))
            return fail(PFT_EINVAL, "mask residues must be < their modulus");
    return PFT_OK;
}

static int gen_switch_key(pft_ctx* c, const uint64_t* s_prime, const Draws& d, SwitchKeyDev* dst) {
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    const size_t nR = (size_t)R * P->n;
    int r;
    if (!dst->data && !c->key_pool.empty()) {
        dst->data = c->key_pool.back();
        c->key_pool.pop_back();
    }
    if (!dst->data && (r = dalloc(c, &dst->data, (size_t)P->dnum * 2 * nR * 8))) return r;
    if ((r = ensure_ws(c, (nR + P->n + nR) * 8))) return r;
    uint64_t* e_rns = c->ws;
    int64_t* e_raw = (int64_t*)(c->ws + nR);
    uint64_t* gs = c->ws + nR + P->n;  // gadget * s'
    const SmallBatch S = sb(P, {c->s}, R, 0, P->L);
    for (uint32_t j = 0; j < P->dnum; ++j) {
        uint64_t* kb = dst->data + (size_t)(2 * j) * nR;
        uint64_t* ka = dst->data + (size_t)(2 * j + 1) * nR;
        if (d.seeded) {
            sample_uniform(c, d, DRAW_KS_A, j, P->mods.data(), R, ka);
            sample_small(c, d, 1, DRAW_KS_E, j, e_raw);
        } else if ((r = upload_u64(c, ka, d.a + (size_t)j * nR, nR)) ||
                   (r = upload_i64(c, e_raw, d.e + (size_t)j * P->n, P->n))) {
            return r;
        }
        ntt_rows(c, ka, 1, R, R, false, P->L);
        launch_int_to_rns(e_raw, sb(P, {e_rns}, R, 0, P->L), c->tabs, P->log_n, c->stream);
        ntt_rows(c, e_rns, 1, R, R, false, P->L);
        const SmallBatch A = sb(P, {ka}, R, 0, P->L), E = sb(P, {e_rns}, R, 0, P->L), B = sb(P, {kb}, R, 0, P->L);
        launch_ew(EW_NEG_MULADD, B, A, &S, &E, c->tabs, P->log_n, c->stream);  // b = -a s + e
        // + (P mod q_t) s' on the q-limbs of digit j
        const uint32_t i0 = j * P->alpha, i1 = std::min(i0 + P->alpha, P->L);
        if (i0 < i1) {
            const SmallBatch Sp = sb(P, {(uint64_t*)s_prime}, i1 - i0, i0), G = sb(P, {gs}, i1 - i0, i0);
            launch_mul_const(G, Sp, c->gadget + i0, c->tabs, P->log_n, c->stream);
            const SmallBatch Bd = sb(P, {kb}, i1 - i0, i0);
            launch_ew(EW_ADD, Bd, Bd, &G, nullptr, c->tabs, P->log_n, c->stream);
        }
        // both halves in the inner product's storage form (launch_key_form)
        launch_key_form(sb(P, {kb, ka}, R, 0, P->L), c->to_mont, c->tabs, P->log_n, c->stream);
    }
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

static int gen_relin_key_core(pft_ctx* c, const Draws& d) {
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    int r;
    if (!c->s_prime && (r = dalloc(c, &c->s_prime, (size_t)R * P->n * 8))) return r;
    const SmallBatch S = sb(P, {c->s}, R, 0, P->L), S2 = sb(P, {c->s_prime}, R, 0, P->L);
    launch_ew(EW_MUL, S2, S, &S, nullptr, c->tabs, P->log_n, c->stream);
    if ((r = gen_switch_key(c, c->s_prime, d, &c->rlk))) return r;
    c->rlk_ok = true;
    return PFT_OK;
}

extern "C" int pft_gen_relin_key(pft_ctx* c, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    int r;
    if ((r = check_switch_draws(c->P, a))) return r;
    return gen_relin_key_core(c, host_draws(a, e));
}

static uint64_t galois_element(int32_t step, uint32_t n) {
    const int64_t half = n / 2;
    int64_t r = ((int64_t)step % half + half) % half;
    return powmod(5, (uint64_t)r, 2ull * n);
}

// kappa^-1 modulo 2N: the units modulo 2N form a group of order N, so the
// inverse is kappa^(N-1).
static uint64_t galois_inverse(uint64_t kappa, uint32_t n) { return powmod(kappa, n - 1, 2ull * n); }

static int32_t norm_step(int32_t step, uint32_t n) {
    const int64_t half = n / 2;
    return (int32_t)((((int64_t)step % half) + half) % half);
}

static ItemPtrs one_item(uint64_t* p) {
    ItemPtrs ip{};
    ip.p[0] = p;
    return ip;
}

static int gen_rotation_key_core(pft_ctx* c, int32_t step, const Draws& d) {
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    int r;
    if (!c->s_prime && (r = dalloc(c, &c->s_prime, (size_t)R * P->n * 8))) return r;
    launch_automorphism_b(1, one_item(c->s), R, WsRef{c->s_prime, 0}, 0, galois_element(step, P->n), P->log_n,
                          c->stream);
    const int32_t ns = norm_step(step, P->n);
    SwitchKeyDev& k = c->rot[ns];
    if (!c->rot_cache_max) return gen_switch_key(c, c->s_prime, d, &k);
    // limited key cache: generate into a slot, keep the pinned host copy
    const size_t bytes = key_bytes(P);
    if (!k.host) {
        void* h = nullptr;
        if (hipHostMalloc(&h, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->rot.erase(ns);
            return fail(PFT_ENOMEM, "pinned host memory for a rotation key (%zu bytes)", bytes);
        }
        k.host = (uint64_t*)h;
    }
    if (!k.data) {
        int idx;
        if ((r = key_slot(c, ns, ns, &idx))) return r;
        if (idx < 0) return fail(PFT_ENOMEM, "no rotation-key slot");
        // the key is written on the context stream
        if ((r = slot_wait_readers(c, idx, c->stream))) return r;
        c->rot_sync[idx].ready_pending = false;
    }
    if ((r = gen_switch_key(c, c->s_prime, d, &k))) return r;
    HIPCK(hipMemcpyAsync(k.host, k.data, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_gen_rotation_key(pft_ctx* c, int32_t step, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    int r;
    if ((r = check_switch_draws(c->P, a))) return r;
    return gen_rotation_key_core(c, step, host_draws(a, e));
}

extern "C" int pft_keygen(pft_ctx* c, uint64_t seed, const int32_t* rot_steps, uint32_t n_steps) {
    if (!c || (n_steps && !rot_steps)) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "key generation cannot be captured in a graph");
    const uint32_t half = c->P->n / 2;
    for (uint32_t i = 0; i < n_steps; ++i)  // refuse before any key changes
        if (norm_step(rot_steps[i], c->P->n) == 0)
            return fail(PFT_EINVAL, "rotation step %d is 0 mod N/2 = %u", rot_steps[i], half);
    int r;
    if ((r = drop_derived_keys(c))) return r;
    if ((r = set_secret_core(c, nullptr, seeded_draws(seed, 0))) || (r = gen_public_key_core(c, seeded_draws(seed, 0))) ||
        (r = gen_relin_key_core(c, seeded_draws(seed, 0))))
        return r;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const int32_t ns = norm_step(rot_steps[i], c->P->n);
        if ((r = gen_rotation_key_core(c, rot_steps[i], seeded_draws(seed, 1u + (uint64_t)ns)))) return r;
    }
    return PFT_OK;
}

extern "C" int pft_set_key_cache(pft_ctx* c, uint32_t max_resident) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (!c->rot.empty()) return fail(PFT_EINVAL, "set the key cache before generating rotation keys");
    c->rot_cache_max = max_resident;
    return PFT_OK;
}

extern "C" int pft_key_cache_plan(pft_ctx* c, const int32_t* steps, uint32_t n_steps) {
    if (!c || (n_steps && !steps)) return fail(PFT_EINVAL, "null argument");
    std::vector<int32_t> plan;
    for (uint32_t i = 0; i < n_steps; ++i) {
        const int32_t ns = norm_step(steps[i], c->P->n);
        if (ns == 0) return fail(PFT_EINVAL, "rotation step %d is 0 mod N/2", steps[i]);
        plan.push_back(ns);
    }
    c->rot_plan.swap(plan);
    c->rot_plan_pos = 0;
    return PFT_OK;
}

extern "C" int pft_key_cache_stats(const pft_ctx* c, uint64_t* out) {
    if (!c || !out) return fail(PFT_EINVAL, "null argument");
    out[0] = c->rot_cache_max;
    out[1] = c->rot_slots.size();
    out[2] = c->rot_hits;
    out[3] = c->rot_misses;
    out[4] = c->rot_bytes_in;
    out[5] = c->rot_prefetches;
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// ENC / DEC, import / export
// ---------------------------------------------------------------------------
static int check_ct(const pft_ctx* c, const pft_ct* ct) {
    if (!ct || !ct->data) return fail(PFT_EINVAL, "null ciphertext");
    if (ct->level < 1 || ct->level > c->P->L) return fail(PFT_ELEVEL, "level %u out of range", ct->level);
    return PFT_OK;
}

// ENC with (v, e0, e1) from host arrays, or from the streams of d.seed
static int encrypt_core(pft_ctx* c, const int64_t* m, uint32_t level, double scale, const int64_t* v,
                        const int64_t* e0, const int64_t* e1, const Draws& d, pft_ct* out) {
    const pft_params* P = c->P;
    if (!c->pk_ok) return fail(PFT_ENOKEY, "no public key for the current secret");
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    const uint32_t n = P->n;
    const size_t nl = (size_t)level * n;
    int r;
    if ((r = ensure_ws(c, (4 * nl + 4 * (size_t)n) * 8))) return r;
    uint64_t* M = c->ws;
    uint64_t* V = M + nl;
    uint64_t* E0 = V + nl;
    uint64_t* E1 = E0 + nl;
    int64_t* raw = (int64_t*)(E1 + nl);
    if ((r = upload_i64(c, raw, m, n))) return r;
    if (d.seeded) {
        sample_small(c, d, 0, DRAW_ENC_V, 0, raw + n);
        sample_small(c, d, 1, DRAW_ENC_E0, 0, raw + 2 * n);
        sample_small(c, d, 1, DRAW_ENC_E1, 0, raw + 3 * n);
    } else if ((r = upload_i64(c, raw + n, v, n)) || (r = upload_i64(c, raw + 2 * n, e0, n)) ||
               (r = upload_i64(c, raw + 3 * n, e1, n))) {
        return r;
    }
    launch_int_to_rns(raw, sb(P, {M, V, E0, E1}, level), c->tabs, P->log_n, c->stream);
    ntt_rows(c, M, 4, level, level, false);
    const size_t nL = (size_t)P->L * n;
    const SmallBatch Bk = sb(P, {c->pk}, level), Ak = sb(P, {c->pk + nL}, level), Vb = sb(P, {V}, level);
    const SmallBatch C0 = sb(P, {out->data}, level), C1 = sb(P, {out->data + nl}, level);
    const SmallBatch E0b = sb(P, {E0}, level), E1b = sb(P, {E1}, level), Mb = sb(P, {M}, level);
    launch_ew(EW_MULADD, C0, Bk, &Vb, &E0b, c->tabs, P->log_n, c->stream);  // b v + e0
    launch_ew(EW_ADD, C0, C0, &Mb, nullptr, c->tabs, P->log_n, c->stream);  // + m
    launch_ew(EW_MULADD, C1, Ak, &Vb, &E1b, c->tabs, P->log_n, c->stream);  // a v + e1
    out->level = level;
    out->scale = scale;
    HIPCK(hipStreamSynchronize(c->stream));  // the raw host inputs were pageable copies
    return PFT_OK;
}

extern "C" int pft_encrypt(pft_ctx* c, const int64_t* m, uint32_t level, double scale, const int64_t* v,
                           const int64_t* e0, const int64_t* e1, pft_ct* out) {
    if (!c || !m || !v || !e0 || !e1 || !out || !out->data) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    if (!check_ternary(v, c->P->n)) return fail(PFT_EINVAL, "v must be ternary");
    return encrypt_core(c, m, level, scale, v, e0, e1, host_draws(nullptr, nullptr), out);
}

extern "C" int pft_encrypt_seeded(pft_ctx* c, const int64_t* m, uint32_t level, double scale, uint64_t seed,
                                  pft_ct* out) {
    if (!c || !m || !out || !out->data) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    return encrypt_core(c, m, level, scale, nullptr, nullptr, nullptr, seeded_draws(seed, 0), out);
}

extern "C" int pft_decrypt(pft_ctx* c, const pft_ct* ct, uint64_t* out) {
    if (!c || !out) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    int r;
    if ((r = check_ct(c, ct))) return r;
    if (!c->s) return fail(PFT_ENOKEY, "no secret");
    const pft_params* P = c->P;
    const size_t nl = (size_t)ct->level * P->n;
    if ((r = ensure_ws(c, nl * 8))) return r;
    const SmallBatch Mu = sb(P, {c->ws}, ct->level), C0 = sb(P, {ct->data}, ct->level);
    const SmallBatch C1 = sb(P, {ct->data + nl}, ct->level), S = sb(P, {c->s}, ct->level);
    launch_ew(EW_MULADD, Mu, C1, &S, &C0, c->tabs, P->log_n, c->stream);
    ntt_rows(c, c->ws, 1, ct->level, ct->level, true);
    HIPCK(hipMemcpyAsync(out, c->ws, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ct_export(pft_ctx* c, const pft_ct* ct, uint64_t* host) {
    if (!c || !host) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    int r;
    if ((r = check_ct(c, ct))) return r;
    const pft_params* P = c->P;
    const size_t nl = (size_t)ct->level * P->n;
    if ((r = ensure_ws(c, 2 * nl * 8))) return r;
    HIPCK(hipMemcpyAsync(c->ws, ct->data, 2 * nl * 8, hipMemcpyDeviceToDevice, c->stream));
    ntt_rows(c, c->ws, 2, ct->level, ct->level, true);
    HIPCK(hipMemcpyAsync(host, c->ws, 2 * nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ct_import(pft_ctx* c, const uint64_t* host, uint32_t level, double scale, pft_ct* ct) {
    if (!c || !host || !ct || !ct->data) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    const pft_params* P = c->P;
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    for (uint32_t b = 0; b < 2; ++b)
        if (!check_uniform(host + (size_t)b * level * P->n, P->q, level, P->n))
            return fail(PFT_EINVAL, "residues must be < q_i");
    const size_t nl = (size_t)level * P->n;
    HIPCK(hipMemcpyAsync(ct->data, host, 2 * nl * 8, hipMemcpyHostToDevice, c->stream));
    ntt_rows(c, ct->data, 2, level, level, false);
    ct->level = level;
    ct->scale = scale;
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_pt_from_coeffs(pft_ctx* c, const int64_t* m, uint32_t level, double scale, pft_pt* pt) {
    if (!c || !m || !pt || !pt->data) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "host transfers cannot be captured in a graph");
    const pft_params* P = c->P;
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    int r;
    if ((r = ensure_ws(c, (size_t)P->n * 8))) return r;
    if ((r = upload_i64(c, (int64_t*)c->ws, m, P->n))) return r;
    launch_int_to_rns((const int64_t*)c->ws, sb(P, {pt->data}, level), c->tabs, P->log_n, c->stream);
    ntt_rows(c, pt->data, 1, level, level, false);
    pt->level = level;
    pt->scale = scale;
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// homomorphic operations
// ---------------------------------------------------------------------------
static bool scales_match(double a, double b) { return std::fabs(a - b) <= std::ldexp(std::fabs(a), -40); }

extern "C" int pft_add(pft_ctx* c, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, a)) || (r = check_ct(c, b))) return r;
    if (!out || !out->data) return fail(PFT_EINVAL, "null output");
    if (a->level != b->level) return fail(PFT_ELEVEL, "HADD needs equal levels (%u vs %u)", a->level, b->level);
    if (!scales_match(a->scale, b->scale)) return fail(PFT_ESCALE, "HADD needs equal scales");
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    const SmallBatch O = sb_rows(P, out->data, 2, l, l), A = sb_rows(P, a->data, 2, l, l),
                     B = sb_rows(P, b->data, 2, l, l);
    launch_ew(EW_ADD, O, A, &B, nullptr, c->tabs, P->log_n, c->stream);
    out->level = l;
    out->scale = a->scale;
    return PFT_OK;
}

static int check_pt(const pft_pt* p, uint32_t level) {
    if (!p || !p->data) return fail(PFT_EINVAL, "null plaintext");
    if (p->level < level) return fail(PFT_ELEVEL, "plaintext level %u below ciphertext level %u", p->level, level);
    return PFT_OK;
}

extern "C" int pft_add_plain(pft_ctx* c, const pft_ct* a, const pft_pt* p, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, a)) || (r = check_pt(p, a->level))) return r;
    if (!out || !out->data) return fail(PFT_EINVAL, "null output");
    if (!scales_match(a->scale, p->scale)) return fail(PFT_ESCALE, "HADDPLAIN needs equal scales");
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    const size_t nl = (size_t)l * P->n;
    const SmallBatch O0 = sb(P, {out->data}, l), A0 = sb(P, {a->data}, l), Pt = sb(P, {p->data}, l);
    launch_ew(EW_ADD, O0, A0, &Pt, nullptr, c->tabs, P->log_n, c->stream);
    if (out->data != a->data)
        HIPCK(hipMemcpyAsync(out->data + nl, a->data + nl, nl * 8, hipMemcpyDeviceToDevice, c->stream));
    out->level = l;
    out->scale = a->scale;
    return PFT_OK;
}

extern "C" int pft_mul_plain(pft_ctx* c, const pft_ct* a, const pft_pt* p, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, a)) || (r = check_pt(p, a->level))) return r;
    if (!out || !out->data) return fail(PFT_EINVAL, "null output");
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    const SmallBatch O = sb_rows(P, out->data, 2, l, l), A = sb_rows(P, a->data, 2, l, l);
    const SmallBatch Pt = sb(P, {p->data, p->data}, l);
    launch_ew(EW_MUL, O, A, &Pt, nullptr, c->tabs, P->log_n, c->stream);
    out->level = l;
    out->scale = a->scale * p->scale;
    return PFT_OK;
}

extern "C" int pft_mod_drop(pft_ctx* c, const pft_ct* in, uint32_t level, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, in))) return r;
    if (!out || !out->data) return fail(PFT_EINVAL, "null output");
    if (level < 1 || level > in->level) return fail(PFT_ELEVEL, "mod_drop to %u from %u", level, in->level);
    const pft_params* P = c->P;
    const size_t lo = (size_t)level * P->n, li = (size_t)in->level * P->n;
    if (out->data == in->data) {
        // in place: poly 1 moves down from row in_level to row level; go
        // through the workspace because the two ranges may overlap
        if (level != in->level) {
            if ((r = ensure_ws(c, lo * 8))) return r;
            HIPCK(hipMemcpyAsync(c->ws, in->data + li, lo * 8, hipMemcpyDeviceToDevice, c->stream));
            HIPCK(hipMemcpyAsync(out->data + lo, c->ws, lo * 8, hipMemcpyDeviceToDevice, c->stream));
        }
    } else {
        HIPCK(hipMemcpyAsync(out->data, in->data, lo * 8, hipMemcpyDeviceToDevice, c->stream));
        HIPCK(hipMemcpyAsync(out->data + lo, in->data + li, lo * 8, hipMemcpyDeviceToDevice, c->stream));
    }
    out->level = level;
    out->scale = in->scale;
    return PFT_OK;
}

// ---- batched hybrid key switching ---------------------------------------
// Per-item workspace words after the op's own prefix.
struct KsLayout {
    uint32_t level, beta, rows;
    uint64_t off_dcoef, off_ext, off_acc, off_conv, end;
};

static KsLayout ks_layout(const pft_params* P, uint32_t level, uint64_t base) {
    KsLayout k{};
    k.level = level;
    k.beta = (level + P->alpha - 1) / P->alpha;
    k.rows = level + P->K;
    const uint64_t n = P->n;
    k.off_dcoef = base;
    k.off_ext = k.off_dcoef + level * n;
    k.off_acc = k.off_ext + (uint64_t)k.beta * k.rows * n;
    k.off_conv = k.off_acc + 2ull * k.rows * n;
    k.end = k.off_conv + 2ull * level * n;
    return k;
}

static ItemPtrs ws_items(WsRef ws, uint32_t n, uint64_t off = 0) {
    ItemPtrs ip{};
    for (uint32_t z = 0; z < n; ++z) ip.p[z] = ws.base + z * ws.stride + off;
    return ip;
}

// Forward transforms whose first pass a fused kernel applies (the base
// conversions, RESCALE's expansion) take their schedule among those that
// start with a radix-16 column pass where the ring is large (N >= 2^15) and
// so is the batch (a class above 256 limbs): there the fused path beats any
// unfused schedule (bag-of-words batch at N = 2^15: 450 -> 530 documents/s),
// while with smaller rings or batches the tuner's unrestricted choice is
// kept (it fuses only when that choice starts with radix 16 anyway; a forced
// fusion was 10-17% slower on the N = 2^14 op list).
static bool fwd_col16_restricted(const pft_ctx* c, uint64_t limbs) {
    return c->P->log_n >= 15 && ntt_class(limbs) >= 9;
}
// Whether a forward transform of `limbs` limbs starts with a radix-16 column
// pass under that choice (or the pinned schedule).
static bool first_pass_col16(pft_ctx* c, uint64_t limbs) {
    const NttSchedule s = ntt_schedule(c, false, limbs, fwd_col16_restricted(c, limbs));
    return s.n_passes >= 2 && s.radix[0] == 4;
}
// Whether an inverse transform of `limbs` limbs can end with a radix-16
// column pass (the schedule chosen among such candidates, or the pinned one).
static bool last_pass_col16(pft_ctx* c, uint64_t limbs) {
    const NttSchedule s = ntt_schedule(c, true, limbs, true);
    return s.n_passes >= 2 && s.radix[0] == 4;
}

// The input of a rotation's key switch: item z's ciphertext src[z]
// ([2][level][N], NTT domain) under X -> X^kappa.  Its c1 image is d and
// its c0 image is the addend of the first output polynomial.
struct KsRot {
    uint64_t kappa, kappa_inv;
    ItemPtrs src;
};

// Key switching of d (NTT domain, [level][N] at ws_z + off_d) for n items:
// out_z = ModDown(sum_j ModUp_j(d) key_j) + (ws rows at off_add0/off_add1),
// plus, for the first polynomial, the rows at off_add0b (out may be those
// rows: each element is read before it is written).
// rot: d and the first addend are the X^kappa images of rot->src (out must
// not overlap rot->src).  Where the inner product is fused with the row pass
// of ModUp's rows, the permutation is folded into the loads of the kernels
// that read them (the first pass of d's inverse transform, the own rows of
// the inner product, the ModDown epilogue); otherwise both images are first
// written to the workspace at off_add0 (c0) and off_d = off_add0 + level N
// (c1).
static void key_switch_b(pft_ctx* c, uint32_t n, WsRef ws, const KsLayout& K, uint64_t off_d,
                         const SwitchKeyDev& key, uint64_t off_add0, uint64_t off_add1, const ItemPtrs& out,
                         uint64_t off_add0b = PFT_NO_OFFSET, const KsRot* rot = nullptr) {
    const pft_params* P = c->P;
    const uint32_t lg = P->log_n, A = P->alpha, level = K.level, rows = K.rows, beta = K.beta;
    const double N = (double)P->n;
    const uint64_t nl = (uint64_t)level * P->n;
    // ModUp's rows: all digits of all items, full digits and the ragged last
    // digit in separate transform launches (different limb counts)
    std::vector<NttJob> full, last;
    uint32_t na_last = 0;
    for (uint32_t z = 0; z < n; ++z)
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t i0 = j * A, na = std::min(i0 + A, level) - i0;
            NttJob job{ws.base + z * ws.stride + K.off_ext + ((uint64_t)j * rows << lg), i0, na};
            (na == A ? full : last).push_back(job);
            if (na != A) na_last = na;
        }
    auto col16 = [&](const std::vector<NttJob>& jobs, uint32_t limbs) {
        return jobs.empty() || first_pass_col16(c, (uint64_t)jobs.size() * limbs);
    };
    // Where the forward schedules start with a radix-16 column pass, ModUp
    // applies that pass itself; then d's inverse transform also stops before
    // its final radix-16 column pass (a schedule chosen among those ending
    // with one) and ModUp applies that pass to its inputs.
    const uint32_t nkb = (std::min(P->alpha, level) + 1) / 2;
    const bool fuse = c->bconv_mfma && c->bconv_fuse && lg >= 8 && nkb <= 6 && col16(full, rows - A) &&
                      col16(last, rows - na_last);
    const bool ifuse_up = fuse && last_pass_col16(c, (uint64_t)n * level);
    // the remaining (row) pass of the rows' forward transform, and the key
    // inner product: fused in one kernel where that pass is the row pass of
    // a (4, log_n - 4) schedule, else a transform launch per digit group and
    // the inner-product kernel
    const uint64_t rs_limbs =
        full.empty() ? (uint64_t)last.size() * (rows - na_last) : (uint64_t)full.size() * (rows - A);
    const NttSchedule rs = ntt_schedule(c, false, rs_limbs, fuse && fwd_col16_restricted(c, rs_limbs));
    const bool fuse_inner =
        fuse && c->inner_fuse && beta <= 8 && row_inner_supported(lg) && rs.n_passes == 2 && rs.radix[0] == 4;
    const bool fold = rot && fuse_inner;
    if (rot && !fold) {
        // both X^kappa images into the workspace
        timed(c, PK_AUTOMORPHISM, 8.0 * 4 * nl * n, 0,
              [&] { launch_automorphism_b(n, rot->src, 2 * level, ws, off_add0, rot->kappa, lg, c->stream); });
    }
    // d -> coefficient form at off_dcoef (the first pass reads d in place, or
    // through the permutation from rot->src; d stays in the NTT domain for
    // the inner product)
    {
        std::vector<NttJob> jobs;
        for (uint32_t z = 0; z < n; ++z) jobs.push_back(NttJob{ws.base + z * ws.stride + K.off_dcoef, 255u, 0u});
        if (fold) {
            NttEpilogue pe{};
            for (uint32_t z = 0; z < n; ++z) pe.perm_src[z] = rot->src.p[z] + nl;
            pe.kappa = rot->kappa;
            pe.kappa_inv = rot->kappa_inv;
            ntt_jobs(c, jobs, level, ~0u, true, 0, &pe, 0, ifuse_up ? 1u : 0u, ifuse_up);
        } else {
            ntt_jobs(c, jobs, level, ~0u, true, 0, nullptr, (int64_t)off_d - (int64_t)K.off_dcoef, ifuse_up ? 1u : 0u,
                     ifuse_up);
        }
    }
    // ModUp base conversion and the forward transforms of its rows
    {
        double rd = 0, wr = 0, macs = 0;
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t na = std::min(j * A + A, level) - j * A;
            rd += na;
            wr += rows - na;
            macs += (double)(rows - na) * na + na;
        }
        // method bytes: rows between two passes of a transform (the fused
        // conversion's inputs when it applies the inverse's last pass, its
        // outputs when it applies the forward's first) are layout cost
        if (fuse) {
            timed(c, PK_MODUP, 8.0 * N * (ifuse_up ? 0.0 : rd) * n, N * macs * n,
                  [&] {
                      launch_modup_col_b(n, ws, K.off_dcoef, K.off_ext, level, c->kc, c->tabs, lg, ifuse_up,
                                         c->stream);
                  },
                  64u + nkb + (ifuse_up ? 16u : 0u));
        } else {
            timed(c, PK_MODUP, 8.0 * N * (rd + wr) * n, N * macs * n, [&] {
                launch_modup_b(n, ws, K.off_dcoef, K.off_ext, level, c->kc, c->tabs, lg, c->bconv_mfma, c->stream);
            }, c->bconv_mfma ? nkb : 0);
        }
        if (fuse_inner) {
            // each launch (one per arithmetic kind of row) is timed on its own
            const uint64_t* c1[PFT_MAX_ITEMS] = {};
            if (fold)
                for (uint32_t z = 0; z < n; ++z) c1[z] = rot->src.p[z] + nl;
            auto inner = [&](hipStream_t st, uint32_t rows_sel) {
                launch_row_inner(n, ws, off_d, K.off_ext, K.off_acc, key.data, level, c->kc, c->tabs,
                                 c->fp_rows.data(), lg, c1, fold ? rot->kappa : 0, fold ? rot->kappa_inv : 0,
                                 c->inner_pairs, st, hook(c), rows_sel);
            };
            // on the context's own stream the 60-bit rows run on the helper
            // stream beside the fp64 rows, so that each launch fills the
            // other's tail; the helper's work is joined back before ModDown
            // (and before anything later reads the accumulators or the key).
            // While this family is being timed per launch the two run one
            // after the other, so that each launch's time is its own.
            const bool split = c->inner_st && c->stream == c->home && !c->prof.on(PK_KEY_INNER) &&
                               hipEventRecord(c->inner_fork, c->stream) == hipSuccess &&
                               hipStreamWaitEvent(c->inner_st, c->inner_fork, 0) == hipSuccess;
            if (split) {
                inner(c->inner_st, ROW_INNER_INT);
                inner(c->stream, ROW_INNER_FP);
                if (hipEventRecord(c->inner_join, c->inner_st) != hipSuccess ||
                    hipStreamWaitEvent(c->stream, c->inner_join, 0) != hipSuccess)
                    (void)hipStreamSynchronize(c->inner_st);  // last resort: never read unfinished rows
            } else {
                inner(c->stream, ROW_INNER_ALL);
            }
        } else {
            const uint32_t first = fuse ? 1u : 0u;
            if (!full.empty())
                ntt_jobs(c, full, rows - A, level, false, 0, nullptr, 0, first,
                         fuse && fwd_col16_restricted(c, (uint64_t)full.size() * (rows - A)));
            if (!last.empty())
                ntt_jobs(c, last, rows - na_last, level, false, 0, nullptr, 0, first,
                         fuse && fwd_col16_restricted(c, (uint64_t)last.size() * (rows - na_last)));
            // key inner product over level + K rows: the key is read once per
            // launch (shared by the batch); each item reads beta inputs and
            // writes two outputs per row
            const double key_once = beta <= 8 ? 1.0 : (double)n;
            timed(c, PK_KEY_INNER,
                  8.0 * N * ((double)beta * rows * n + 2.0 * beta * rows * key_once + 2.0 * rows * n),
                  2.0 * N * beta * rows * n, [&] {
                launch_key_inner_b(n, ws, off_d, K.off_ext, K.off_acc, key.data, level, c->kc, c->tabs, lg,
                                   c->stream);
            }, beta <= 8 ? beta : 0);
        }
    }
    // ModDown: the conversion of the special rows to the q-limbs is fused
    // with the first pass of conv's forward transform where its schedule
    // allows, and then also with the final pass of the special rows' inverse
    // transform (as for ModUp); the forward transform of conv finishes
    // ModDown in its final pass: out_b[i] = (acc_b[i] - conv_b[i]) P^-1 (+ add_b)
    const uint32_t down_kb = (P->K + 1) / 2;
    const bool fuse_down = c->bconv_mfma && c->bconv_fuse && lg >= 8 && down_kb <= 6 &&
                           first_pass_col16(c, 2ull * n * level);
    const bool ifuse_down = fuse_down && last_pass_col16(c, 2ull * n * P->K);
    // special rows of both accumulators to coefficient form
    {
        std::vector<NttJob> jobs;
        for (uint32_t z = 0; z < n; ++z)
            for (uint32_t b = 0; b < 2; ++b)
                jobs.push_back(NttJob{ws.base + z * ws.stride + K.off_acc + ((uint64_t)b * rows << lg), 0u, level});
        ntt_jobs(c, jobs, P->K, level, true, 0, nullptr, 0, ifuse_down ? 1u : 0u, ifuse_down);
    }
    if (fuse_down) {
        timed(c, PK_MODDOWN_CONV, 8.0 * N * (ifuse_down ? 0.0 : 2.0 * P->K) * n, 2.0 * N * P->K * level * n,
              [&] {
                  launch_moddown_col_b(n, ws, K.off_acc, K.off_conv, level, c->kc, c->tabs, lg, ifuse_down,
                                       c->stream);
              },
              64u + down_kb + (ifuse_down ? 16u : 0u));
    } else {
        timed(c, PK_MODDOWN_CONV, 8.0 * N * (2.0 * P->K + 2.0 * level) * n, 2.0 * N * P->K * level * n, [&] {
            launch_moddown_conv_b(n, ws, K.off_acc, K.off_conv, level, c->kc, c->tabs, lg, c->bconv_mfma, c->stream);
        }, c->bconv_mfma ? down_kb : 0);
    }
    {
        std::vector<NttJob> jobs;
        for (uint32_t z = 0; z < n; ++z)
            for (uint32_t b = 0; b < 2; ++b)
                jobs.push_back(NttJob{ws.base + z * ws.stride + K.off_conv + ((uint64_t)b * level << lg), 255u, 0u});
        NttEpilogue epi{};
        const uint64_t off_add[2] = {off_add0, off_add1};
        const uint64_t off_add2[2] = {off_add0b, PFT_NO_OFFSET};
        for (uint32_t b = 0; b < 2; ++b) {
            const int64_t conv0 = (int64_t)(K.off_conv + ((uint64_t)b * level << lg));
            epi.d_acc[b] = (int64_t)(K.off_acc + ((uint64_t)b * K.rows << lg)) - conv0;
            epi.d_add[b] = off_add[b] == PFT_NO_OFFSET ? PFT_EPI_NO_ADD : (int64_t)off_add[b] - conv0;
            epi.d_add2[b] = off_add2[b] == PFT_NO_OFFSET ? PFT_EPI_NO_ADD : (int64_t)off_add2[b] - conv0;
        }
        for (uint32_t z = 0; z < n; ++z) epi.out[z] = out.p[z];
        epi.pinv = c->kc.down_pinv;
        epi.pinv_fp = c->kc.down_pinv + P->L;
        epi.level = level;
        if (fold) {
            // the c0 image comes through the permutation in place of off_add0
            epi.d_add[0] = PFT_EPI_NO_ADD;
            for (uint32_t z = 0; z < n; ++z) epi.perm_src[z] = rot->src.p[z];
            epi.kappa = rot->kappa;
            epi.kappa_inv = rot->kappa_inv;
        }
        ntt_jobs(c, jobs, level, ~0u, false, 0, &epi, 0, fuse_down ? 1u : 0u,
                 fuse_down && fwd_col16_restricted(c, 2ull * n * level));
    }
}

// Items of one batched call grouped into launches of at most PFT_MAX_ITEMS
// ciphertexts of equal level.
template <typename F>
static int for_level_groups(uint32_t n, const pft_ct* in, F&& f) {
    std::vector<uint32_t> idx(n);
    for (uint32_t i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return in[x].level > in[y].level; });
    size_t s = 0;
    while (s < n) {
        size_t e = s;
        while (e < n && e - s < PFT_MAX_ITEMS && in[idx[e]].level == in[idx[s]].level) ++e;
        std::vector<uint32_t> grp(idx.begin() + s, idx.begin() + e);
        int r = f(grp);
        if (r) return r;
        s = e;
    }
    return PFT_OK;
}

extern "C" int pft_mul_relin(pft_ctx* c, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    return pft_mul_relin_batch(c, 1, a, b, out);
}

// HMUL + relinearisation of n pairs.  fixed: null, the context workspace
// (grown as needed); else a caller-provided device scratch of fixed_bytes:
// every level group's workspace must fit in it (checked before anything is
// enqueued; PFT_ENOMEM otherwise), and the NTT autotuner (which allocates)
// is not consulted for new batch classes.
static int mul_relin_core(pft_ctx* c, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out, uint64_t* fixed,
                          size_t fixed_bytes);

extern "C" int pft_mul_relin_batch(pft_ctx* c, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    return mul_relin_core(c, n, a, b, out, nullptr, 0);
}

extern "C" int pft_mul_relin_batch_noalloc(pft_ctx* c, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (!c->scratch) return fail(PFT_EHIP, "the fixed device scratch of device %d is not available", c->device);
    return mul_relin_core(c, n, a, b, out, c->scratch, PFT_NOALLOC_SCRATCH_BYTES);
}

static int mul_relin_core(pft_ctx* c, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out, uint64_t* fixed,
                          size_t fixed_bytes) {
    if (!c || !a || !b || !out) return fail(PFT_EINVAL, "null argument");
    if (!c->rlk_ok) return fail(PFT_ENOKEY, "no relinearisation key for the current secret");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &a[i])) || (r = check_ct(c, &b[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (a[i].level != b[i].level) return fail(PFT_ELEVEL, "HMUL needs equal levels");
        if (out[i].data == a[i].data || out[i].data == b[i].data) return fail(PFT_EINVAL, "output aliases an input");
    }
    const pft_params* P = c->P;
    if (fixed) {
        // every level group must fit the fixed scratch: refuse before any launch
        r = for_level_groups(n, a, [&](const std::vector<uint32_t>& g) -> int {
            const uint32_t l = a[g[0]].level;
            const size_t need = g.size() * ks_layout(P, l, 3ull * l * P->n).end * 8;
            if (need > fixed_bytes)
                return fail(PFT_ENOMEM,
                            "HMUL+relin of %zu ciphertexts at level %u needs %zu bytes of scratch, more than the "
                            "fixed %zu bytes",
                            g.size(), l, need, fixed_bytes);
            return PFT_OK;
        });
        if (r) return r;
    }
    struct NoTune {  // no autotuning (it allocates) while the fixed scratch is in use
        pft_ctx* c;
        bool was;
        ~NoTune() { c->ntt_tune = was; }
    } nt{c, c->ntt_tune};
    if (fixed) c->ntt_tune = false;
    return for_level_groups(n, a, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = a[g[0]].level, cnt = (uint32_t)g.size();
        const uint64_t nl = (uint64_t)l * P->n;
        const KsLayout K = ks_layout(P, l, 3 * nl);
        int rr;
        if (!fixed && (rr = ensure_ws(c, (size_t)cnt * K.end * 8))) return rr;
        const WsRef ws{fixed ? fixed : c->ws, K.end};
        ItemPtrs A{}, B{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            A.p[z] = a[g[z]].data;
            B.p[z] = b[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        timed(c, PK_TENSOR, 8.0 * nl * 7 * cnt, 4.0 * nl * cnt,
              [&] { launch_tensor_b(cnt, A, B, ws, 0, l, c->tabs, P->log_n, c->stream); });
        key_switch_b(c, cnt, ws, K, 2 * nl, c->rlk, 0, nl, O);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = a[g[z]].scale * b[g[z]].scale;
        }
        return PFT_OK;
    });
}

extern "C" int pft_rescale(pft_ctx* c, const pft_ct* in, uint32_t mode, pft_ct* out) {
    return pft_rescale_batch(c, 1, in, mode, out);
}

extern "C" int pft_rescale_batch(pft_ctx* c, uint32_t n, const pft_ct* in, uint32_t mode, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    if (mode == PFT_RESCALE_DEFAULT) mode = c->P->rescale_mode;
    if (mode > 1) return fail(PFT_EINVAL, "mode must be 0 (round), 1 (floor) or PFT_RESCALE_DEFAULT");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (in[i].level < 2) return fail(PFT_ELEVEL, "cannot rescale at level 1");
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (out[i].data == in[i].data) return fail(PFT_EINVAL, "rescale output aliases its input");
    }
    const pft_params* P = c->P;
    const uint32_t lg = P->log_n;
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        const uint64_t N = P->n;
        const uint64_t off_last = 0, off_tmp = 2 * N, words = 2 * N + 2 * (uint64_t)(l - 1) * N;
        int rr;
        if ((rr = ensure_ws(c, (size_t)cnt * words * 8))) return rr;
        const WsRef ws{c->ws, words};
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        // limb l-1 of both polynomials -> coefficient form
        launch_copy_rows_b(cnt, I, (uint64_t)(l - 1) * N, ws_items(ws, cnt), off_last, 1, lg, c->stream);
        launch_copy_rows_b(cnt, I, (uint64_t)(2 * l - 1) * N, ws_items(ws, cnt), off_last + N, 1, lg, c->stream);
        std::vector<NttJob> jl, jt;
        for (uint32_t z = 0; z < cnt; ++z)
            for (uint32_t b = 0; b < 2; ++b) {
                jl.push_back(NttJob{ws.base + z * ws.stride + off_last + b * N, 255u, 0u});
                jt.push_back(NttJob{ws.base + z * ws.stride + off_tmp + b * (l - 1) * N, 255u, 0u});
            }
        ntt_jobs(c, jl, 1, ~0u, true, l - 1);  // modulus of row 0 is q_{l-1}
        const double nd = (double)N;
        // the expansion applies the first pass of tmp's transform itself
        // where that schedule starts with a radix-16 column pass
        const bool fuse = lg >= 8 && first_pass_col16(c, (uint64_t)jt.size() * (l - 1));
        if (fuse)  // its rows leave after the first transform pass: layout cost
            timed(c, PK_RESCALE, 8.0 * nd * 2.0 * cnt, 0,
                  [&] { launch_rescale_col_b(cnt, ws, off_last, off_tmp, l, mode, c->tabs, lg, c->stream); }, 1u);
        else
            timed(c, PK_RESCALE, 8.0 * nd * (2.0 + 2.0 * (l - 1)) * cnt, 0,
                  [&] { launch_rescale_expand_b(cnt, ws, off_last, off_tmp, l, mode, c->tabs, lg, c->stream); });
        // the forward transform of tmp finishes in its final pass:
        // out[b][k] = (c[b][k] - tmp[b][k]) q_last^-1 mod q_k
        NttEpilogue epi{};
        for (uint32_t b = 0; b < 2; ++b) {
            epi.d_acc[b] = PFT_EPI_ITEM_ACC;
            epi.d_add[b] = epi.d_add2[b] = PFT_EPI_NO_ADD;
        }
        for (uint32_t z = 0; z < cnt; ++z) {
            epi.out[z] = O.p[z];
            epi.acc_item[z] = I.p[z];
        }
        epi.acc_level = l;
        epi.level = l - 1;
        epi.pinv = c->rescale_qinv + (size_t)(l - 1) * P->L;
        epi.pinv_fp = c->rescale_qinv + (size_t)P->L * P->L + (size_t)(l - 1) * P->L;
        ntt_jobs(c, jt, l - 1, ~0u, false, 0, &epi, 0, fuse ? 1u : 0u,
                 fuse && fwd_col16_restricted(c, (uint64_t)jt.size() * (l - 1)));
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l - 1;
            out[g[z]].scale = in[g[z]].scale / (double)P->q[l - 1];
        }
        return PFT_OK;
    });
}

static bool has_rot(pft_ctx* c, int32_t step) { return c->rot.count(norm_step(step, c->P->n)) != 0; }

// The rotation key for `step`, made resident first under a limited key
// cache (a miss copies the pinned host copy into a slot; the context stream
// waits for it; with a limited cache nothing is captured).  With a plan, the
// next key of the plan is then copied in ahead of its use.  The context
// stream is noted as a reader of the key's slot.  Null with *err set if the
// key is missing or cannot be made resident.
static const SwitchKeyDev* use_rot(pft_ctx* c, int32_t step, int* err) {
    const int32_t ns = norm_step(step, c->P->n);
    auto it = c->rot.find(ns);
    if (it == c->rot.end()) {
        *err = fail(PFT_ENOKEY, "no rotation key for step %d", step);
        return nullptr;
    }
    SwitchKeyDev& k = it->second;
    if (!c->rot_cache_max) return &k;
    if (c->capturing) {
        // a replay would read whatever key then occupies the slot
        *err = fail(PFT_EINVAL, "rotations cannot be captured while the rotation-key cache is limited");
        return nullptr;
    }
    const size_t d = plan_next_use(c, ns);
    if (d != SIZE_MAX) c->rot_plan_pos = (c->rot_plan_pos + d + 1) % c->rot_plan.size();
    int r;
    if (k.data) {
        ++c->rot_hits;
    } else {
        bool copied;
        if ((r = key_fill(c, ns, INT32_MIN, &copied))) {
            *err = r;
            return nullptr;
        }
        ++c->rot_misses;
    }
    k.last_use = ++c->rot_clock;
    pft_ctx::SlotSync& ss = c->rot_sync[k.slot];
    if (ss.ready_pending && hipStreamWaitEvent(c->stream, ss.ready, 0) != hipSuccess) {
        *err = fail(PFT_EHIP, "rotation key upload: %s", hipGetErrorString(hipGetLastError()));
        return nullptr;
    }
    if (std::find(ss.readers.begin(), ss.readers.end(), c->stream) == ss.readers.end())
        ss.readers.push_back(c->stream);
    if (!c->rot_plan.empty()) {
        // copy the plan's next key in while this rotation runs
        const int32_t nxt = c->rot_plan[c->rot_plan_pos];
        auto jt = c->rot.find(nxt);
        if (jt != c->rot.end() && !jt->second.data) {
            bool copied;
            if ((r = key_fill(c, nxt, ns, &copied))) {
                *err = r;
                return nullptr;
            }
            if (copied) ++c->rot_prefetches;
        }
    }
    return &k;
}

extern "C" int pft_rotate(pft_ctx* c, const pft_ct* in, int32_t step, pft_ct* out) {
    return pft_rotate_batch(c, 1, in, step, out);
}

extern "C" int pft_rotate_batch(pft_ctx* c, uint32_t n, const pft_ct* in, int32_t step, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    const bool identity = norm_step(step, c->P->n) == 0;
    if (!identity && !has_rot(c, step)) return fail(PFT_ENOKEY, "no rotation key for step %d", step);
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (out[i].data == in[i].data) return fail(PFT_EINVAL, "rotate output aliases its input");
    }
    if (identity) {
        // a rotation by a multiple of N/2 slots leaves every slot in place
        // (kappa = 1): the input itself, no key switch
        return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
            const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
            ItemPtrs I{}, O{};
            for (uint32_t z = 0; z < cnt; ++z) {
                I.p[z] = in[g[z]].data;
                O.p[z] = out[g[z]].data;
            }
            launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, c->P->log_n, c->stream);
            for (uint32_t z = 0; z < cnt; ++z) {
                out[g[z]].level = l;
                out[g[z]].scale = in[g[z]].scale;
            }
            return PFT_OK;
        });
    }
    const SwitchKeyDev* key = use_rot(c, step, &r);
    if (!key) return r;
    const pft_params* P = c->P;
    const uint64_t kappa = galois_element(step, P->n), kappa_inv = galois_inverse(kappa, P->n);
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        const uint64_t nl = (uint64_t)l * P->n;
        const KsLayout K = ks_layout(P, l, 2 * nl);
        int rr;
        if ((rr = ensure_ws(c, (size_t)cnt * K.end * 8))) return rr;
        const WsRef ws{c->ws, K.end};
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        KsRot kr{kappa, kappa_inv, I};
        key_switch_b(c, cnt, ws, K, nl, *key, 0, PFT_NO_OFFSET, O, PFT_NO_OFFSET, &kr);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = in[g[z]].scale;
        }
        return PFT_OK;
    });
}

extern "C" int pft_total_sum(pft_ctx* c, const pft_ct* in, uint32_t n_slots, pft_ct* out) {
    return pft_total_sum_batch(c, 1, in, n_slots, out);
}

// Rotation by `step` built from power-of-two rotations (the cost model of the
// paper's ROTATE: one automorphism and key switch per set bit of the step):
// r = step mod N/2, then for every set bit k of r, ascending, ct <- ROTATE(ct,
// 2^k) with the key for 2^k.  Two ciphertext regions of the workspace
// alternate as source and destination.
extern "C" int pft_rotate_pow2_batch(pft_ctx* c, uint32_t n, const pft_ct* in, int32_t step, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
    }
    const pft_params* P = c->P;
    const uint32_t half = P->n / 2;
    const uint32_t rr0 = (uint32_t)(((int64_t)step % (int64_t)half + half) % half);
    for (uint32_t k = 0; (1u << k) < half; ++k)
        if (((rr0 >> k) & 1u) && !has_rot(c, (int32_t)(1u << k)))
            return fail(PFT_ENOKEY, "no rotation key for step %u", 1u << k);
    const uint32_t lg = P->log_n;
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        const uint64_t nl = (uint64_t)l * P->n;
        const uint64_t offs[2] = {0, 2 * nl};
        const KsLayout K = ks_layout(P, l, 4 * nl);
        int e;
        if ((e = ensure_ws(c, (size_t)cnt * K.end * 8))) return e;
        const WsRef ws{c->ws, K.end};
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        launch_copy_rows_b(cnt, I, 0, ws_items(ws, cnt), offs[0], 2 * l, lg, c->stream);
        uint32_t cur = 0;
        for (uint32_t k = 0; (1u << k) < half; ++k) {
            if (!((rr0 >> k) & 1u)) continue;
            const uint64_t src = offs[cur], dst = offs[1 - cur];
            const uint64_t kappa = galois_element((int32_t)(1u << k), P->n);
            int ke;
            const SwitchKeyDev* rk = use_rot(c, (int32_t)(1u << k), &ke);
            if (!rk) return ke;
            KsRot kr{kappa, galois_inverse(kappa, P->n), ws_items(ws, cnt, src)};
            key_switch_b(c, cnt, ws, K, dst + nl, *rk, dst, PFT_NO_OFFSET, ws_items(ws, cnt, dst), PFT_NO_OFFSET, &kr);
            cur = 1 - cur;
        }
        launch_copy_rows_b(cnt, ws_items(ws, cnt, offs[cur]), 0, O, 0, 2 * l, lg, c->stream);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = in[g[z]].scale;
        }
        return PFT_OK;
    });
}

extern "C" int pft_rotate_pow2(pft_ctx* c, const pft_ct* in, int32_t step, pft_ct* out) {
    return pft_rotate_pow2_batch(c, 1, in, step, out);
}

extern "C" int pft_total_sum_batch(pft_ctx* c, uint32_t n, const pft_ct* in, uint32_t n_slots, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
    }
    if (n_slots < 1 || n_slots > c->P->n / 2 || (n_slots & (n_slots - 1)))
        return fail(PFT_EINVAL, "n_slots must be a power of two <= N/2");
    for (uint32_t s = 1; s < n_slots; s <<= 1)
        if (!has_rot(c, (int32_t)s)) return fail(PFT_ENOKEY, "no rotation key for step %u", s);
    const pft_params* P = c->P;
    const uint32_t lg = P->log_n;
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        const uint64_t nl = (uint64_t)l * P->n;
        const uint64_t off_cur = 0, off_rot = 2 * nl;
        const KsLayout K = ks_layout(P, l, 4 * nl);
        int rr;
        if ((rr = ensure_ws(c, (size_t)cnt * K.end * 8))) return rr;
        const WsRef ws{c->ws, K.end};
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        launch_copy_rows_b(cnt, I, 0, ws_items(ws, cnt), off_cur, 2 * l, lg, c->stream);
        // the running sum alternates between the two regions: the step reads
        // one (its X^kappa image and itself) and writes the other
        uint64_t a = off_cur, b = off_rot;
        for (uint32_t s = 1; s < n_slots; s <<= 1) {
            // cur + ROTATE(cur, s)   (Alg. 2): (cur0 + kappa(cur0) + ks0, cur1 + ks1),
            // finished by the ModDown epilogue into the other region
            const uint64_t kappa = galois_element((int32_t)s, P->n);
            int ke;
            const SwitchKeyDev* rk = use_rot(c, (int32_t)s, &ke);
            if (!rk) return ke;
            KsRot kr{kappa, galois_inverse(kappa, P->n), ws_items(ws, cnt, a)};
            key_switch_b(c, cnt, ws, K, b + nl, *rk, b, a + nl, ws_items(ws, cnt, b), a, &kr);
            std::swap(a, b);
        }
        launch_copy_rows_b(cnt, ws_items(ws, cnt, a), 0, O, 0, 2 * l, lg, c->stream);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = in[g[z]].scale;
        }
        return PFT_OK;
    });
}

// ---------------------------------------------------------------------------
// constant multiplication and PtMatVec (Sec. 4.1: v H and h O by HMULPLAIN,
// HADD and ROTATE; diagonal method in baby-step/giant-step form)
// ---------------------------------------------------------------------------
static int64_t round_half_away(double x) { return (int64_t)(x >= 0 ? std::floor(x + 0.5) : -std::floor(-x + 0.5)); }

extern "C" int pft_mul_const_batch(pft_ctx* c, uint32_t n, const pft_ct* in, const double* values, pft_ct* out) {
    if (!c || !in || !values || !out) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "mul_const copies host constants and cannot be captured");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (!(std::fabs(values[i]) < 4.0)) return fail(PFT_EINVAL, "constant must satisfy |value| < 4");
    }
    const pft_params* P = c->P;
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        const double qs = (double)P->q[l - 1];
        std::vector<TwPair> consts((size_t)cnt * l);
        for (uint32_t z = 0; z < cnt; ++z) {
            const int64_t m = round_half_away(values[g[z]] * qs);
            for (uint32_t i = 0; i < l; ++i) {
                const uint64_t q = P->q[i];
                const uint64_t v = m >= 0 ? (uint64_t)m % q : (q - ((0ull - (uint64_t)m) % q)) % q;
                consts[(size_t)z * l + i] = pair(v, q);
            }
        }
        if (c->cbuf_n < consts.size()) {
            HIPCK(hipStreamSynchronize(c->stream));
            dev_free(c, c->cbuf);
            c->cbuf = nullptr;
            c->cbuf_n = 0;
            void* v = nullptr;
            int rr = dev_alloc(c, &v, consts.size() * sizeof(TwPair), "constant buffer");
            if (rr) return rr;
            c->cbuf = (TwPair*)v;
            c->cbuf_n = consts.size();
        }
        HIPCK(hipMemcpyAsync(c->cbuf, consts.data(), consts.size() * sizeof(TwPair), hipMemcpyHostToDevice,
                             c->stream));
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        launch_scale_const_b(cnt, I, O, c->cbuf, l, c->tabs, P->log_n, c->stream);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = in[g[z]].scale * qs;
        }
        return PFT_OK;
    });
}

extern "C" int pft_mul_const(pft_ctx* c, const pft_ct* in, double value, pft_ct* out) {
    return pft_mul_const_batch(c, 1, in, &value, out);
}

// Per-call constants [n][level] (pairs) into the context's constant buffer.
static int upload_consts(pft_ctx* c, const std::vector<TwPair>& consts) {
    if (c->cbuf_n < consts.size()) {
        HIPCK(hipStreamSynchronize(c->stream));
        dev_free(c, c->cbuf);
        c->cbuf = nullptr;
        c->cbuf_n = 0;
        void* v = nullptr;
        int r = dev_alloc(c, &v, consts.size() * sizeof(TwPair), "constant buffer");
        if (r) return r;
        c->cbuf = (TwPair*)v;
        c->cbuf_n = consts.size();
    }
    HIPCK(hipMemcpyAsync(c->cbuf, consts.data(), consts.size() * sizeof(TwPair), hipMemcpyHostToDevice, c->stream));
    return PFT_OK;
}

extern "C" int pft_add_const_batch(pft_ctx* c, uint32_t n, const pft_ct* in, const double* values, pft_ct* out) {
    if (!c || !in || !values || !out) return fail(PFT_EINVAL, "null argument");
    if (c->capturing) return fail(PFT_EINVAL, "add_const copies host constants and cannot be captured");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (!(std::fabs(values[i] * in[i].scale) < 4611686018427387904.0))
            return fail(PFT_EINVAL, "constant times scale must stay below 2^62 in magnitude");
    }
    const pft_params* P = c->P;
    return for_level_groups(n, in, [&](const std::vector<uint32_t>& g) -> int {
        const uint32_t l = in[g[0]].level, cnt = (uint32_t)g.size();
        std::vector<TwPair> consts((size_t)cnt * l);
        for (uint32_t z = 0; z < cnt; ++z) {
            const int64_t m = round_half_away(values[g[z]] * in[g[z]].scale);
            for (uint32_t i = 0; i < l; ++i) {
                const uint64_t q = P->q[i];
                const uint64_t v = m >= 0 ? (uint64_t)m % q : (q - ((0ull - (uint64_t)m) % q)) % q;
                consts[(size_t)z * l + i] = TwPair{v, 0};
            }
        }
        int rr;
        if ((rr = upload_consts(c, consts))) return rr;
        ItemPtrs I{}, O{};
        for (uint32_t z = 0; z < cnt; ++z) {
            I.p[z] = in[g[z]].data;
            O.p[z] = out[g[z]].data;
        }
        launch_add_const_b(cnt, I, O, c->cbuf, l, c->tabs, P->log_n, c->stream);
        for (uint32_t z = 0; z < cnt; ++z) {
            out[g[z]].level = l;
            out[g[z]].scale = in[g[z]].scale;
        }
        return PFT_OK;
    });
}

extern "C" int pft_add_const(pft_ctx* c, const pft_ct* in, double value, pft_ct* out) {
    return pft_add_const_batch(c, 1, in, &value, out);
}

struct pft_ptmat {
    pft_ctx* ctx = nullptr;
    uint32_t n_o = 0, n_i = 0, n_in = 0, level = 0, b = 0, G = 0;
    double pt_scale = 0;
    uint64_t* pt = nullptr;  // [G][n_in * b][level][N], NTT domain, times 2^64 mod q
    std::vector<int64_t> coeffs;  // host [n_in][G][b][N]: the integer plaintexts, for the plan export
};

// Baby-step count b (a power of two dividing n_o) that minimises the key
// switches of one product, n_in (b - 1) baby rotations of the inputs plus
// G - 1 giant rotations of the partial sums (G = n_o / b); ties go to the
// larger b.  For n_in = 1 this is b = 2^ceil(log2(n_o)/2).
static void bsgs_plan(uint32_t n_o, uint32_t n_in, uint32_t* b, uint32_t* G) {
    uint64_t best = ~0ull;
    for (uint32_t bb = 1; bb <= n_o; bb <<= 1) {
        const uint64_t cost = (uint64_t)n_in * (bb - 1) + (n_o / bb - 1);
        if (cost <= best) {
            best = cost;
            *b = bb;
        }
    }
    *G = n_o / *b;
}

static int ptmat_check(const pft_ctx* c, uint32_t n_o, uint32_t n_i, uint32_t n_in, uint32_t level) {
    const uint32_t t = c->P->n / 2;
    if (!n_o || (n_o & (n_o - 1)) || !n_i || (n_i & (n_i - 1)) || n_i > t || n_o > n_i)
        return fail(PFT_EINVAL, "need powers of two n_o <= n_i <= N/2");
    if (n_in < 1 || n_in > 4096) return fail(PFT_EINVAL, "n_in must be in 1..4096");
    if (level < 2 || level > c->P->L) return fail(PFT_ELEVEL, "plaintext matrix level must be in 2..L");
    return PFT_OK;
}

// coeffs: [n_in][G][b][N] integer plaintexts of the pre-rotated diagonals.
static int ptmat_upload(pft_ctx* c, pft_ptmat* m, const int64_t* coeffs) {
    const pft_params* P = c->P;
    const uint32_t J = m->n_in * m->b, l = m->level;
    const size_t N = P->n, words = (size_t)m->G * J * l * N;
    int r;
    if ((r = dalloc(c, &m->pt, words * 8))) return r;
    if ((r = ensure_ws(c, (size_t)J * N * 8))) return r;
    for (uint32_t g = 0; g < m->G; ++g) {
        for (uint32_t cc = 0; cc < m->n_in; ++cc)
            for (uint32_t rr = 0; rr < m->b; ++rr) {
                const int64_t* src = coeffs + (((size_t)cc * m->G + g) * m->b + rr) * N;
                if ((r = upload_i64(c, (int64_t*)c->ws + ((size_t)cc * m->b + rr) * N, src, N))) return r;
            }
        uint64_t* dst = m->pt + (size_t)g * J * l * N;
        for (uint32_t j0 = 0; j0 < J; j0 += PFT_SMALL_POLYS) {
            const uint32_t nj = std::min<uint32_t>(PFT_SMALL_POLYS, J - j0);
            SmallBatch out = sb_rows(P, dst + (size_t)j0 * l * N, nj, l, l);
            launch_int_to_rns((const int64_t*)c->ws + (size_t)j0 * N, out, c->tabs, P->log_n, c->stream);
            launch_mul_const(out, out, c->to_mont, c->tabs, P->log_n, c->stream);  // [0, q) kept; NTT below
        }
        ntt_rows(c, dst, J, l, l, false);
        HIPCK(hipStreamSynchronize(c->stream));  // the staged host rows are reused for the next g
    }
    return PFT_OK;
}

extern "C" int pft_ptmat_create_from_coeffs(pft_ctx* c, const int64_t* coeffs, uint32_t n_o, uint32_t n_i,
                                            uint32_t n_in, uint32_t level, double pt_scale, pft_ptmat** out) {
    if (!c || !coeffs || !out) return fail(PFT_EINVAL, "null argument");
    int r;
    if ((r = ptmat_check(c, n_o, n_i, n_in, level))) return r;
    auto* m = new pft_ptmat();
    m->ctx = c;
    m->n_o = n_o;
    m->n_i = n_i;
    m->n_in = n_in;
    m->level = level;
    m->pt_scale = pt_scale;
    bsgs_plan(n_o, n_in, &m->b, &m->G);
    if ((r = ptmat_upload(c, m, coeffs))) {
        delete m;
        return r;
    }
    m->coeffs.assign(coeffs, coeffs + (size_t)n_in * m->G * m->b * c->P->n);
    *out = m;
    return PFT_OK;
}

// The operations of one document's PtMatVec in the order pft_ptmatvec runs
// them (see pft_ptmat_plan in pft.h for the register convention).
static std::vector<pft_op> ptmat_plan_ops(uint32_t n_o, uint32_t n_i, uint32_t n_in) {
    uint32_t b, G;
    bsgs_plan(n_o, n_in, &b, &G);
    std::vector<pft_op> ops;
    auto baby = [&](uint32_t cc, uint32_t rr) { return rr == 0 ? cc : n_in + cc * (b - 1) + (rr - 1); };
    const uint32_t prod = n_in + n_in * (b - 1), acc = prod + 1, tmp = prod + 2, tot = prod + 3;
    auto op = [&](uint32_t kind, uint32_t a, uint32_t bb, uint32_t out, int32_t step) {
        ops.push_back(pft_op{kind, a, bb, out, step, 0});
    };
    for (uint32_t rr = 1; rr < b; ++rr)
        for (uint32_t cc = 0; cc < n_in; ++cc) op(PFT_OP_ROTATE, cc, 0, baby(cc, rr), (int32_t)rr);
    for (uint32_t g = 0; g < G; ++g) {
        const uint32_t sum = g == 0 ? tot : acc;
        bool first = true;
        for (uint32_t cc = 0; cc < n_in; ++cc)
            for (uint32_t rr = 0; rr < b; ++rr) {
                const uint32_t diag = (cc * G + g) * b + rr;
                op(PFT_OP_MUL_PLAIN, baby(cc, rr), diag, first ? sum : prod, 0);
                if (!first) op(PFT_OP_ADD, sum, prod, sum, 0);
                first = false;
            }
        if (g == 0) continue;
        op(PFT_OP_ROTATE, acc, 0, tmp, (int32_t)(g * b));
        op(PFT_OP_ADD, tot, tmp, tot, 0);
    }
    for (uint32_t st = n_o; st < n_i; st <<= 1) {
        op(PFT_OP_ROTATE, tot, 0, tmp, (int32_t)st);
        op(PFT_OP_ADD, tot, tmp, tot, 0);
    }
    return ops;
}

static int copy_plan(const std::vector<pft_op>& ops, pft_op* out, uint32_t max_ops, uint32_t* n_ops) {
    if (n_ops) *n_ops = (uint32_t)ops.size();
    if (out)
        for (size_t i = 0; i < ops.size() && i < max_ops; ++i) out[i] = ops[i];
    return PFT_OK;
}

extern "C" int pft_ptmat_plan(uint32_t n_o, uint32_t n_i, uint32_t n_in, pft_op* ops, uint32_t max_ops,
                              uint32_t* n_ops) {
    if (!n_o || (n_o & (n_o - 1)) || !n_i || (n_i & (n_i - 1)) || n_o > n_i)
        return fail(PFT_EINVAL, "need powers of two n_o <= n_i");
    if (n_in < 1 || n_in > 4096) return fail(PFT_EINVAL, "n_in must be in 1..4096");
    return copy_plan(ptmat_plan_ops(n_o, n_i, n_in), ops, max_ops, n_ops);
}

extern "C" int pft_ptmat_plan_export(const pft_ptmat* m, pft_op* ops, uint32_t max_ops, uint32_t* n_ops,
                                     int64_t* diag_coeffs) {
    if (!m) return fail(PFT_EINVAL, "null matrix");
    if (diag_coeffs) std::copy(m->coeffs.begin(), m->coeffs.end(), diag_coeffs);
    return copy_plan(ptmat_plan_ops(m->n_o, m->n_i, m->n_in), ops, max_ops, n_ops);
}

extern "C" int pft_diagonals_encode(const pft_params* P, const double* M, uint32_t n_o, uint32_t n_i, uint32_t n_in,
                                    double scale, int64_t* out) {
    if (!P || !M || !out) return fail(PFT_EINVAL, "null argument");
    const uint32_t t = P->n / 2, cols = n_in * n_i;
    if (!n_o || (n_o & (n_o - 1)) || !n_i || (n_i & (n_i - 1)) || n_i > t || n_o > n_i)
        return fail(PFT_EINVAL, "need powers of two n_o <= n_i <= N/2");
    if (n_in < 1) return fail(PFT_EINVAL, "n_in must be at least 1");
    uint32_t b, G;
    bsgs_plan(n_o, n_in, &b, &G);
    std::vector<double> diag(t), zero(t, 0.0);
    int r;
    for (uint32_t cc = 0; cc < n_in; ++cc)
        for (uint32_t g = 0; g < G; ++g)
            for (uint32_t rr = 0; rr < b; ++rr) {
                const uint32_t i = g * b + rr;
                // P^c_{g,r}[k] = D^c_i[(k - g b) mod t], D^c_i[k] = M[k mod n_o][c n_i + (k + i) mod n_i]
                for (uint32_t k = 0; k < t; ++k) {
                    const uint32_t kk = (k + t - (g * b) % t) % t;
                    diag[k] = M[(size_t)(kk % n_o) * cols + (size_t)cc * n_i + (kk + i) % n_i];
                }
                int64_t* dst = out + (((size_t)cc * G + g) * b + rr) * P->n;
                if ((r = pft_encode(P, diag.data(), zero.data(), t, scale, dst))) return r;
            }
    return PFT_OK;
}

extern "C" int pft_ptmat_create(pft_ctx* c, const double* M, uint32_t n_o, uint32_t n_i, uint32_t n_in,
                                uint32_t level, pft_ptmat** out) {
    if (!c || !M || !out) return fail(PFT_EINVAL, "null argument");
    int r;
    if ((r = ptmat_check(c, n_o, n_i, n_in, level))) return r;
    const pft_params* P = c->P;
    uint32_t b, G;
    bsgs_plan(n_o, n_in, &b, &G);
    const double pt_scale = (double)P->q[level - 1];
    std::vector<int64_t> coeffs((size_t)n_in * G * b * P->n);
    if ((r = pft_diagonals_encode(P, M, n_o, n_i, n_in, pt_scale, coeffs.data()))) return r;
    return pft_ptmat_create_from_coeffs(c, coeffs.data(), n_o, n_i, n_in, level, pt_scale, out);
}

extern "C" void pft_ptmat_destroy(pft_ptmat* m) { delete m; }  // device rows are freed with the context

extern "C" int pft_ptmat_info(const pft_ptmat* m, uint32_t* info) {
    if (!m || !info) return fail(PFT_EINVAL, "null argument");
    info[0] = m->n_o;
    info[1] = m->n_i;
    info[2] = m->n_in;
    info[3] = m->level;
    info[4] = m->b;
    info[5] = m->G;
    return PFT_OK;
}

static std::vector<uint32_t> ptmat_steps(const pft_ptmat* m) {
    std::vector<uint32_t> st;
    for (uint32_t r = 1; r < m->b; ++r) st.push_back(r);
    for (uint32_t g = 1; g < m->G; ++g) st.push_back(g * m->b);
    for (uint32_t s = m->n_o; s < m->n_i; s <<= 1) st.push_back(s);
    return st;
}

static std::vector<pft_ct> cts_at(uint64_t* base, size_t stride, uint64_t off, uint32_t n, uint32_t level,
                                  double scale) {
    std::vector<pft_ct> v(n);
    for (uint32_t z = 0; z < n; ++z) v[z] = pft_ct{base + z * stride + off, level, 0, scale};
    return v;
}

extern "C" int pft_ptmatvec(pft_ctx* c, const pft_ptmat* m, uint32_t n_docs, const pft_ct* in, pft_ct* out) {
    if (!c || !m || !in || !out) return fail(PFT_EINVAL, "null argument");
    if (m->ctx != c) return fail(PFT_EINVAL, "plaintext matrix belongs to another context");
    const pft_params* P = c->P;
    const uint32_t l = m->level, J = m->n_in * m->b, lg = P->log_n;
    int r;
    for (uint32_t z = 0; z < n_docs; ++z) {
        if (!out[z].data) return fail(PFT_EINVAL, "null output");
        for (uint32_t cc = 0; cc < m->n_in; ++cc) {
            const pft_ct& x = in[(size_t)z * m->n_in + cc];
            if ((r = check_ct(c, &x))) return r;
            if (x.level != l) return fail(PFT_ELEVEL, "input level %u differs from the matrix level %u", x.level, l);
            if (!scales_match(x.scale, in[0].scale)) return fail(PFT_ESCALE, "inputs need equal scales");
        }
    }
    for (uint32_t st : ptmat_steps(m))
        if (!has_rot(c, (int32_t)st)) return fail(PFT_ENOKEY, "no rotation key for step %u", st);
    if (n_docs == 0) return PFT_OK;
    const double scale = in[0].scale;
    const uint64_t ct_words = 2ull * l * P->n;
    // per document: baby[n_in][b] | acc[G] (acc[0] collects the total) | tmp
    const uint64_t off_baby = 0, off_acc = (uint64_t)J * ct_words, off_tot = off_acc,
                   off_tmp = off_acc + (uint64_t)m->G * ct_words, stride = off_tmp + ct_words;
    if ((r = ensure_aux(c, (size_t)n_docs * stride * 8))) return r;
    uint64_t* A = c->aux;
    // inputs -> baby[c][0]
    for (uint32_t z0 = 0; z0 < n_docs * m->n_in; z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = std::min<uint32_t>(PFT_MAX_ITEMS, n_docs * m->n_in - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            const uint32_t z = (z0 + u) / m->n_in, cc = (z0 + u) % m->n_in;
            I.p[u] = in[z0 + u].data;
            O.p[u] = A + z * stride + off_baby + (uint64_t)cc * m->b * ct_words;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    // baby steps: baby[c][r] = ROTATE(baby[c][0], r)
    for (uint32_t rr = 1; rr < m->b; ++rr) {
        std::vector<pft_ct> src, dst;
        for (uint32_t z = 0; z < n_docs; ++z)
            for (uint32_t cc = 0; cc < m->n_in; ++cc) {
                const uint64_t base = z * stride + off_baby + (uint64_t)cc * m->b * ct_words;
                src.push_back(pft_ct{A + base, l, 0, scale});
                dst.push_back(pft_ct{A + base + rr * ct_words, l, 0, scale});
            }
        if ((r = pft_rotate_batch(c, (uint32_t)src.size(), src.data(), (int32_t)rr, dst.data()))) return r;
    }
    // giant steps: tot = sum_g ROTATE(acc[g], g b), acc[g] = sum_{c,r} P_{g,c,r}
    // baby[c][r]; the inner sums of several giant steps come from one pass
    // over the baby steps
    const uint32_t gt = pt_dot_multi_steps();
    for (uint32_t g0 = 0; g0 < m->G; g0 += gt) {
        const uint32_t n_g = std::min(gt, m->G - g0);
        const uint64_t* ptg = m->pt + (size_t)g0 * J * l * P->n;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 1024) {
            const uint32_t cnt = std::min<uint32_t>(1024, n_docs - z0);
            const WsRef w{A + z0 * stride, stride};
            timed(c, PK_ELEMENTWISE,
                  8.0 * (double)cnt * ct_words * (J + n_g) + 8.0 * (double)n_g * J * l * P->n,
                  (double)cnt * ct_words * J * n_g, [&] {
                      launch_pt_dot_multi_b(cnt, w, off_baby, ct_words, ptg, J, n_g, off_acc + g0 * ct_words, l,
                                            c->tabs, lg, c->stream);
                  });
        }
    }
    for (uint32_t g = 1; g < m->G; ++g) {
        std::vector<pft_ct> src = cts_at(A, stride, off_acc + g * ct_words, n_docs, l, scale * m->pt_scale);
        std::vector<pft_ct> dst = cts_at(A, stride, off_tmp, n_docs, l, scale * m->pt_scale);
        if ((r = pft_rotate_batch(c, n_docs, src.data(), (int32_t)(g * m->b), dst.data()))) return r;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 65535) {
            const uint32_t cnt = std::min<uint32_t>(65535, n_docs - z0);
            launch_add_ct_b(cnt, WsRef{A + z0 * stride, stride}, off_tot, off_tmp, off_tot, l, c->tabs, lg, c->stream);
        }
    }
    // rotate-and-sum over the n_i / n_o blocks
    for (uint32_t s = m->n_o; s < m->n_i; s <<= 1) {
        std::vector<pft_ct> src = cts_at(A, stride, off_tot, n_docs, l, scale * m->pt_scale);
        std::vector<pft_ct> dst = cts_at(A, stride, off_tmp, n_docs, l, scale * m->pt_scale);
        if ((r = pft_rotate_batch(c, n_docs, src.data(), (int32_t)s, dst.data()))) return r;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 65535) {
            const uint32_t cnt = std::min<uint32_t>(65535, n_docs - z0);
            launch_add_ct_b(cnt, WsRef{A + z0 * stride, stride}, off_tot, off_tmp, off_tot, l, c->tabs, lg, c->stream);
        }
    }
    for (uint32_t z0 = 0; z0 < n_docs; z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = std::min<uint32_t>(PFT_MAX_ITEMS, n_docs - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            I.p[u] = A + (z0 + u) * stride + off_tot;
            O.p[u] = out[z0 + u].data;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    for (uint32_t z = 0; z < n_docs; ++z) {
        out[z].level = l;
        out[z].scale = scale * m->pt_scale;
    }
    return PFT_OK;
}

// ---- encrypted-weight matrix-vector product (Sec. 4.2) --------------------
extern "C" int pft_ctmatvec(pft_ctx* c, uint32_t n_o, uint32_t n_i, uint32_t n_in, const pft_ct* diags,
                            uint32_t n_docs, const pft_ct* in, pft_ct* out) {
    if (!c || !diags || !in || !out) return fail(PFT_EINVAL, "null argument");
    if (!c->rlk_ok) return fail(PFT_ENOKEY, "no relinearisation key for the current secret");
    const pft_params* P = c->P;
    const uint32_t t = P->n / 2;
    if (!n_o || (n_o & (n_o - 1)) || !n_i || (n_i & (n_i - 1)) || n_i > t || n_o > n_i)
        return fail(PFT_EINVAL, "need powers of two n_o <= n_i <= N/2");
    if (n_in < 1) return fail(PFT_EINVAL, "n_in must be at least 1");
    pft_ptmat plan;  // only the plan fields, for the rotation steps
    plan.n_o = n_o;
    plan.n_i = n_i;
    bsgs_plan(n_o, n_in, &plan.b, &plan.G);
    const uint32_t b = plan.b, G = plan.G, J = n_in * b;
    if (J > PFT_MAX_ITEMS) return fail(PFT_EINVAL, "n_in * b = %u exceeds %u diagonal terms per giant step", J,
                                       (unsigned)PFT_MAX_ITEMS);
    int r;
    const uint32_t nd = n_in * G * b;
    if ((r = check_ct(c, &diags[0]))) return r;
    const uint32_t l = diags[0].level;
    for (uint32_t j = 0; j < nd; ++j) {
        if ((r = check_ct(c, &diags[j]))) return r;
        if (diags[j].level != l) return fail(PFT_ELEVEL, "diagonals need equal levels");
        if (!scales_match(diags[j].scale, diags[0].scale)) return fail(PFT_ESCALE, "diagonals need equal scales");
    }
    for (uint32_t z = 0; z < n_docs; ++z) {
        if (!out[z].data) return fail(PFT_EINVAL, "null output");
        for (uint32_t cc = 0; cc < n_in; ++cc) {
            const pft_ct& x = in[(size_t)z * n_in + cc];
            if ((r = check_ct(c, &x))) return r;
            if (x.level != l) return fail(PFT_ELEVEL, "input level %u differs from the diagonals' level %u", x.level, l);
            if (!scales_match(x.scale, in[0].scale)) return fail(PFT_ESCALE, "inputs need equal scales");
        }
    }
    for (uint32_t st : ptmat_steps(&plan))
        if (!has_rot(c, (int32_t)st)) return fail(PFT_ENOKEY, "no rotation key for step %u", st);
    if (n_docs == 0) return PFT_OK;
    const double scale = in[0].scale * diags[0].scale;
    const uint32_t lg = P->log_n;
    const uint64_t nl = (uint64_t)l * P->n, ct_words = 2 * nl;
    // per document in aux: baby[n_in][b] | acc[G] (acc[0] collects the total) | tmp
    const uint64_t off_baby = 0, off_acc = (uint64_t)J * ct_words, off_tot = off_acc,
                   off_tmp = off_acc + (uint64_t)G * ct_words, stride = off_tmp + ct_words;
    if ((r = ensure_aux(c, (size_t)n_docs * stride * 8))) return r;
    // per document in ws: the summed tensor [3][l][N], then key switching
    const KsLayout K = ks_layout(P, l, 3 * nl);
    const uint32_t chunk = PFT_MAX_ITEMS;
    uint64_t* A = c->aux;
    for (uint32_t z0 = 0; z0 < n_docs * n_in; z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = std::min<uint32_t>(PFT_MAX_ITEMS, n_docs * n_in - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            const uint32_t z = (z0 + u) / n_in, cc = (z0 + u) % n_in;
            I.p[u] = in[z0 + u].data;
            O.p[u] = A + z * stride + off_baby + (uint64_t)cc * b * ct_words;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    const double in_scale = in[0].scale;
    for (uint32_t rr = 1; rr < b; ++rr) {
        std::vector<pft_ct> src, dst;
        for (uint32_t z = 0; z < n_docs; ++z)
            for (uint32_t cc = 0; cc < n_in; ++cc) {
                const uint64_t base = z * stride + off_baby + (uint64_t)cc * b * ct_words;
                src.push_back(pft_ct{A + base, l, 0, in_scale});
                dst.push_back(pft_ct{A + base + rr * ct_words, l, 0, in_scale});
            }
        if ((r = pft_rotate_batch(c, (uint32_t)src.size(), src.data(), (int32_t)rr, dst.data()))) return r;
    }
    // the tensor sums of several giant steps from one pass over the baby
    // steps, each giant step then relinearised into acc[g]
    const uint32_t gt = std::max(1u, std::min(ct_dot_multi_steps(), (uint32_t)PFT_MAX_ITEMS / J));
    for (uint32_t g0 = 0; g0 < G; g0 += gt) {
        const uint32_t n_g = std::min(gt, G - g0);
        ItemPtrs E{};
        for (uint32_t g = 0; g < n_g; ++g)
            for (uint32_t cc = 0; cc < n_in; ++cc)
                for (uint32_t rr = 0; rr < b; ++rr)
                    E.p[g * J + cc * b + rr] = diags[((size_t)cc * G + g0 + g) * b + rr].data;
        // at most `chunk` key-switch items in the workspace, as one giant step at a time
        const uint32_t zc = std::max(1u, chunk / n_g);
        for (uint32_t z0 = 0; z0 < n_docs; z0 += zc) {
            const uint32_t cnt = std::min(zc, n_docs - z0);
            if ((r = ensure_ws(c, (size_t)n_g * cnt * K.end * 8))) return r;
            const WsRef ws{c->ws, K.end};
            timed(c, PK_TENSOR, 8.0 * cnt * (2.0 * J * ct_words + 3.0 * n_g * nl) + 8.0 * n_g * J * ct_words,
                  4.0 * cnt * n_g * J * nl, [&] {
                      launch_ct_dot_multi_b(cnt, E, J, n_g, WsRef{A + z0 * stride, stride}, off_baby, ct_words, ws, 0,
                                            l, c->to_mont, c->tabs, lg, c->stream);
                  });
            for (uint32_t g = 0; g < n_g; ++g) {
                ItemPtrs O{};
                for (uint32_t u = 0; u < cnt; ++u) O.p[u] = A + (z0 + u) * stride + off_acc + (g0 + g) * ct_words;
                key_switch_b(c, cnt, WsRef{c->ws + (size_t)g * cnt * K.end, K.end}, K, 2 * nl, c->rlk, 0, nl, O);
            }
        }
    }
    for (uint32_t g = 1; g < G; ++g) {
        std::vector<pft_ct> src = cts_at(A, stride, off_acc + g * ct_words, n_docs, l, scale);
        std::vector<pft_ct> dst = cts_at(A, stride, off_tmp, n_docs, l, scale);
        if ((r = pft_rotate_batch(c, n_docs, src.data(), (int32_t)(g * b), dst.data()))) return r;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 65535) {
            const uint32_t cnt = std::min<uint32_t>(65535, n_docs - z0);
            launch_add_ct_b(cnt, WsRef{A + z0 * stride, stride}, off_tot, off_tmp, off_tot, l, c->tabs, lg, c->stream);
        }
    }
    for (uint32_t s = n_o; s < n_i; s <<= 1) {
        std::vector<pft_ct> src = cts_at(A, stride, off_tot, n_docs, l, scale);
        std::vector<pft_ct> dst = cts_at(A, stride, off_tmp, n_docs, l, scale);
        if ((r = pft_rotate_batch(c, n_docs, src.data(), (int32_t)s, dst.data()))) return r;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 65535) {
            const uint32_t cnt = std::min<uint32_t>(65535, n_docs - z0);
            launch_add_ct_b(cnt, WsRef{A + z0 * stride, stride}, off_tot, off_tmp, off_tot, l, c->tabs, lg, c->stream);
        }
    }
    for (uint32_t z0 = 0; z0 < n_docs; z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = std::min<uint32_t>(PFT_MAX_ITEMS, n_docs - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            I.p[u] = A + (z0 + u) * stride + off_tot;
            O.p[u] = out[z0 + u].data;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    for (uint32_t z = 0; z < n_docs; ++z) {
        out[z].level = l;
        out[z].scale = scale;
    }
    return PFT_OK;
}

// ---- plaintext dot products with TotalSum (Sec. 4.1, column packing) ------
struct pft_ptdot {
    pft_ctx* ctx = nullptr;
    uint32_t n_out = 0, J = 0, level = 0;
    double pt_scale = 0;
    uint64_t* pt = nullptr;  // [n_out][J][level][N], NTT domain, times 2^64 mod q
};

extern "C" int pft_ptdot_create_from_coeffs(pft_ctx* c, const int64_t* coeffs, uint32_t n_out, uint32_t J,
                                            uint32_t level, double pt_scale, pft_ptdot** out) {
    if (!c || !coeffs || !out) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (!n_out || !J) return fail(PFT_EINVAL, "n_out and J must be positive");
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "plaintext level must be in 1..L");
    const size_t N = P->n;
    auto* m = new pft_ptdot();
    m->ctx = c;
    m->n_out = n_out;
    m->J = J;
    m->level = level;
    m->pt_scale = pt_scale;
    int r;
    if ((r = dalloc(c, &m->pt, (size_t)n_out * J * level * N * 8))) {
        delete m;
        return r;
    }
    // stage PFT_SMALL_POLYS integer polynomials at a time through ws
    if ((r = ensure_ws(c, (size_t)PFT_SMALL_POLYS * N * 8))) {
        delete m;
        return r;
    }
    const size_t total = (size_t)n_out * J;
    for (size_t j0 = 0; j0 < total; j0 += PFT_SMALL_POLYS) {
        const uint32_t nj = (uint32_t)std::min<size_t>(PFT_SMALL_POLYS, total - j0);
        if ((r = upload_i64(c, (int64_t*)c->ws, coeffs + j0 * N, (size_t)nj * N))) {
            delete m;
            return r;
        }
        uint64_t* dst = m->pt + j0 * level * N;
        SmallBatch sb = sb_rows(P, dst, nj, level, level);
        launch_int_to_rns((const int64_t*)c->ws, sb, c->tabs, P->log_n, c->stream);
        launch_mul_const(sb, sb, c->to_mont, c->tabs, P->log_n, c->stream);
        ntt_rows(c, dst, nj, level, level, false);
        HIPCK(hipStreamSynchronize(c->stream));  // the staged rows are reused next
    }
    *out = m;
    return PFT_OK;
}

extern "C" int pft_ptdot_create(pft_ctx* c, const double* slots, uint32_t n_out, uint32_t J, uint32_t level,
                                pft_ptdot** out) {
    if (!c || !slots || !out) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "plaintext level must be in 1..L");
    const uint32_t t = P->n / 2;
    const double pt_scale = (double)P->q[level - 1];
    std::vector<int64_t> coeffs((size_t)n_out * J * P->n);
    int r;
    for (size_t u = 0; u < (size_t)n_out * J; ++u)
        if ((r = pft_encode(P, slots + u * t, nullptr, t, pt_scale, coeffs.data() + u * P->n))) return r;
    return pft_ptdot_create_from_coeffs(c, coeffs.data(), n_out, J, level, pt_scale, out);
}

extern "C" void pft_ptdot_destroy(pft_ptdot* m) { delete m; }  // device rows are freed with the context

extern "C" int pft_ptdot_apply(pft_ctx* c, const pft_ptdot* m, uint32_t n_docs, const pft_ct* in, uint32_t n_sum,
                               pft_ct* out) {
    if (!c || !m || !in || !out) return fail(PFT_EINVAL, "null argument");
    if (m->ctx != c) return fail(PFT_EINVAL, "plaintexts belong to another context");
    const pft_params* P = c->P;
    if (!n_sum || (n_sum & (n_sum - 1)) || n_sum > P->n / 2)
        return fail(PFT_EINVAL, "n_sum must be a power of two <= N/2");
    const uint32_t l = m->level, J = m->J, K = m->n_out, lg = P->log_n;
    int r;
    for (size_t u = 0; u < (size_t)n_docs * J; ++u) {
        if ((r = check_ct(c, &in[u]))) return r;
        if (in[u].level != l) return fail(PFT_ELEVEL, "input level %u differs from the plaintext level %u",
                                          in[u].level, l);
        if (!scales_match(in[u].scale, in[0].scale)) return fail(PFT_ESCALE, "inputs need equal scales");
    }
    for (size_t u = 0; u < (size_t)n_docs * K; ++u)
        if (!out[u].data) return fail(PFT_EINVAL, "null output");
    for (uint32_t s = 1; s < n_sum; s <<= 1)
        if (!has_rot(c, (int32_t)s)) return fail(PFT_ENOKEY, "no rotation key for step %u", s);
    if (n_docs == 0) return PFT_OK;
    const double scale = in[0].scale * m->pt_scale;
    const uint64_t ct_words = 2ull * l * P->n;
    // per document in aux: inputs [J] | outputs [n_out]
    const uint64_t off_out = (uint64_t)J * ct_words, stride = off_out + (uint64_t)K * ct_words;
    if ((r = ensure_aux(c, (size_t)n_docs * stride * 8))) return r;
    uint64_t* A = c->aux;
    for (size_t z0 = 0; z0 < (size_t)n_docs * J; z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = (uint32_t)std::min<size_t>(PFT_MAX_ITEMS, (size_t)n_docs * J - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            const size_t z = (z0 + u) / J, j = (z0 + u) % J;
            I.p[u] = in[z0 + u].data;
            O.p[u] = A + z * stride + j * ct_words;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    // several outputs' sums from one pass over the inputs
    const uint32_t kt = pt_dot_multi_steps();
    for (uint32_t k0 = 0; k0 < K; k0 += kt) {
        const uint32_t nk = std::min(kt, K - k0);
        const uint64_t* ptk = m->pt + (size_t)k0 * J * l * P->n;
        for (uint32_t z0 = 0; z0 < n_docs; z0 += 1024) {
            const uint32_t cnt = std::min<uint32_t>(1024, n_docs - z0);
            timed(c, PK_ELEMENTWISE, 8.0 * (double)cnt * ct_words * (J + nk) + 8.0 * (double)nk * J * l * P->n,
                  (double)cnt * ct_words * J * nk, [&] {
                      launch_pt_dot_multi_b(cnt, WsRef{A + z0 * stride, stride}, 0, ct_words, ptk, J, nk,
                                            off_out + (uint64_t)k0 * ct_words, l, c->tabs, lg, c->stream);
                  });
        }
    }
    std::vector<pft_ct> res;
    res.reserve((size_t)n_docs * K);
    for (uint32_t z = 0; z < n_docs; ++z)
        for (uint32_t k = 0; k < K; ++k) res.push_back(pft_ct{A + z * stride + off_out + k * ct_words, l, 0, scale});
    if (n_sum > 1 && (r = pft_total_sum_batch(c, (uint32_t)res.size(), res.data(), n_sum, res.data()))) return r;
    for (size_t z0 = 0; z0 < res.size(); z0 += PFT_MAX_ITEMS) {
        const uint32_t cnt = (uint32_t)std::min<size_t>(PFT_MAX_ITEMS, res.size() - z0);
        ItemPtrs I{}, O{};
        for (uint32_t u = 0; u < cnt; ++u) {
            I.p[u] = res[z0 + u].data;
            O.p[u] = out[z0 + u].data;
        }
        launch_copy_rows_b(cnt, I, 0, O, 0, 2 * l, lg, c->stream);
    }
    for (size_t u = 0; u < res.size(); ++u) {
        out[u].level = l;
        out[u].scale = scale;
    }
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// raw transforms
// ---------------------------------------------------------------------------
static int raw_ntt(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs, bool inv) {
    if (!c || !data) return fail(PFT_EINVAL, "null argument");
    if (n_limbs < 1 || n_limbs > c->P->L) return fail(PFT_EINVAL, "n_limbs must be in 1..L");
    ntt_rows(c, data, n_polys, n_limbs, n_limbs, inv);
    return PFT_OK;
}

extern "C" int pft_ntt_forward(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs) {
    return raw_ntt(c, data, n_polys, n_limbs, false);
}
extern "C" int pft_ntt_inverse(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs) {
    return raw_ntt(c, data, n_polys, n_limbs, true);
}

// Schedules cross the boundary as four words: up to three radices in
// forward order (then zeros) and the flags word.
static void sched_words(const NttSchedule& s, uint32_t* w) {
    for (uint32_t k = 0; k < 3; ++k) w[k] = k < s.n_passes ? s.radix[k] : 0;
    w[3] = s.flags;
}

extern "C" int pft_ntt_candidates(const pft_params* p, uint32_t* scheds, uint32_t max_count) {
    if (!p) return fail(PFT_EINVAL, "null params");
    NttSchedule cand[32];
    const int n = ntt_candidates(p->log_n, cand, 32);
    if (scheds)
        for (uint32_t i = 0; i < std::min<uint32_t>((uint32_t)n, max_count); ++i) sched_words(cand[i], scheds + 4 * i);
    return n;
}

extern "C" int pft_bconv_mode(pft_ctx* c, int mode) {
    if (!c) return fail(PFT_EINVAL, "null context");
    if (mode < 0 || mode > 4)
        return fail(PFT_EINVAL,
                    "mode must be 0 (VALU), 1 (MFMA), 2 (MFMA, fused passes), 3 (2 + fused inner product, digit "
                    "pairs) or 4 (3 with one digit per row pass)");
    c->bconv_mfma = mode >= 1;
    c->bconv_fuse = mode >= 2;
    c->inner_fuse = mode >= 3;
    c->inner_pairs = mode == 3;
    return PFT_OK;
}

extern "C" int pft_ntt_autotune(pft_ctx* c, int enable) {
    if (!c) return fail(PFT_EINVAL, "null context");
    c->ntt_tune = enable != 0;
    if (!c->ntt_tune) c->ntt_tuned.clear();
    return PFT_OK;
}

extern "C" int pft_ntt_set_schedule(pft_ctx* c, int inverse, const uint32_t* sched) {
    if (!c) return fail(PFT_EINVAL, "null context");
    NttSchedule s{};
    if (sched) {
        for (uint32_t k = 0; k < 3 && sched[k]; ++k) {
            if (sched[k] > 16) return fail(PFT_EINVAL, "bad radix %u", sched[k]);
            s.radix[s.n_passes++] = (uint8_t)sched[k];
        }
        s.flags = sched[3];
        if (!ntt_schedule_valid(c->P->log_n, s)) return fail(PFT_EINVAL, "not a candidate schedule for this ring");
    }
    c->ntt_pinned[inverse ? 1 : 0] = s;
    return PFT_OK;
}

extern "C" int pft_ntt_tuning_export(pft_ctx* c, uint32_t* entries, uint32_t max_count) {
    if (!c) return fail(PFT_EINVAL, "null context");
    uint32_t i = 0;
    for (const auto& kv : c->ntt_tuned) {
        if (entries && i < max_count) {
            entries[6 * i] = kv.first >= 64 ? 1u : 0u;
            entries[6 * i + 1] = kv.first & 63u;  // class, + 32 for the first-radix-4 choices
            sched_words(kv.second, entries + 6 * i + 2);
        }
        ++i;
    }
    return (int)i;
}

extern "C" int pft_ntt_tuning_import(pft_ctx* c, const uint32_t* entries, uint32_t count) {
    if (!c || (!entries && count)) return fail(PFT_EINVAL, "null argument");
    std::map<uint32_t, NttSchedule> add;
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t* e = entries + 6 * i;
        if (e[0] > 1 || (e[1] & 31u) > 10 || e[1] > 42) return fail(PFT_EINVAL, "entry %u: bad direction or class", i);
        NttSchedule s{};
        for (uint32_t k = 0; k < 3 && e[2 + k]; ++k) s.radix[s.n_passes++] = (uint8_t)std::min<uint32_t>(e[2 + k], 255u);
        s.flags = e[5];
        if (!ntt_schedule_valid(c->P->log_n, s)) return fail(PFT_EINVAL, "entry %u: not a candidate schedule", i);
        if (e[1] >= 32 && !(s.n_passes >= 2 && s.radix[0] == 4))
            return fail(PFT_EINVAL, "entry %u: a first-radix-4 class needs a schedule starting with 4", i);
        add[(e[0] ? 64u : 0u) + e[1]] = s;
    }
    for (const auto& kv : add) c->ntt_tuned[kv.first] = kv.second;
    return PFT_OK;
}

extern "C" int pft_ntt_get_schedule(pft_ctx* c, int inverse, uint64_t n_limbs, uint32_t* sched) {
    if (!c || !sched) return fail(PFT_EINVAL, "null argument");
    sched_words(ntt_schedule(c, inverse != 0, n_limbs ? n_limbs : 1), sched);
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// ENCODE / DECODE on the host (client side, Sec. 5.1)
// ---------------------------------------------------------------------------
typedef std::complex<double> cd;

// in-place iterative radix-2 FFT of length m (power of two); sign -1 forward
static void fft_pow2(std::vector<cd>& a, int sign) {
    const size_t m = a.size();
    for (size_t i = 1, j = 0; i < m; ++i) {
        size_t bit = m >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= m; len <<= 1) {
        const double ang = sign * 2.0 * M_PI / (double)len;
        for (size_t s = 0; s < m; s += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                const cd w(std::cos(ang * k), std::sin(ang * k));
                const cd u = a[s + k], v = a[s + k + len / 2] * w;
                a[s + k] = u + v;
                a[s + k + len / 2] = u - v;
            }
        }
    }
}

extern "C" int pft_encode(const pft_params* P, const double* re, const double* im, uint32_t n_slots, double scale,
                          int64_t* out) {
    if (!P || !re || !out) return fail(PFT_EINVAL, "null argument");
    if (n_slots > P->n / 2) return fail(PFT_EINVAL, "at most N/2 slots");
    const uint32_t n = P->n;
    std::vector<cd> Z(2 * n, cd(0, 0));
    uint64_t e = 1;
    for (uint32_t j = 0; j < n_slots; ++j) {
        Z[e] = cd(re[j], im ? im[j] : 0.0);
        e = e * 5 % (2 * n);
    }
    fft_pow2(Z, -1);
    const double f = 2.0 * scale / n;
    for (uint32_t k = 0; k < n; ++k) {
        const double x = f * Z[k].real();
        const double rnd = x >= 0 ? std::floor(x + 0.5) : -std::floor(-x + 0.5);
        if (!(std::fabs(rnd) < 4611686018427387904.0)) return fail(PFT_EINVAL, "encoded coefficient exceeds 2^62");
        out[k] = (int64_t)rnd;
    }
    return PFT_OK;
}

extern "C" int pft_decode(const pft_params* P, const uint64_t* res, uint32_t level, double scale, uint32_t n_slots,
                          double* re, double* im) {
    if (!P || !res || !re || !im) return fail(PFT_EINVAL, "null argument");
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level out of range");
    if (n_slots > P->n / 2) return fail(PFT_EINVAL, "at most N/2 slots");
    const uint32_t n = P->n;
    // centred CRT lift of each coefficient: x = sum_i y_i Qhat_i - v Q with
    // y_i = r_i Qhat_i^-1 mod q_i and v = round(sum_i y_i / q_i); evaluated
    // mod 2^64, exact when |x| < 2^63.
    std::vector<uint64_t> hinv(level), hmod(level);
    uint64_t Qmod = 1;
    for (uint32_t i = 0; i < level; ++i) {
        uint64_t h = 1, h64 = 1;
        for (uint32_t o = 0; o < level; ++o)
            if (o != i) {
                h = mulmod(h, P->q[o] % P->q[i], P->q[i]);
                h64 *= P->q[o];
            }
        hinv[i] = invmod(h, P->q[i]);
        hmod[i] = h64;
        Qmod *= P->q[i];
    }
    std::vector<cd> M(2 * n, cd(0, 0));
    for (uint32_t k = 0; k < n; ++k) {
        long double frac = 0;
        uint64_t acc = 0;
        for (uint32_t i = 0; i < level; ++i) {
            const uint64_t y = mulmod(res[(size_t)i * n + k], hinv[i], P->q[i]);
            frac += (long double)y / (long double)P->q[i];
            acc += y * hmod[i];
        }
        const uint64_t v = (uint64_t)std::llround((double)frac);
        acc -= v * Qmod;
        M[k] = cd((double)(int64_t)acc, 0);
    }
    fft_pow2(M, +1);
    uint64_t e = 1;
    for (uint32_t j = 0; j < n_slots; ++j) {
        re[j] = M[e].real() / scale;
        im[j] = M[e].imag() / scale;
        e = e * 5 % (2 * n);
    }
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// per-kernel-family timing (HIP events on the context stream)
// ---------------------------------------------------------------------------
extern "C" int pft_prof_enable(pft_ctx* c, uint32_t mask) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (c->capturing) return fail(PFT_EINVAL, "timing cannot change during graph capture");
    HIPCK(hipStreamSynchronize(c->stream));
    c->prof.reset();
    c->prof.mask = mask & ((1u << PK_COUNT) - 1u);
    return PFT_OK;
}

extern "C" int pft_prof_read(pft_ctx* c, uint32_t kid, double* total_ms, uint64_t* launches, double* bytes,
                             double* ops) {
    if (!c || !total_ms || !launches || !bytes || !ops) return fail(PFT_EINVAL, "null argument");
    if (kid >= PK_COUNT) return fail(PFT_EINVAL, "kernel family %u out of range", kid);
    HIPCK(hipStreamSynchronize(c->stream));
    double ms = 0, by = 0, op = 0;
    uint64_t cnt = 0;
    for (const auto& r : c->prof.recs) {
        if (r.kid != (int)kid) continue;
        float t = 0;
        HIPCK(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        by += r.bytes;
        op += r.ops;
        ++cnt;
    }
    *total_ms = ms;
    *launches = cnt;
    *bytes = by;
    *ops = op;
    return PFT_OK;
}

extern "C" int pft_prof_read_variants(pft_ctx* c, uint32_t kid, uint32_t max_count, uint32_t* variants,
                                      double* total_ms, uint64_t* launches, double* bytes, double* ops) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (kid >= PK_COUNT) return fail(PFT_EINVAL, "kernel family %u out of range", kid);
    HIPCK(hipStreamSynchronize(c->stream));
    struct Acc {
        double ms = 0, by = 0, op = 0;
        uint64_t n = 0;
    };
    std::map<uint32_t, Acc> acc;
    for (const auto& r : c->prof.recs) {
        if (r.kid != (int)kid) continue;
        float t = 0;
        HIPCK(hipEventElapsedTime(&t, r.a, r.b));
        Acc& a = acc[r.variant];
        a.ms += t;
        a.by += r.bytes;
        a.op += r.ops;
        ++a.n;
    }
    std::vector<std::pair<uint32_t, Acc>> v(acc.begin(), acc.end());
    std::stable_sort(v.begin(), v.end(), [](const std::pair<uint32_t, Acc>& x, const std::pair<uint32_t, Acc>& y) {
        return x.second.ms > y.second.ms;
    });
    for (uint32_t i = 0; i < std::min<uint32_t>((uint32_t)v.size(), max_count); ++i) {
        if (variants) variants[i] = v[i].first;
        if (total_ms) total_ms[i] = v[i].second.ms;
        if (launches) launches[i] = v[i].second.n;
        if (bytes) bytes[i] = v[i].second.by;
        if (ops) ops[i] = v[i].second.op;
    }
    return (int)v.size();
}

// ---------------------------------------------------------------------------
// Op-list executor
// ---------------------------------------------------------------------------
// The list runs as if each op were issued alone, in order.  Plan: op j joins
// wave 1 + max(wave of every earlier op sharing a ciphertext with j where
// either writes it); within a wave, ops of equal (kind, input level,
// step/mode) form one group, executed as one batched call (one fused launch
// per stage for the whole group).  Groups of a wave are independent, so each
// runs on its own stream (the context stream and side streams forked from it
// with an event, joined back before the next wave) with its own workspace;
// ciphertexts of different levels therefore occupy the device together.
// Inside pft_graph_begin/end the side streams join the capture, so the whole
// list becomes one graph with a parallel branch per group.
namespace {
struct ExecGroup {
    uint32_t kind, level, mode;
    int32_t step;
    std::vector<uint32_t> ops;
};
}  // namespace

static int exec_group(pft_ctx* c, pft_ct* cts, const pft_op* ops, const ExecGroup& g) {
    const uint32_t n = (uint32_t)g.ops.size();
    std::vector<pft_ct> a(n), b(n), o(n);
    for (uint32_t i = 0; i < n; ++i) {
        const pft_op& op = ops[g.ops[i]];
        a[i] = cts[op.a];
        b[i] = cts[op.kind == PFT_OP_ADD || op.kind == PFT_OP_MUL_RELIN ? op.b : op.a];
        o[i] = cts[op.out];
    }
    int r = PFT_OK;
    switch (g.kind) {
        case PFT_OP_NTT:
        case PFT_OP_INTT: {
            std::vector<NttJob> jobs;
            for (uint32_t i = 0; i < n; ++i)
                for (uint32_t p = 0; p < 2; ++p)
                    jobs.push_back(NttJob{a[i].data + ((size_t)p * g.level << c->P->log_n), 255u, 0u});
            ntt_jobs(c, jobs, g.level, ~0u, g.kind == PFT_OP_INTT);
            return PFT_OK;
        }
        case PFT_OP_ADD:
            for (uint32_t i = 0; i < n && !r; ++i) r = pft_add(c, &a[i], &b[i], &o[i]);
            break;
        case PFT_OP_MUL_RELIN: r = pft_mul_relin_batch(c, n, a.data(), b.data(), o.data()); break;
        case PFT_OP_RESCALE: r = pft_rescale_batch(c, n, a.data(), g.mode, o.data()); break;
        case PFT_OP_ROTATE: r = pft_rotate_batch(c, n, a.data(), g.step, o.data()); break;
        default: return fail(PFT_EINVAL, "unknown op kind %u", g.kind);
    }
    if (r) return r;
    for (uint32_t i = 0; i < n; ++i) {
        cts[ops[g.ops[i]].out].level = o[i].level;
        cts[ops[g.ops[i]].out].scale = o[i].scale;
    }
    return PFT_OK;
}

static int side_branch(pft_ctx* c, size_t k) {
    while (c->side.size() < k) {
        hipStream_t st;
        HIPCK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->side.push_back(st);
        hipEvent_t e;
        HIPCK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->side_ev.push_back(e);
        c->side_ws.push_back({nullptr, 0});
    }
    return PFT_OK;
}

// Waves and groups of an op list given the input levels (shared by
// pft_exec_plan and pft_exec_batch).  Returns the number of waves or an error.
static int plan_ops(const pft_op* ops, uint32_t n_ops, const uint32_t* levels, uint32_t n_cts,
                    std::vector<std::vector<ExecGroup>>& plan) {
    std::vector<uint32_t> lvl(levels, levels + n_cts);
    std::vector<uint32_t> wave(n_ops, 0), in_level(n_ops, 0);
    std::vector<int64_t> last_write(n_cts, -1), last_read_wave(n_cts, 0);
    uint32_t n_waves = 0;
    for (uint32_t j = 0; j < n_ops; ++j) {
        const pft_op& op = ops[j];
        const bool two = op.kind == PFT_OP_ADD || op.kind == PFT_OP_MUL_RELIN;
        const bool in_place = op.kind == PFT_OP_NTT || op.kind == PFT_OP_INTT;
        if (op.kind < PFT_OP_NTT || op.kind > PFT_OP_ROTATE) return fail(PFT_EINVAL, "op %u: unknown kind %u", j, op.kind);
        if (op.a >= n_cts || (two && op.b >= n_cts) || (!in_place && op.out >= n_cts))
            return fail(PFT_EINVAL, "op %u: ciphertext index out of range", j);
        const uint32_t out = in_place ? op.a : op.out;
        if (two && lvl[op.a] != lvl[op.b]) return fail(PFT_ELEVEL, "op %u: operands at different levels", j);
        if ((op.kind == PFT_OP_MUL_RELIN || op.kind == PFT_OP_ROTATE) && (out == op.a || (two && out == op.b)))
            return fail(PFT_EINVAL, "op %u: output aliases an input", j);
        if (op.kind == PFT_OP_RESCALE && lvl[op.a] < 2) return fail(PFT_ELEVEL, "op %u: rescale needs level >= 2", j);
        in_level[j] = lvl[op.a];
        // after every earlier writer of what j touches and every earlier
        // reader of what j writes
        uint32_t w = 0;
        const uint32_t reads[2] = {op.a, two ? op.b : op.a};
        for (uint32_t r : reads)
            if (last_write[r] >= 0) w = std::max<uint32_t>(w, wave[last_write[r]] + 1);
        if (last_write[out] >= 0) w = std::max<uint32_t>(w, wave[last_write[out]] + 1);
        w = std::max<uint32_t>(w, (uint32_t)last_read_wave[out]);
        wave[j] = w;
        n_waves = std::max(n_waves, w + 1);
        for (uint32_t r : reads) last_read_wave[r] = std::max<int64_t>(last_read_wave[r], w + 1);
        last_write[out] = j;
        lvl[out] = op.kind == PFT_OP_RESCALE ? lvl[op.a] - 1 : lvl[op.a];
    }
    plan.assign(n_waves, {});
    for (uint32_t j = 0; j < n_ops; ++j) {
        const pft_op& op = ops[j];
        const uint32_t mode = op.kind == PFT_OP_RESCALE ? op.mode : 0;
        const int32_t step = op.kind == PFT_OP_ROTATE ? op.step : 0;
        auto& gs = plan[wave[j]];
        auto it = std::find_if(gs.begin(), gs.end(), [&](const ExecGroup& g) {
            return g.kind == op.kind && g.level == in_level[j] && g.mode == mode && g.step == step;
        });
        if (it == gs.end()) {
            gs.push_back(ExecGroup{op.kind, in_level[j], mode, step, {}});
            it = gs.end() - 1;
        }
        it->ops.push_back(j);
    }
    return (int)n_waves;
}

extern "C" int pft_exec_plan(const pft_op* ops, uint32_t n_ops, const uint32_t* levels, uint32_t n_cts,
                             uint32_t* wave, uint32_t* group) {
    if ((!ops && n_ops) || (!levels && n_cts)) return fail(PFT_EINVAL, "null argument");
    std::vector<std::vector<ExecGroup>> plan;
    const int nw = plan_ops(ops, n_ops, levels, n_cts, plan);
    if (nw < 0) return nw;
    for (uint32_t w = 0; w < plan.size(); ++w)
        for (uint32_t g = 0; g < plan[w].size(); ++g)
            for (uint32_t j : plan[w][g].ops) {
                if (wave) wave[j] = w;
                if (group) group[j] = g;
            }
    return nw;
}

extern "C" int pft_exec_batch(pft_ctx* c, pft_ct* cts, uint32_t n_cts, const pft_op* ops, uint32_t n_ops) {
    if (!c || (!cts && n_cts) || (!ops && n_ops)) return fail(PFT_EINVAL, "null argument");
    if (c->prof.mask) return fail(PFT_EINVAL, "disable kernel timing before pft_exec_batch");
    std::vector<uint32_t> levels(n_cts);
    for (uint32_t i = 0; i < n_cts; ++i) levels[i] = cts[i].level;
    std::vector<std::vector<ExecGroup>> plan;
    const int nw = plan_ops(ops, n_ops, levels.data(), n_cts, plan);
    if (nw < 0) return nw;
    const uint32_t n_waves = (uint32_t)nw;
    size_t max_groups = 0;
    for (auto& gs : plan) max_groups = std::max(max_groups, gs.size());
    int r;
    if ((r = side_branch(c, max_groups > 0 ? max_groups - 1 : 0))) return r;

    const hipStream_t main = c->stream;
    hipEvent_t fork = nullptr;
    HIPCK(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    r = PFT_OK;
    for (uint32_t w = 0; w < n_waves && !r; ++w) {
        const auto& gs = plan[w];
        if (gs.size() > 1) {
            if (hipEventRecord(fork, main) != hipSuccess) r = fail(PFT_EHIP, "hipEventRecord failed");
            for (size_t k = 1; k < gs.size() && !r; ++k)
                if (hipStreamWaitEvent(c->side[k - 1], fork, 0) != hipSuccess) r = fail(PFT_EHIP, "fork failed");
        }
        for (size_t k = 0; k < gs.size() && !r; ++k) {
            if (k == 0) {
                r = exec_group(c, cts, ops, gs[k]);
                continue;
            }
            // run on side stream k-1 with its own workspace
            uint64_t* const mws = c->ws;
            const size_t mbytes = c->ws_bytes;
            c->stream = c->prof.st = c->side[k - 1];
            c->ws = c->side_ws[k - 1].first;
            c->ws_bytes = c->side_ws[k - 1].second;
            r = exec_group(c, cts, ops, gs[k]);
            c->side_ws[k - 1] = {c->ws, c->ws_bytes};
            c->stream = c->prof.st = main;
            c->ws = mws;
            c->ws_bytes = mbytes;
            if (!r && hipEventRecord(c->side_ev[k - 1], c->side[k - 1]) != hipSuccess)
                r = fail(PFT_EHIP, "hipEventRecord failed");
        }
        for (size_t k = 1; k < gs.size(); ++k)
            if (hipStreamWaitEvent(main, c->side_ev[k - 1], 0) != hipSuccess && !r) r = fail(PFT_EHIP, "join failed");
    }
    (void)hipEventDestroy(fork);
    return r;
}

// ---------------------------------------------------------------------------
// HIP graphs: capture a sequence of calls on the context stream, replay it
// ---------------------------------------------------------------------------
struct pft_graph {
    pft_ctx* ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int pft_ctx_reserve(pft_ctx* c, uint64_t ws_bytes, uint64_t aux_bytes) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (c->capturing) return fail(PFT_EINVAL, "cannot reserve during graph capture");
    int r;
    if ((r = ensure_ws(c, ws_bytes)) || (r = ensure_aux(c, aux_bytes))) return r;
    return PFT_OK;
}

extern "C" int pft_graph_begin(pft_ctx* c) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if (c->capturing) return fail(PFT_EINVAL, "a capture is already open");
    if (!c->stream) return fail(PFT_EINVAL, "graph capture needs a context created on a non-null stream");
    if (c->prof.mask) return fail(PFT_EINVAL, "disable kernel timing before capturing");
    HIPCK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
    c->capturing = true;
    return PFT_OK;
}

extern "C" int pft_graph_end(pft_ctx* c, pft_graph** out) {
    if (!c || !out) return fail(PFT_EINVAL, "null argument");
    if (!c->capturing) return fail(PFT_EINVAL, "no capture is open");
    c->capturing = false;
    auto* g = new pft_graph();
    hipError_t e = hipStreamEndCapture(c->stream, &g->graph);
    if (e != hipSuccess) {
        delete g;
        return fail(PFT_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g->graph);
        delete g;
        return fail(PFT_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    g->ctx = c;
    ++c->live_graphs;
    *out = g;
    return PFT_OK;
}

extern "C" int pft_graph_launch(pft_ctx* c, pft_graph* g) {
    if (!c || !g) return fail(PFT_EINVAL, "null argument");
    if (g->ctx != c) return fail(PFT_EINVAL, "graph belongs to another context");
    if (c->capturing) return fail(PFT_EINVAL, "cannot launch a graph during capture");
    HIPCK(hipGraphLaunch(g->exec, c->stream));
    return PFT_OK;
}

extern "C" void pft_graph_destroy(pft_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->ctx) --g->ctx->live_graphs;
    delete g;
}
