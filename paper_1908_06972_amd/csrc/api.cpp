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

extern "C" int pft_params_create(const pft_param_spec* s, pft_params** out) {
    if (!s || !out) return fail(PFT_EINVAL, "null argument");
    if (!ntt_supported(s->log_n)) return fail(PFT_EPARAM, "log_n %u unsupported (12..16)", s->log_n);
    if (s->n_q < 1 || s->n_q > 64) return fail(PFT_EPARAM, "n_q must be in 1..64");
    if (s->n_p < 1 || s->n_p > 12) return fail(PFT_EPARAM, "n_p must be in 1..12");
    if (s->dnum < 1 || s->dnum > s->n_q) return fail(PFT_EPARAM, "dnum must be in 1..n_q");
    uint32_t alpha = (s->n_q + s->dnum - 1) / s->dnum;
    if (alpha > 12) return fail(PFT_EPARAM, "alpha = ceil(L/dnum) must be <= 12");
    if ((s->n_q + s->n_p) * 2 > 128) return fail(PFT_EPARAM, "too many primes");
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
    P->mods = P->q;
    P->mods.insert(P->mods.end(), P->p.begin(), P->p.end());
    for (uint64_t m : P->mods) P->psi.push_back(primitive_2n_root(m, P->n));
    *out = P;
    return PFT_OK;
}

extern "C" void pft_params_destroy(pft_params* P) { delete P; }

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
};

struct pft_ctx {
    const pft_params* P = nullptr;
    int device = 0;
    hipStream_t stream = nullptr;
    DevTables tabs{};
    KsConsts kc{};
    TwPair* rescale_qinv = nullptr;  // [L][L]: row l-1 holds q_{l-1}^-1 mod q_k
    TwPair* gadget = nullptr;        // [L]: (P mod q_i) as Shoup pairs
    TwPair* to_mont = nullptr;       // [L+K]: 2^64 mod m as Shoup pairs
    std::vector<void*> allocs;
    uint64_t device_bytes = 0;
    uint64_t* s = nullptr;   // [L+K][N] secret, NTT domain
    uint64_t* pk = nullptr;  // [2][L][N] (b, a), NTT domain
    SwitchKeyDev rlk;
    std::map<int32_t, SwitchKeyDev> rot;  // keyed by step mod N/2
    uint64_t* ws = nullptr;
    size_t ws_bytes = 0;
};

template <typename T>
static int dalloc(pft_ctx* c, T** p, size_t bytes) {
    void* v = nullptr;
    hipError_t e = hipMalloc(&v, bytes);
    if (e != hipSuccess) return fail(PFT_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
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
    if (c->ws) {
        HIPCK(hipStreamSynchronize(c->stream));
        HIPCK(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&c->ws, bytes);
    if (e != hipSuccess) return fail(PFT_ENOMEM, "workspace hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    c->ws_bytes = bytes;
    return PFT_OK;
}

static TwPair pair(uint64_t w, uint64_t q) { return TwPair{w, shoup_companion(w, q)}; }

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
            fw[(size_t)m * n + k] = pair(pw[r], q);
            iw[(size_t)m * n + k] = pair(ipw[r], q);
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
    std::vector<TwPair> phatinv(K), pinv(L), gadget(L), tomont(L + K);
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
        gadget[i] = pair(pm, P->q[i]);
    }
    for (uint32_t m = 0; m < L + K; ++m) tomont[m] = pair(to_mont(1, P->mods[m]), P->mods[m]);
    std::vector<TwPair> rq((size_t)L * L, TwPair{0, 0});
    for (uint32_t lvl = 2; lvl <= L; ++lvl)
        for (uint32_t k = 0; k + 1 < lvl; ++k)
            rq[(size_t)(lvl - 1) * L + k] = pair(invmod(P->q[lvl - 1] % P->q[k], P->q[k]), P->q[k]);

    TwPair *d_hatinv, *d_phatinv, *d_pinv;
    uint64_t *d_cmat, *d_downc;
    if ((r = upload(c, &d_hatinv, hatinv)) || (r = upload(c, &d_cmat, cmat)) || (r = upload(c, &d_phatinv, phatinv)) ||
        (r = upload(c, &d_downc, downc)) || (r = upload(c, &d_pinv, pinv)) || (r = upload(c, &c->rescale_qinv, rq)) ||
        (r = upload(c, &c->gadget, gadget)) || (r = upload(c, &c->to_mont, tomont)))
        return r;
    c->kc = KsConsts{d_hatinv, d_cmat, d_phatinv, d_downc, d_pinv, L, K, dnum, A};
    return PFT_OK;
}

extern "C" int pft_ctx_create(const pft_params* P, int device, void* stream, pft_ctx** out) {
    if (!P || !out) return fail(PFT_EINVAL, "null argument");
    HIPCK(hipSetDevice(device));
    auto* c = new pft_ctx();
    c->P = P;
    c->device = device;
    c->stream = (hipStream_t)stream;
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
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->ws) (void)hipFree(c->ws);
    delete c;
}

extern "C" int pft_ctx_synchronize(pft_ctx* c) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ctx_device_bytes(const pft_ctx* c, uint64_t* bytes) {
    if (!c || !bytes) return fail(PFT_EINVAL, "null argument");
    *bytes = c->device_bytes;
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// batch descriptors
// ---------------------------------------------------------------------------
// n_polys polynomials of n_limbs consecutive rows starting at row `first`,
// rows [0, split) mod q_row, rows >= split mod p_(row - split).
static PolyBatch pb_make(const pft_params* P, std::initializer_list<uint64_t*> ptrs, uint32_t n_limbs,
                         uint32_t first = 0, uint32_t split = ~0u) {
    PolyBatch b{};
    uint32_t i = 0;
    for (uint64_t* p : ptrs) b.ptr[i++] = p;
    b.n_polys = i;
    b.n_limbs = n_limbs;
    b.gap_at = 0;
    b.gap_len = first;
    b.split = split;
    b.off0 = 0;
    b.off1 = P->L;
    return b;
}

static PolyBatch pb_rows(const pft_params* P, uint64_t* base, uint32_t n_polys, uint32_t rows_per_poly,
                         uint32_t n_limbs, uint32_t split = ~0u) {
    PolyBatch b{};
    for (uint32_t i = 0; i < n_polys; ++i) b.ptr[i] = base + ((size_t)i * rows_per_poly << P->log_n);
    b.n_polys = n_polys;
    b.n_limbs = n_limbs;
    b.gap_at = 0;
    b.gap_len = 0;
    b.split = split;
    b.off0 = 0;
    b.off1 = P->L;
    return b;
}

static void ntt(pft_ctx* c, const PolyBatch& b, bool inverse) {
    launch_ntt(b, c->tabs, c->P->log_n, inverse, c->stream);
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

extern "C" int pft_set_secret(pft_ctx* c, const int64_t* s) {
    if (!c || !s) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (!check_ternary(s, P->n)) return fail(PFT_EINVAL, "secret must be ternary");
    int r;
    if (!c->s && (r = dalloc(c, &c->s, (size_t)(P->L + P->K) * P->n * 8))) return r;
    if ((r = ensure_ws(c, (size_t)P->n * 8))) return r;
    if ((r = upload_i64(c, (int64_t*)c->ws, s, P->n))) return r;
    PolyBatch b = pb_rows(P, c->s, 1, P->L + P->K, P->L + P->K, P->L);
    launch_int_to_rns((const int64_t*)c->ws, b, c->tabs, P->log_n, c->stream);
    ntt(c, b, false);
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_gen_public_key(pft_ctx* c, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    if (!check_uniform(a, P->q, P->L, P->n)) return fail(PFT_EINVAL, "mask residues must be < q_i");
    int r;
    const size_t nL = (size_t)P->L * P->n;
    if (!c->pk && (r = dalloc(c, &c->pk, 2 * nL * 8))) return r;
    if ((r = ensure_ws(c, (nL + P->n) * 8))) return r;
    uint64_t* e_rns = c->ws;
    int64_t* e_raw = (int64_t*)(c->ws + nL);
    uint64_t* pa = c->pk + nL;
    if ((r = upload_u64(c, pa, a, nL)) || (r = upload_i64(c, e_raw, e, P->n))) return r;
    PolyBatch A = pb_rows(P, pa, 1, P->L, P->L);
    ntt(c, A, false);
    PolyBatch E = pb_rows(P, e_rns, 1, P->L, P->L);
    launch_int_to_rns(e_raw, E, c->tabs, P->log_n, c->stream);
    ntt(c, E, false);
    // b = -(a s) + e
    PolyBatch S = pb_rows(P, c->s, 1, P->L, P->L);
    PolyBatch B = pb_rows(P, c->pk, 1, P->L, P->L);
    launch_ew(EW_NEG_MULADD, B, A, &S, &E, c->tabs, P->log_n, c->stream);
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

// s_prime: [L+K][N] NTT domain (device).  Builds the switching key into *dst.
static int gen_switch_key(pft_ctx* c, const uint64_t* s_prime, const uint64_t* a, const int64_t* e,
                          SwitchKeyDev* dst) {
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    const size_t nR = (size_t)R * P->n;
    for (uint32_t j = 0; j < P->dnum; ++j)
        if (!check_uniform(a + (size_t)j * nR, P->mods, R, P->n))
            return fail(PFT_EINVAL, "mask residues must be < their modulus");
    int r;
    if (!dst->data && (r = dalloc(c, &dst->data, (size_t)P->dnum * 2 * nR * 8))) return r;
    if ((r = ensure_ws(c, (nR + P->n + nR) * 8))) return r;
    uint64_t* e_rns = c->ws;
    int64_t* e_raw = (int64_t*)(c->ws + nR);
    uint64_t* gs = c->ws + nR + P->n;  // gadget * s'
    PolyBatch S = pb_rows(P, c->s, 1, R, R, P->L);
    for (uint32_t j = 0; j < P->dnum; ++j) {
        uint64_t* kb = dst->data + (size_t)(2 * j) * nR;
        uint64_t* ka = dst->data + (size_t)(2 * j + 1) * nR;
        if ((r = upload_u64(c, ka, a + (size_t)j * nR, nR)) || (r = upload_i64(c, e_raw, e + (size_t)j * P->n, P->n)))
            return r;
        PolyBatch A = pb_rows(P, ka, 1, R, R, P->L);
        ntt(c, A, false);
        PolyBatch E = pb_rows(P, e_rns, 1, R, R, P->L);
        launch_int_to_rns(e_raw, E, c->tabs, P->log_n, c->stream);
        ntt(c, E, false);
        PolyBatch B = pb_rows(P, kb, 1, R, R, P->L);
        launch_ew(EW_NEG_MULADD, B, A, &S, &E, c->tabs, P->log_n, c->stream);  // b = -a s + e
        // + (P mod q_t) s' on the q-limbs of digit j
        const uint32_t i0 = j * P->alpha, i1 = std::min(i0 + P->alpha, P->L);
        if (i0 < i1) {
            PolyBatch Sp = pb_make(P, {(uint64_t*)s_prime}, i1 - i0, i0);
            PolyBatch G = pb_make(P, {gs}, i1 - i0, i0);
            launch_mul_const(G, Sp, c->gadget + i0, c->tabs, P->log_n, c->stream);
            PolyBatch Bd = pb_make(P, {kb}, i1 - i0, i0);
            launch_ew(EW_ADD, Bd, Bd, &G, nullptr, c->tabs, P->log_n, c->stream);
        }
        // store both halves times 2^64 (Montgomery form) for the inner product
        launch_mul_const(B, B, c->to_mont, c->tabs, P->log_n, c->stream);
        launch_mul_const(A, A, c->to_mont, c->tabs, P->log_n, c->stream);
    }
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_gen_relin_key(pft_ctx* c, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    uint64_t* s2;
    int r;
    if ((r = dalloc(c, &s2, (size_t)R * P->n * 8))) return r;  // kept: small, freed with ctx
    PolyBatch S = pb_rows(P, c->s, 1, R, R, P->L);
    PolyBatch S2 = pb_rows(P, s2, 1, R, R, P->L);
    launch_ew(EW_MUL, S2, S, &S, nullptr, c->tabs, P->log_n, c->stream);
    return gen_switch_key(c, s2, a, e, &c->rlk);
}

static uint64_t galois_element(int32_t step, uint32_t n) {
    const int64_t half = n / 2;
    int64_t r = ((int64_t)step % half + half) % half;
    return powmod(5, (uint64_t)r, 2ull * n);
}

static int32_t norm_step(int32_t step, uint32_t n) {
    const int64_t half = n / 2;
    return (int32_t)((((int64_t)step % half) + half) % half);
}

extern "C" int pft_gen_rotation_key(pft_ctx* c, int32_t step, const uint64_t* a, const int64_t* e) {
    if (!c || !a || !e) return fail(PFT_EINVAL, "null argument");
    if (!c->s) return fail(PFT_ENOKEY, "set the secret first");
    const pft_params* P = c->P;
    const uint32_t R = P->L + P->K;
    uint64_t* srot;
    int r;
    if ((r = dalloc(c, &srot, (size_t)R * P->n * 8))) return r;
    launch_automorphism(c->s, srot, 1, R, galois_element(step, P->n), P->log_n, c->stream);
    SwitchKeyDev& k = c->rot[norm_step(step, P->n)];
    return gen_switch_key(c, srot, a, e, &k);
}

// ---------------------------------------------------------------------------
// ENC / DEC, import / export
// ---------------------------------------------------------------------------
static int check_ct(const pft_ctx* c, const pft_ct* ct) {
    if (!ct || !ct->data) return fail(PFT_EINVAL, "null ciphertext");
    if (ct->level < 1 || ct->level > c->P->L) return fail(PFT_ELEVEL, "level %u out of range", ct->level);
    return PFT_OK;
}

extern "C" int pft_encrypt(pft_ctx* c, const int64_t* m, uint32_t level, double scale, const int64_t* v,
                           const int64_t* e0, const int64_t* e1, pft_ct* out) {
    if (!c || !m || !v || !e0 || !e1 || !out || !out->data) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (!c->pk) return fail(PFT_ENOKEY, "no public key");
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    if (!check_ternary(v, P->n)) return fail(PFT_EINVAL, "v must be ternary");
    const uint32_t n = P->n;
    const size_t nl = (size_t)level * n;
    int r;
    if ((r = ensure_ws(c, (4 * nl + 4 * (size_t)n) * 8))) return r;
    uint64_t* M = c->ws;
    uint64_t* V = M + nl;
    uint64_t* E0 = V + nl;
    uint64_t* E1 = E0 + nl;
    int64_t* raw = (int64_t*)(E1 + nl);
    if ((r = upload_i64(c, raw, m, n)) || (r = upload_i64(c, raw + n, v, n)) || (r = upload_i64(c, raw + 2 * n, e0, n)) ||
        (r = upload_i64(c, raw + 3 * n, e1, n)))
        return r;
    PolyBatch all = pb_make(P, {M, V, E0, E1}, level);
    launch_int_to_rns(raw, all, c->tabs, P->log_n, c->stream);
    ntt(c, all, false);
    const size_t nL = (size_t)P->L * n;
    PolyBatch Bk = pb_make(P, {c->pk}, level), Ak = pb_make(P, {c->pk + nL}, level);
    PolyBatch Vb = pb_make(P, {V}, level);
    PolyBatch C0 = pb_make(P, {out->data}, level), C1 = pb_make(P, {out->data + nl}, level);
    PolyBatch E0b = pb_make(P, {E0}, level), E1b = pb_make(P, {E1}, level), Mb = pb_make(P, {M}, level);
    launch_ew(EW_MULADD, C0, Bk, &Vb, &E0b, c->tabs, P->log_n, c->stream);  // b v + e0
    launch_ew(EW_ADD, C0, C0, &Mb, nullptr, c->tabs, P->log_n, c->stream);  // + m
    launch_ew(EW_MULADD, C1, Ak, &Vb, &E1b, c->tabs, P->log_n, c->stream);  // a v + e1
    out->level = level;
    out->scale = scale;
    HIPCK(hipStreamSynchronize(c->stream));  // the raw host inputs were pageable copies
    return PFT_OK;
}

extern "C" int pft_decrypt(pft_ctx* c, const pft_ct* ct, uint64_t* out) {
    if (!c || !out) return fail(PFT_EINVAL, "null argument");
    int r;
    if ((r = check_ct(c, ct))) return r;
    if (!c->s) return fail(PFT_ENOKEY, "no secret");
    const pft_params* P = c->P;
    const size_t nl = (size_t)ct->level * P->n;
    if ((r = ensure_ws(c, nl * 8))) return r;
    PolyBatch Mu = pb_make(P, {c->ws}, ct->level);
    PolyBatch C0 = pb_make(P, {ct->data}, ct->level), C1 = pb_make(P, {ct->data + nl}, ct->level);
    PolyBatch S = pb_make(P, {c->s}, ct->level);
    launch_ew(EW_MULADD, Mu, C1, &S, &C0, c->tabs, P->log_n, c->stream);
    ntt(c, Mu, true);
    HIPCK(hipMemcpyAsync(out, c->ws, nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ct_export(pft_ctx* c, const pft_ct* ct, uint64_t* host) {
    if (!c || !host) return fail(PFT_EINVAL, "null argument");
    int r;
    if ((r = check_ct(c, ct))) return r;
    const pft_params* P = c->P;
    const size_t nl = (size_t)ct->level * P->n;
    if ((r = ensure_ws(c, 2 * nl * 8))) return r;
    HIPCK(hipMemcpyAsync(c->ws, ct->data, 2 * nl * 8, hipMemcpyDeviceToDevice, c->stream));
    ntt(c, pb_rows(P, c->ws, 2, ct->level, ct->level), true);
    HIPCK(hipMemcpyAsync(host, c->ws, 2 * nl * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_ct_import(pft_ctx* c, const uint64_t* host, uint32_t level, double scale, pft_ct* ct) {
    if (!c || !host || !ct || !ct->data) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    for (uint32_t b = 0; b < 2; ++b)
        if (!check_uniform(host + (size_t)b * level * P->n, P->q, level, P->n))
            return fail(PFT_EINVAL, "residues must be < q_i");
    const size_t nl = (size_t)level * P->n;
    HIPCK(hipMemcpyAsync(ct->data, host, 2 * nl * 8, hipMemcpyHostToDevice, c->stream));
    ntt(c, pb_rows(P, ct->data, 2, level, level), false);
    ct->level = level;
    ct->scale = scale;
    HIPCK(hipStreamSynchronize(c->stream));
    return PFT_OK;
}

extern "C" int pft_pt_from_coeffs(pft_ctx* c, const int64_t* m, uint32_t level, double scale, pft_pt* pt) {
    if (!c || !m || !pt || !pt->data) return fail(PFT_EINVAL, "null argument");
    const pft_params* P = c->P;
    if (level < 1 || level > P->L) return fail(PFT_ELEVEL, "level %u out of range", level);
    int r;
    if ((r = ensure_ws(c, (size_t)P->n * 8))) return r;
    if ((r = upload_i64(c, (int64_t*)c->ws, m, P->n))) return r;
    PolyBatch b = pb_make(P, {pt->data}, level);
    launch_int_to_rns((const int64_t*)c->ws, b, c->tabs, P->log_n, c->stream);
    ntt(c, b, false);
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
    if ((r = check_ct(c, a)) || (r = check_ct(c, b)) || (r = check_ct(c, out))) return r;
    if (a->level != b->level) return fail(PFT_ELEVEL, "HADD needs equal levels (%u vs %u)", a->level, b->level);
    if (!scales_match(a->scale, b->scale)) return fail(PFT_ESCALE, "HADD needs equal scales");
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    PolyBatch O = pb_rows(P, out->data, 2, l, l), A = pb_rows(P, a->data, 2, l, l), B = pb_rows(P, b->data, 2, l, l);
    launch_ew(EW_ADD, O, A, &B, nullptr, c->tabs, P->log_n, c->stream);
    out->level = l;
    out->scale = a->scale;
    return PFT_OK;
}

static int check_pt(const pft_ctx* c, const pft_pt* p, uint32_t level) {
    if (!p || !p->data) return fail(PFT_EINVAL, "null plaintext");
    if (p->level < level) return fail(PFT_ELEVEL, "plaintext level %u below ciphertext level %u", p->level, level);
    (void)c;
    return PFT_OK;
}

extern "C" int pft_add_plain(pft_ctx* c, const pft_ct* a, const pft_pt* p, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, a)) || (r = check_ct(c, out)) || (r = check_pt(c, p, a->level))) return r;
    if (!scales_match(a->scale, p->scale)) return fail(PFT_ESCALE, "HADDPLAIN needs equal scales");
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    const size_t nl = (size_t)l * P->n;
    PolyBatch O0 = pb_make(P, {out->data}, l), A0 = pb_make(P, {a->data}, l), Pt = pb_make(P, {p->data}, l);
    launch_ew(EW_ADD, O0, A0, &Pt, nullptr, c->tabs, P->log_n, c->stream);
    if (out->data != a->data) {
        HIPCK(hipMemcpyAsync(out->data + nl, a->data + nl, nl * 8, hipMemcpyDeviceToDevice, c->stream));
    }
    out->level = l;
    out->scale = a->scale;
    return PFT_OK;
}

extern "C" int pft_mul_plain(pft_ctx* c, const pft_ct* a, const pft_pt* p, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, a)) || (r = check_ct(c, out)) || (r = check_pt(c, p, a->level))) return r;
    const pft_params* P = c->P;
    const uint32_t l = a->level;
    PolyBatch O = pb_rows(P, out->data, 2, l, l), A = pb_rows(P, a->data, 2, l, l);
    PolyBatch Pt = pb_make(P, {p->data, p->data}, l);
    launch_ew(EW_MUL, O, A, &Pt, nullptr, c->tabs, P->log_n, c->stream);
    out->level = l;
    out->scale = a->scale * p->scale;
    return PFT_OK;
}

extern "C" int pft_mod_drop(pft_ctx* c, const pft_ct* in, uint32_t level, pft_ct* out) {
    int r;
    if (!c) return fail(PFT_EINVAL, "null ctx");
    if ((r = check_ct(c, in)) || !out || !out->data) return r ? r : fail(PFT_EINVAL, "null output");
    if (level < 1 || level > in->level) return fail(PFT_ELEVEL, "mod_drop to %u from %u", level, in->level);
    const pft_params* P = c->P;
    const size_t lo = (size_t)level * P->n, li = (size_t)in->level * P->n;
    // [2][level][N] from [2][in_level][N]; poly 1 moves down when levels differ
    HIPCK(hipMemcpyAsync(out->data, in->data, lo * 8, hipMemcpyDeviceToDevice, c->stream));
    if (out->data != in->data || level != in->level)
        HIPCK(hipMemcpyAsync(out->data + lo, in->data + li, lo * 8, hipMemcpyDeviceToDevice, c->stream));
    out->level = level;
    out->scale = in->scale;
    return PFT_OK;
}

// Scratch needed by one key switch at `level`.
static size_t ks_ws_words(const pft_params* P, uint32_t level) {
    const uint32_t beta = (level + P->alpha - 1) / P->alpha;
    const size_t rows = level + P->K;
    return ((size_t)level + beta * rows + 2 * rows + 2 * (size_t)level) << P->log_n;
}

// Hybrid key switching of d (NTT domain, [level][N]) with `key`; writes
// out[2][level][N] = ModDown(sum_j ModUp_j(d) * key_j) + (add0, add1).
// ws must hold ks_ws_words(level) words.
static void key_switch(pft_ctx* c, const uint64_t* d_ntt, const SwitchKeyDev& key, uint32_t level,
                       const uint64_t* add0, const uint64_t* add1, uint64_t* out, uint64_t* ws) {
    const pft_params* P = c->P;
    const uint32_t lg = P->log_n, K = P->K, A = P->alpha;
    const uint32_t beta = (level + A - 1) / A, rows = level + K;
    uint64_t* d_coef = ws;
    uint64_t* ext = d_coef + ((size_t)level << lg);
    uint64_t* acc = ext + ((size_t)beta * rows << lg);
    uint64_t* conv = acc + ((size_t)2 * rows << lg);
    (void)hipMemcpyAsync(d_coef, d_ntt, ((size_t)level << lg) * 8, hipMemcpyDeviceToDevice, c->stream);
    ntt(c, pb_make(P, {d_coef}, level), true);
    launch_modup(d_coef, ext, level, c->kc, c->tabs, lg, c->stream);
    for (uint32_t j = 0; j < beta; ++j) {
        const uint32_t i0 = j * A, na = std::min(i0 + A, level) - i0;
        PolyBatch b{};
        b.ptr[0] = ext + ((size_t)j * rows << lg);
        b.n_polys = 1;
        b.n_limbs = rows - na;
        b.gap_at = i0;
        b.gap_len = na;
        b.split = level;
        b.off0 = 0;
        b.off1 = P->L;
        ntt(c, b, false);
    }
    launch_key_inner(d_ntt, ext, key.data, acc, level, c->kc, c->tabs, lg, c->stream);
    // ModDown: special rows of both accumulators to coefficient form
    PolyBatch sp = pb_make(P, {acc, acc + ((size_t)rows << lg)}, K, level, level);
    ntt(c, sp, true);
    launch_moddown_conv(acc, conv, level, c->kc, c->tabs, lg, c->stream);
    ntt(c, pb_rows(P, conv, 2, level, level), false);
    launch_moddown_final(acc, conv, add0, add1, out, level, c->kc, c->tabs, lg, c->stream);
}

static int mul_relin_one(pft_ctx* c, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    const pft_params* P = c->P;
    const uint32_t l = a->level, lg = P->log_n;
    const size_t nl = (size_t)l << lg;
    int r;
    if ((r = ensure_ws(c, (3 * nl + ks_ws_words(P, l)) * 8))) return r;
    uint64_t *d0 = c->ws, *d1 = d0 + nl, *d2 = d1 + nl, *ws = d2 + nl;
    launch_tensor(a->data, b->data, d0, d1, d2, l, c->tabs, lg, c->stream);
    key_switch(c, d2, c->rlk, l, d0, d1, out->data, ws);
    out->level = l;
    out->scale = a->scale * b->scale;
    return PFT_OK;
}

extern "C" int pft_mul_relin(pft_ctx* c, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    return pft_mul_relin_batch(c, 1, a, b, out);
}

extern "C" int pft_mul_relin_batch(pft_ctx* c, uint32_t n, const pft_ct* a, const pft_ct* b, pft_ct* out) {
    if (!c || !a || !b || !out) return fail(PFT_EINVAL, "null argument");
    if (!c->rlk.data) return fail(PFT_ENOKEY, "no relinearisation key");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &a[i])) || (r = check_ct(c, &b[i])) || (r = check_ct(c, &out[i]))) return r;
        if (a[i].level != b[i].level) return fail(PFT_ELEVEL, "HMUL needs equal levels");
        if (out[i].data == a[i].data || out[i].data == b[i].data) return fail(PFT_EINVAL, "output aliases an input");
    }
    for (uint32_t i = 0; i < n; ++i)
        if ((r = mul_relin_one(c, &a[i], &b[i], &out[i]))) return r;
    return PFT_OK;
}

static int rescale_one(pft_ctx* c, const pft_ct* in, uint32_t mode, pft_ct* out) {
    const pft_params* P = c->P;
    const uint32_t l = in->level, lg = P->log_n;
    const size_t n = (size_t)1 << lg;
    int r;
    if ((r = ensure_ws(c, (2 * n + 2 * (size_t)(l - 1) * n) * 8))) return r;
    uint64_t* last = c->ws;
    uint64_t* tmp = last + 2 * n;
    HIPCK(hipMemcpyAsync(last, in->data + (size_t)(l - 1) * n, n * 8, hipMemcpyDeviceToDevice, c->stream));
    HIPCK(hipMemcpyAsync(last + n, in->data + (size_t)(2 * l - 1) * n, n * 8, hipMemcpyDeviceToDevice, c->stream));
    PolyBatch Lb = pb_make(P, {last, last + n}, 1, l - 1);
    Lb.gap_len = 0;
    Lb.off0 = l - 1;  // both rows are limb l-1
    Lb.split = ~0u;
    ntt(c, Lb, true);
    launch_rescale_expand(last, tmp, l, mode, c->tabs, lg, c->stream);
    ntt(c, pb_rows(P, tmp, 2, l - 1, l - 1), false);
    launch_rescale_final(in->data, tmp, out->data, l, c->rescale_qinv + (size_t)(l - 1) * P->L, c->tabs, lg,
                         c->stream);
    out->level = l - 1;
    out->scale = in->scale / (double)P->q[l - 1];
    return PFT_OK;
}

extern "C" int pft_rescale(pft_ctx* c, const pft_ct* in, uint32_t mode, pft_ct* out) {
    return pft_rescale_batch(c, 1, in, mode, out);
}

extern "C" int pft_rescale_batch(pft_ctx* c, uint32_t n, const pft_ct* in, uint32_t mode, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    if (mode > 1) return fail(PFT_EINVAL, "mode must be 0 (round) or 1 (floor)");
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i]))) return r;
        if (in[i].level < 2) return fail(PFT_ELEVEL, "cannot rescale at level 1");
        if (!out[i].data) return fail(PFT_EINVAL, "null output");
        if (out[i].data == in[i].data) return fail(PFT_EINVAL, "rescale output aliases its input");
    }
    for (uint32_t i = 0; i < n; ++i)
        if ((r = rescale_one(c, &in[i], mode, &out[i]))) return r;
    return PFT_OK;
}

static int rotate_one(pft_ctx* c, const pft_ct* in, const SwitchKeyDev& key, uint64_t kappa, pft_ct* out) {
    const pft_params* P = c->P;
    const uint32_t l = in->level, lg = P->log_n;
    const size_t nl = (size_t)l << lg;
    int r;
    if ((r = ensure_ws(c, (2 * nl + ks_ws_words(P, l)) * 8))) return r;
    uint64_t* rot = c->ws;  // [2][l][N]: c0(X^kappa), c1(X^kappa)
    launch_automorphism(in->data, rot, 2, l, kappa, lg, c->stream);
    key_switch(c, rot + nl, key, l, rot, nullptr, out->data, rot + 2 * nl);
    out->level = l;
    out->scale = in->scale;
    return PFT_OK;
}

static const SwitchKeyDev* find_rot(pft_ctx* c, int32_t step) {
    auto it = c->rot.find(norm_step(step, c->P->n));
    return it == c->rot.end() ? nullptr : &it->second;
}

extern "C" int pft_rotate(pft_ctx* c, const pft_ct* in, int32_t step, pft_ct* out) {
    return pft_rotate_batch(c, 1, in, step, out);
}

extern "C" int pft_rotate_batch(pft_ctx* c, uint32_t n, const pft_ct* in, int32_t step, pft_ct* out) {
    if (!c || !in || !out) return fail(PFT_EINVAL, "null argument");
    const SwitchKeyDev* key = find_rot(c, step);
    if (!key) return fail(PFT_ENOKEY, "no rotation key for step %d", step);
    int r;
    for (uint32_t i = 0; i < n; ++i) {
        if ((r = check_ct(c, &in[i])) || (r = check_ct(c, &out[i]))) return r;
        if (out[i].data == in[i].data) return fail(PFT_EINVAL, "rotate output aliases its input");
    }
    const uint64_t kappa = galois_element(step, c->P->n);
    for (uint32_t i = 0; i < n; ++i)
        if ((r = rotate_one(c, &in[i], *key, kappa, &out[i]))) return r;
    return PFT_OK;
}

extern "C" int pft_total_sum(pft_ctx* c, const pft_ct* in, uint32_t n_slots, pft_ct* out) {
    if (!c) return fail(PFT_EINVAL, "null ctx");
    int r;
    if ((r = check_ct(c, in)) || (r = check_ct(c, out))) return r;
    if (n_slots < 1 || n_slots > c->P->n / 2 || (n_slots & (n_slots - 1)))
        return fail(PFT_EINVAL, "n_slots must be a power of two <= N/2");
    for (uint32_t s = 1; s < n_slots; s <<= 1)
        if (!find_rot(c, (int32_t)s)) return fail(PFT_ENOKEY, "no rotation key for step %u", s);
    const pft_params* P = c->P;
    const uint32_t l = in->level, lg = P->log_n;
    const size_t nl = (size_t)l << lg;
    if ((r = ensure_ws(c, (4 * nl + ks_ws_words(P, l)) * 8))) return r;
    uint64_t* cur = c->ws;           // [2][l][N]
    uint64_t* rot = cur + 2 * nl;    // [2][l][N]
    uint64_t* ws = rot + 2 * nl;
    HIPCK(hipMemcpyAsync(cur, in->data, 2 * nl * 8, hipMemcpyDeviceToDevice, c->stream));
    PolyBatch Cur = pb_rows(P, cur, 2, l, l);
    for (uint32_t s = 1; s < n_slots; s <<= 1) {
        // rot = ROTATE(cur, s); cur = cur + rot
        launch_automorphism(cur, rot, 2, l, galois_element((int32_t)s, P->n), lg, c->stream);
        key_switch(c, rot + nl, *find_rot(c, (int32_t)s), l, rot, nullptr, rot, ws);
        PolyBatch Rot = pb_rows(P, rot, 2, l, l);
        launch_ew(EW_ADD, Cur, Cur, &Rot, nullptr, c->tabs, lg, c->stream);
    }
    HIPCK(hipMemcpyAsync(out->data, cur, 2 * nl * 8, hipMemcpyDeviceToDevice, c->stream));
    out->level = l;
    out->scale = in->scale;
    return PFT_OK;
}

// ---------------------------------------------------------------------------
// raw transforms
// ---------------------------------------------------------------------------
static int raw_ntt(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs, bool inv) {
    if (!c || !data) return fail(PFT_EINVAL, "null argument");
    if (n_limbs < 1 || n_limbs > c->P->L) return fail(PFT_EINVAL, "n_limbs must be in 1..L");
    const pft_params* P = c->P;
    for (uint32_t p0 = 0; p0 < n_polys; p0 += PFT_MAX_POLYS) {
        const uint32_t np = std::min<uint32_t>(PFT_MAX_POLYS, n_polys - p0);
        ntt(c, pb_rows(P, data + ((size_t)p0 * n_limbs << P->log_n), np, n_limbs, n_limbs), inv);
    }
    return PFT_OK;
}

extern "C" int pft_ntt_forward(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs) {
    return raw_ntt(c, data, n_polys, n_limbs, false);
}
extern "C" int pft_ntt_inverse(pft_ctx* c, uint64_t* data, uint32_t n_polys, uint32_t n_limbs) {
    return raw_ntt(c, data, n_polys, n_limbs, true);
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
