/*
 * ring_oracle.c -- TEST INFRASTRUCTURE ONLY: the plain, slow CPU oracle for the
 * RNS polynomial arithmetic of the CKKS scheme of PrivFT (arXiv:1908.06972).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product (the HIP library) never links,
 * loads or calls it, and this file shares no code, header, table or constant
 * generator with the product.
 *
 * Every routine here is the textbook definition written out with 128-bit
 * integer arithmetic: `(a*b) % q` through unsigned __int128, one coefficient at
 * a time, no lazy reduction, no Shoup/Barrett/Montgomery tricks, no blocking.
 *
 * What is defined where (citations are to the paper):
 *   - R_q = Z_q[X]/(X^N+1) and the RNS chain q_l = p_1...p_l: Sec. 3.4
 *     (The CKKS levelled FHE scheme), first paragraphs.
 *   - products in R_q (HMUL, HMULPLAIN): Sec. 3.4, homomorphic operations.
 *   - X -> X^kappa (ROTATE): Sec. 3.4, ROTATE and its footnote; Sec. 6.5
 *     (text after Table 2) for the Galois element per rotation.
 *   - RESCALE by the last prime via Eq. (1) and Alg. 3: Sec. 5.1.
 *   - fast base conversion (used by hybrid key switching, which the paper
 *     only cites): it is the exact integer sum Y = sum_i [x_i*Qhat_i^-1]_{q_i}*Qhat_i,
 *     reduced modulo each target prime.
 *
 * The negacyclic product has two modes:
 *   mode 0: schoolbook convolution, the definition (O(N^2));
 *   mode 1: via this file's own textbook transform (pre-twist by psi^j, an
 *           iterative radix-2 cyclic transform with omega = psi^2, bit reversal),
 *           needed only to make N = 2^15..2^16 affordable.  The test suite pins
 *           mode 1 to mode 0 bit for bit.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + b) % q); }
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a + q - (b % q)) % q); }

uint64_t or_powmod(uint64_t b, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime q by Fermat's little theorem */
uint64_t or_invmod(uint64_t a, uint64_t q) { return or_powmod(a, q - 2, q); }

static uint32_t bitrev(uint32_t x, uint32_t logn) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < logn; ++i) r |= ((x >> i) & 1u) << (logn - 1 - i);
    return r;
}

static uint32_t log2u(uint32_t n) {
    uint32_t l = 0;
    while ((1u << l) < n) ++l;
    return l;
}

/* ---- ring product in Z_q[X]/(X^N+1): the schoolbook definition ---------- */
static void negacyclic_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* out,
                                  uint32_t n, uint64_t q) {
    for (uint32_t k = 0; k < n; ++k) {
        /* out_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j */
        uint64_t pos = 0, neg = 0;
        for (uint32_t i = 0; i <= k; ++i) pos = addmod(pos, mulmod(a[i], b[k - i], q), q);
        for (uint32_t i = k + 1; i < n; ++i) neg = addmod(neg, mulmod(a[i], b[n + k - i], q), q);
        out[k] = submod(pos, neg, q);
    }
}

/* ---- the transform (used for mode 1 and as the definition the HIP NTT is
 * tested against) ------------------------------------------------------- */

/* Definition, O(N^2): out[k] = sum_j a_j * psi^((2*brv(k)+1)*j) mod q, i.e. the
 * evaluation of a(X) at the odd powers of a primitive 2N-th root psi, stored in
 * bit-reversed order. */
void or_ntt_definition(const uint64_t* a, uint64_t* out, uint32_t n, uint64_t q, uint64_t psi) {
    uint32_t logn = log2u(n);
    for (uint32_t k = 0; k < n; ++k) {
        uint64_t x = or_powmod(psi, 2ull * bitrev(k, logn) + 1, q); /* evaluation point */
        uint64_t acc = 0, xp = 1;
        for (uint32_t j = 0; j < n; ++j) {
            acc = addmod(acc, mulmod(a[j], xp, q), q);
            xp = mulmod(xp, x, q);
        }
        out[k] = acc;
    }
}

/* Textbook iterative radix-2 cyclic DFT over Z_q of length n with root w (in
 * place, natural order in and out): bit-reversal permutation followed by
 * log2(n) Cooley-Tukey stages. */
static void cyclic_dft(uint64_t* x, uint32_t n, uint64_t q, uint64_t w) {
    uint32_t logn = log2u(n);
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t r = bitrev(i, logn);
        if (r > i) { uint64_t t = x[i]; x[i] = x[r]; x[r] = t; }
    }
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint64_t wl = or_powmod(w, n / len, q); /* primitive len-th root */
        for (uint32_t s = 0; s < n; s += len) {
            uint64_t wj = 1;
            for (uint32_t j = 0; j < len / 2; ++j) {
                uint64_t u = x[s + j], v = mulmod(x[s + j + len / 2], wj, q);
                x[s + j] = addmod(u, v, q);
                x[s + j + len / 2] = submod(u, v, q);
                wj = mulmod(wj, wl, q);
            }
        }
    }
}

/* Same result as or_ntt_definition in O(N log N): A(psi^(2i+1)) =
 * sum_j (a_j psi^j) (psi^2)^(ij), then index k holds A(psi^(2 brv(k)+1)). */
void or_ntt_fast(const uint64_t* a, uint64_t* out, uint32_t n, uint64_t q, uint64_t psi) {
    uint32_t logn = log2u(n);
    uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * n);
    uint64_t pj = 1;
    for (uint32_t j = 0; j < n; ++j) { t[j] = mulmod(a[j] % q, pj, q); pj = mulmod(pj, psi, q); }
    cyclic_dft(t, n, q, mulmod(psi, psi, q));
    for (uint32_t k = 0; k < n; ++k) out[k] = t[bitrev(k, logn)];
    free(t);
}

/* Inverse of or_ntt_fast: un-permute, inverse cyclic DFT (root omega^-1, times
 * 1/n), then undo the pre-twist (times psi^-j). */
void or_intt_fast(const uint64_t* in, uint64_t* out, uint32_t n, uint64_t q, uint64_t psi) {
    uint32_t logn = log2u(n);
    uint64_t* t = (uint64_t*)malloc(sizeof(uint64_t) * n);
    for (uint32_t k = 0; k < n; ++k) t[bitrev(k, logn)] = in[k] % q;
    uint64_t psi_inv = or_invmod(psi, q);
    cyclic_dft(t, n, q, mulmod(psi_inv, psi_inv, q));
    uint64_t n_inv = or_invmod(n % q, q), pj = n_inv;
    for (uint32_t j = 0; j < n; ++j) { out[j] = mulmod(t[j], pj, q); pj = mulmod(pj, psi_inv, q); }
    free(t);
}

static int g_mul_mode = 0; /* 0: schoolbook, 1: transform */
void or_set_mul_mode(int mode) { g_mul_mode = mode; }
int or_get_mul_mode(void) { return g_mul_mode; }

/* Negacyclic product of one limb; psi is only used in mode 1. */
void or_mul_limb(const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t n, uint64_t q,
                 uint64_t psi, int mode) {
    if (mode == 0) {
        negacyclic_schoolbook(a, b, out, n, q);
        return;
    }
    uint64_t* fa = (uint64_t*)malloc(sizeof(uint64_t) * n);
    uint64_t* fb = (uint64_t*)malloc(sizeof(uint64_t) * n);
    or_ntt_fast(a, fa, n, q, psi);
    or_ntt_fast(b, fb, n, q, psi);
    for (uint32_t k = 0; k < n; ++k) fa[k] = mulmod(fa[k], fb[k], q);
    or_intt_fast(fa, out, n, q, psi);
    free(fa);
    free(fb);
}

/* Product of two RNS polynomials [nl][n], limb i modulo q[i]; mode as set by
 * or_set_mul_mode.  Limbs are independent; OpenMP spreads them over cores. */
void or_poly_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, uint32_t n,
                 const uint64_t* q, const uint64_t* psi, uint32_t nl) {
    int mode = g_mul_mode;
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < (int)nl; ++i)
        or_mul_limb(a + (size_t)i * n, b + (size_t)i * n, out + (size_t)i * n, n, q[i], psi[i], mode);
}

/* Coefficient-wise product c_k = a_k * b_k mod q (one limb); used for
 * plaintext constants and for the transform domain inside or_mul_limb. */
void or_pointwise_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, uint64_t count, uint64_t q) {
    for (uint64_t k = 0; k < count; ++k) out[k] = mulmod(a[k], b[k], q);
}

/* c_k = a_k * c mod q (one limb) */
void or_scalar_mul(const uint64_t* a, uint64_t c, uint64_t* out, uint64_t count, uint64_t q) {
    for (uint64_t k = 0; k < count; ++k) out[k] = mulmod(a[k], c, q);
}

/* ---- X -> X^kappa in coefficient form (ROTATE, Sec. 3.4) -------------- */
/* Coefficient j of a moves to position j*kappa mod 2N; positions >= N wrap
 * with a sign flip because X^N = -1. kappa must be odd. */
void or_automorphism(const uint64_t* a, uint64_t* out, uint32_t n, uint64_t q, uint64_t kappa) {
    uint64_t two_n = 2ull * n;
    for (uint32_t j = 0; j < n; ++j) {
        uint64_t e = ((uint64_t)j * kappa) % two_n;
        uint64_t v = a[j] % q;
        if (e < n) out[e] = v;
        else out[e - n] = submod(0, v, q);
    }
}

/* ---- fast base conversion ------------------------------------------------
 * Source base {s_0..s_{m-1}} with product D, target primes {t_0..t_{r-1}}.
 * For every coefficient position k:
 *   xt_i = x_i[k] * (D/s_i)^-1 mod s_i
 *   Y    = sum_i xt_i * (D/s_i)            (an exact integer in [0, m*D))
 *   out_t[k] = Y mod t
 * which is computed as sum_i xt_i * ((D/s_i) mod t) mod t.  Y equals x mod D
 * plus u*D for some 0 <= u < m; the test suite checks that property against
 * big-integer CRT. */
void or_base_convert(const uint64_t* x, const uint64_t* src, uint32_t m,
                     const uint64_t* dst, uint32_t r, uint64_t* out, uint32_t n) {
    uint64_t* hat_inv = (uint64_t*)malloc(sizeof(uint64_t) * m);     /* (D/s_i)^-1 mod s_i */
    uint64_t* hat_mod = (uint64_t*)malloc(sizeof(uint64_t) * m * r); /* (D/s_i) mod t     */
    for (uint32_t i = 0; i < m; ++i) {
        uint64_t h = 1;
        for (uint32_t l = 0; l < m; ++l)
            if (l != i) h = mulmod(h, src[l] % src[i], src[i]);
        hat_inv[i] = or_invmod(h, src[i]);
        for (uint32_t t = 0; t < r; ++t) {
            uint64_t ht = 1;
            for (uint32_t l = 0; l < m; ++l)
                if (l != i) ht = mulmod(ht, src[l] % dst[t], dst[t]);
            hat_mod[(size_t)i * r + t] = ht;
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < (int64_t)n; ++k) {
        for (uint32_t t = 0; t < r; ++t) {
            uint64_t acc = 0;
            for (uint32_t i = 0; i < m; ++i) {
                uint64_t xt = mulmod(x[(size_t)i * n + k] % src[i], hat_inv[i], src[i]);
                acc = addmod(acc, mulmod(xt % dst[t], hat_mod[(size_t)i * r + t], dst[t]), dst[t]);
            }
            out[(size_t)t * n + k] = acc;
        }
    }
    free(hat_inv);
    free(hat_mod);
}

/* One coefficient of a negacyclic product, O(N): used by the test suite for
 * spot checks of mode 1 at N = 2^16 where the full schoolbook is too slow. */
uint64_t or_mul_coeff(const uint64_t* a, const uint64_t* b, uint32_t n, uint64_t q, uint32_t k) {
    uint64_t pos = 0, neg = 0;
    for (uint32_t i = 0; i <= k; ++i) pos = addmod(pos, mulmod(a[i], b[k - i], q), q);
    for (uint32_t i = k + 1; i < n; ++i) neg = addmod(neg, mulmod(a[i], b[n + k - i], q), q);
    return submod(pos, neg, q);
}
