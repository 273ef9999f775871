// ntt.hip -- negacyclic NTT / inverse NTT per RNS limb for gfx950.
//
// Forward: A[k] = sum_j a_j psi^((2 brv(k) + 1) j) (evaluation of a(X) at the
// odd powers of the primitive 2N-th root psi, bit-reversed order).  It is
// computed by log2(N) radix-2 stages; stage s (0-based) pairs index j with
// j + N/2^(s+1) and uses the twiddle psi^brv(2^s + (j >> (log2 N - s))).
// The inverse runs the stages backwards with Gentleman-Sande butterflies and
// psi^-brv(.) twiddles, and folds N^-1 into its last stage.
//
// Decomposition.  A pass executes a window of LOG_M consecutive stages.  The
// elements touched by those stages split into independent sub-problems of
// M = 2^LOG_M elements (fixed high index bits above the window, fixed low
// bits below it).  A 256-thread workgroup owns 4096 elements: C = 4096/M
// sub-problems, 16 elements per thread held in registers.  Inside a pass the
// stages run in phases of up to 4 (radix-16 in registers); between phases the
// elements are exchanged through LDS.  Global memory is read and written in
// a coalesced order through LDS (consecutive lanes touch consecutive
// addresses: along the sub-problem index when low bits exist, else along
// the sub-problem itself).
//   N = 2^12: one pass of 12 stages.   N = 2^13: 7 + 6.   N = 2^14: 7 + 7.
//   N = 2^15: 8 + 7.                   N = 2^16: 8 + 8.
// Butterflies keep residues lazily reduced (forward in [0, 4q), inverse in
// [0, 2q)); q < 2^60 leaves headroom.  Outputs of a full transform are in
// [0, q).
#include "pft_device.h"
#include "pft_kernels.h"

namespace {

// Harvey forward butterfly: X, Y in [0, 4q) -> X + WY, X - WY in [0, 4q).
__device__ __forceinline__ void fwd_bfly(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wp, uint64_t q,
                                         uint64_t two_q) {
    uint64_t x = X >= two_q ? X - two_q : X;
    uint64_t t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + two_q;
}

// Gentleman-Sande inverse butterfly: X, Y in [0, 2q) -> X + Y, (X - Y) W in [0, 2q).
__device__ __forceinline__ void inv_bfly(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wp, uint64_t q,
                                         uint64_t two_q) {
    uint64_t u = X + Y;
    u = u >= two_q ? u - two_q : u;
    uint64_t v = shoup_lazy(X + two_q - Y, w, wp, q);
    X = u;
    Y = v;
}

template <int LOG_M, int PH>
struct Phase {
    static constexpr int HB = LOG_M - 1 - 4 * PH;           // highest stage bit of this phase
    static constexpr int LB = (HB - 3 > 0) ? HB - 3 : 0;     // lowest stage bit
    static constexpr int WLO = (HB - 3 >= 0) ? HB - 3 : 0;  // window of the 16 register elements
    __device__ __forceinline__ static uint32_t r_of(uint32_t l, int e) {
        return ((l >> WLO) << (WLO + 4)) | ((uint32_t)e << WLO) | (l & ((1u << WLO) - 1u));
    }
};

template <int LOG_M, int PH, bool INV>
__device__ __forceinline__ void run_phase(uint64_t (&x)[16], uint32_t l, uint32_t high, uint32_t s0,
                                          const TwPair* __restrict__ twt, const DevMod& md, bool fold_last) {
    using Ph = Phase<LOG_M, PH>;
    const uint64_t q = md.q, two_q = md.two_q;
    if constexpr (!INV) {
#pragma unroll
        for (int bit = Ph::HB; bit >= Ph::LB; --bit) {
            const int spp = LOG_M - 1 - bit;
            const uint32_t s = s0 + spp;
            const int pos = bit - Ph::WLO;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                if (e & (1 << pos)) continue;
                const uint32_t r = Ph::r_of(l, e);
                const uint32_t i = (high << spp) | (r >> (bit + 1));
                const TwPair tp = twt[(1u << s) + i];
                fwd_bfly(x[e], x[e | (1 << pos)], tp.w, tp.wp, q, two_q);
            }
        }
    } else {
#pragma unroll
        for (int bit = Ph::LB; bit <= Ph::HB; ++bit) {
            const int spp = LOG_M - 1 - bit;
            const uint32_t s = s0 + spp;
            const int pos = bit - Ph::WLO;
            if (PH == 0 && bit == Ph::HB && fold_last) {
                // stage 0 with N^-1 folded in: outputs fully reduced
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    if (e & (1 << pos)) continue;
                    uint64_t X = x[e], Y = x[e | (1 << pos)];
                    uint64_t u = X + Y;
                    u = u >= two_q ? u - two_q : u;
                    x[e] = shoup(u, md.n_inv, md.n_inv_sh, q);
                    x[e | (1 << pos)] = shoup(X + two_q - Y, md.last_inv, md.last_inv_sh, q);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    if (e & (1 << pos)) continue;
                    const uint32_t r = Ph::r_of(l, e);
                    const uint32_t i = (high << spp) | (r >> (bit + 1));
                    const TwPair tp = twt[(1u << s) + i];
                    inv_bfly(x[e], x[e | (1 << pos)], tp.w, tp.wp, q, two_q);
                }
            }
        }
    }
}

template <int LOG_M, int PH>
__device__ __forceinline__ void lds_read(uint64_t (&x)[16], const uint64_t* lds, uint32_t c, uint32_t l) {
    constexpr int LDSW = (1 << LOG_M) + 1;
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = lds[c * LDSW + Phase<LOG_M, PH>::r_of(l, e)];
}
template <int LOG_M, int PH>
__device__ __forceinline__ void lds_write(const uint64_t (&x)[16], uint64_t* lds, uint32_t c, uint32_t l) {
    constexpr int LDSW = (1 << LOG_M) + 1;
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[c * LDSW + Phase<LOG_M, PH>::r_of(l, e)] = x[e];
}

template <int LOG_M, bool INV, int PH>
__device__ __forceinline__ void phases_fwd(uint64_t (&x)[16], uint64_t* lds, uint32_t c, uint32_t l, uint32_t high,
                                           uint32_t s0, const TwPair* __restrict__ twt, const DevMod& md) {
    constexpr int NPH = (LOG_M + 3) / 4;
    if constexpr (PH < NPH) {
        lds_read<LOG_M, PH>(x, lds, c, l);
        run_phase<LOG_M, PH, false>(x, l, high, s0, twt, md, false);
        lds_write<LOG_M, PH>(x, lds, c, l);
        __syncthreads();
        phases_fwd<LOG_M, INV, PH + 1>(x, lds, c, l, high, s0, twt, md);
    }
}

template <int LOG_M, int PH>
__device__ __forceinline__ void phases_inv(uint64_t (&x)[16], uint64_t* lds, uint32_t c, uint32_t l, uint32_t high,
                                           uint32_t s0, const TwPair* __restrict__ twt, const DevMod& md,
                                           bool fold_last) {
    if constexpr (PH >= 0) {
        lds_read<LOG_M, PH>(x, lds, c, l);
        run_phase<LOG_M, PH, true>(x, l, high, s0, twt, md, fold_last);
        lds_write<LOG_M, PH>(x, lds, c, l);
        __syncthreads();
        phases_inv<LOG_M, PH - 1>(x, lds, c, l, high, s0, twt, md, fold_last);
    }
}

template <int LOG_M, bool INV>
__global__ __launch_bounds__(256) void k_ntt_pass(PolyBatch b, const DevMod* __restrict__ mods,
                                                  const TwPair* __restrict__ tw, uint32_t log_n, uint32_t s0,
                                                  uint32_t final_pass) {
    constexpr int M = 1 << LOG_M;
    constexpr int T = M / 16;
    constexpr int C = 256 / T;
    constexpr int LDSW = M + 1;
    __shared__ uint64_t lds[C * LDSW];

    const uint32_t tid = threadIdx.x;
    const uint32_t job = blockIdx.y;
    const uint32_t limb = job / b.n_polys;
    const uint32_t poly = job - limb * b.n_polys;
    const uint32_t row = pb_row(b, poly, limb);
    const uint32_t mi = pb_mod(b, row);
    uint64_t* __restrict__ data = b.ptr[poly] + ((size_t)row << log_n);
    const DevMod md = mods[mi];
    const TwPair* __restrict__ twt = tw + ((size_t)mi << log_n);

    const uint32_t lbits = log_n - s0 - LOG_M;
    const uint32_t lmask = (1u << lbits) - 1u;
    const uint32_t sp0 = blockIdx.x * C;

    // coalesced global -> LDS
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t idx = tid + 256u * k;
        uint32_t c, r;
        if (lbits > 0) {
            c = idx % C;
            r = idx / C;
        } else {
            c = idx / M;
            r = idx % M;
        }
        const uint32_t sp = sp0 + c;
        const size_t j = ((((size_t)(sp >> lbits) << LOG_M) | r) << lbits) | (sp & lmask);
        lds[c * LDSW + r] = data[j];
    }
    __syncthreads();

    const uint32_t c = tid / T, l = tid % T;
    const uint32_t high = (sp0 + c) >> lbits;
    uint64_t x[16];
    if constexpr (!INV) {
        phases_fwd<LOG_M, INV, 0>(x, lds, c, l, high, s0, twt, md);
    } else {
        constexpr int NPH = (LOG_M + 3) / 4;
        phases_inv<LOG_M, NPH - 1>(x, lds, c, l, high, s0, twt, md, final_pass != 0 && s0 == 0);
    }

    // LDS -> global, coalesced
    const uint64_t q = md.q, two_q = md.two_q;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t idx = tid + 256u * k;
        uint32_t cc, r;
        if (lbits > 0) {
            cc = idx % C;
            r = idx / C;
        } else {
            cc = idx / M;
            r = idx % M;
        }
        const uint32_t sp = sp0 + cc;
        const size_t j = ((((size_t)(sp >> lbits) << LOG_M) | r) << lbits) | (sp & lmask);
        uint64_t v = lds[cc * LDSW + r];
        if (!INV && final_pass) {
            v = v >= two_q ? v - two_q : v;
            v = v >= q ? v - q : v;
        }
        data[j] = v;
    }
}

template <int LOG_M, bool INV>
void launch_pass(const PolyBatch& b, const DevTables& t, uint32_t log_n, uint32_t s0, bool final_pass,
                 hipStream_t st, ProfHook* g_prof) {
    const uint32_t jobs = b.n_polys * b.n_limbs;
    dim3 grid((1u << log_n) / 4096u, jobs);
    const int kid = INV ? PK_NTT_INV : PK_NTT_FWD;
    if (g_prof) g_prof->begin(kid);
    hipLaunchKernelGGL((k_ntt_pass<LOG_M, INV>), grid, dim3(256), 0, st, b, t.mods, INV ? t.tw_inv : t.tw_fwd,
                       log_n, s0, (uint32_t)final_pass);
    if (g_prof) {
        const double elems = (double)jobs * (double)(1u << log_n);
        // read + write every residue once; N/2 butterflies per stage
        g_prof->end(kid, 16.0 * elems, 0.5 * elems * LOG_M);
    }
}

}  // namespace

bool ntt_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 16; }

void launch_ntt(const PolyBatch& b, const DevTables& t, uint32_t log_n, bool inverse, hipStream_t st,
                ProfHook* prof) {
    if (b.n_polys == 0 || b.n_limbs == 0) return;
    if (!inverse) {
        switch (log_n) {
            case 12: launch_pass<12, false>(b, t, 12, 0, true, st, prof); break;
            case 13: launch_pass<7, false>(b, t, 13, 0, false, st, prof); launch_pass<6, false>(b, t, 13, 7, true, st, prof); break;
            case 14: launch_pass<7, false>(b, t, 14, 0, false, st, prof); launch_pass<7, false>(b, t, 14, 7, true, st, prof); break;
            case 15: launch_pass<8, false>(b, t, 15, 0, false, st, prof); launch_pass<7, false>(b, t, 15, 8, true, st, prof); break;
            case 16: launch_pass<8, false>(b, t, 16, 0, false, st, prof); launch_pass<8, false>(b, t, 16, 8, true, st, prof); break;
            default: break;
        }
    } else {
        switch (log_n) {
            case 12: launch_pass<12, true>(b, t, 12, 0, true, st, prof); break;
            case 13: launch_pass<6, true>(b, t, 13, 7, false, st, prof); launch_pass<7, true>(b, t, 13, 0, true, st, prof); break;
            case 14: launch_pass<7, true>(b, t, 14, 7, false, st, prof); launch_pass<7, true>(b, t, 14, 0, true, st, prof); break;
            case 15: launch_pass<7, true>(b, t, 15, 8, false, st, prof); launch_pass<8, true>(b, t, 15, 0, true, st, prof); break;
            case 16: launch_pass<8, true>(b, t, 16, 8, false, st, prof); launch_pass<8, true>(b, t, 16, 0, true, st, prof); break;
            default: break;
        }
    }
}
