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
// the sub-problem itself).  The split of the stages into passes is a
// schedule (ntt_candidates below lists them per N; the first is the default,
// e.g. one pass of 12 stages at N = 2^12 and 8 + 8 at N = 2^16); a
// context's autotuner or a tuning table picks one per direction and batch
// size (the large-ring workload uses 4 + 12 for its forward transforms).
// Arithmetic, chosen per limb (uniform within a workgroup):
//   * q < 2^50: fp64.  A residue fits the 53-bit significand, and MI355X issues
//     fp64 FMA at the full VALU rate, so an exact product modulo q costs six
//     fp64 instructions instead of some twenty 32-bit integer ones (bounds at
//     fmulmod below).
//   * otherwise (q < 2^60): 64-bit integer Shoup butterflies kept lazily
//     reduced (forward below 8q inside a pass and below 4q between passes,
//     inverse in [0, 2q)).
// Inputs below 4q are accepted; outputs of a full transform are in [0, q).
#include "bconv_device.h"
#include "pft_device.h"
#include "pft_kernels.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <vector>

namespace {

// ---- integer butterflies (any q < 2^60)

// Harvey forward butterflies (WY by Shoup, below 2q for any Y < 2^64).
// Without reducing X: X + WY and X - WY + 2q stay below B + 2q for X, Y
// below B.
__device__ __forceinline__ void fwd_bfly_low(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wp, uint64_t q,
                                             uint64_t two_q) {
    const uint64_t x = X;
    const uint64_t t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + two_q;
}
// The same with X below 8q reduced below 2q in two steps.
__device__ __forceinline__ void fwd_bfly_r8(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wp, uint64_t q,
                                            uint64_t two_q) {
    const uint64_t four_q = two_q << 1;
    uint64_t x = X >= four_q ? X - four_q : X;
    x = x >= two_q ? x - two_q : x;
    const uint64_t t = shoup_lazy(Y, w, wp, q);
    X = x + t;
    Y = x - t + two_q;
}
// Integer forward stages of a pass reduce X only at stages spp with
// (LOG_M - 1 - spp) divisible by 3, counted from the pass's last stage so
// that the last stage reduces: from inputs below 4q, the (at most two)
// stages before a reducing one leave values below 6q and 8q (< 2^63 for q
// < 2^60), the reducing stage brings X below 2q in two steps, and every
// pass ends below 4q as with a reduction at every stage.
__device__ __forceinline__ constexpr bool int_fwd_reduces(int log_m, int spp) { return (log_m - 1 - spp) % 3 == 0; }

// Gentleman-Sande inverse butterfly: X, Y in [0, 2q) -> X + Y, (X - Y) W in [0, 2q).
__device__ __forceinline__ void inv_bfly(uint64_t& X, uint64_t& Y, uint64_t w, uint64_t wp, uint64_t q,
                                         uint64_t two_q) {
    uint64_t u = X + Y;
    u = u >= two_q ? u - two_q : u;
    uint64_t v = shoup_lazy(X + two_q - Y, w, wp, q);
    X = u;
    Y = v;
}

// ---- fp64 butterflies (q < 2^50): fmulmod / freduce in pft_device.h
// Forward: X is reduced on every third stage of a pass (pass-local stage
// index = 0 mod 3).  With inputs within B q a reducing stage leaves
// (1 + B/4) q and a skipping one (5B/4 + 1/2) q.  A pass starts with a
// reducing stage, so at most two skipping stages follow one another; from
// inputs below 4q the bound settles at 2.1q after a reducing stage and stays
// below 4.5q (|values| < 2^53, and fmulmod's quotient is then off by at most
// 1/2 + 4.5/4, so every step stays exact).
__device__ __forceinline__ void fwd_bfly_fp(uint64_t& X, uint64_t& Y, const TwPair& tp, double q, double qinv,
                                            bool reduce_x) {
#pragma clang fp contract(off)
    const double x = reduce_x ? freduce(as_f(X), q, qinv) : as_f(X);
    const double t = fmulmod(as_f(Y), as_f(tp.w), as_f(tp.wp), q);
    X = as_u(x + t);
    Y = as_u(x - t);
}
// Inverse: X + Y is left unreduced on every third stage of a pass (stages in
// execution order, index = 2 mod 3).  Inputs within B q give X within q/2
// (reduced) or 2B q (not), Y within (1/2 + B/2) q; with two reducing stages
// between skipping ones the bound settles at 1.5q and stays below 4q.
__device__ __forceinline__ void inv_bfly_fp(uint64_t& X, uint64_t& Y, const TwPair& tp, double q, double qinv,
                                            bool reduce_x) {
#pragma clang fp contract(off)
    const double x = as_f(X), y = as_f(Y);
    X = as_u(reduce_x ? freduce(x + y, q, qinv) : x + y);
    Y = as_u(fmulmod(x - y, as_f(tp.w), as_f(tp.wp), q));
}
// Register phase PH of a radix-2^LOG_M pass with E = 2^EB residues per
// thread: stage bits HB down to LB; element e of thread l is index r_of(l, e)
// of its sub-problem (the EB window bits sit at WLO).
template <int LOG_M, int PH, int EB>
struct Phase {
    static constexpr int HB = LOG_M - 1 - EB * PH;                       // highest stage bit of this phase
    static constexpr int LB = (HB - (EB - 1) > 0) ? HB - (EB - 1) : 0;   // lowest stage bit
    static constexpr int WLO = (HB - (EB - 1) >= 0) ? HB - (EB - 1) : 0; // window of the register elements
    __device__ __forceinline__ static uint32_t r_of(uint32_t l, int e) {
        return ((l >> WLO) << (WLO + EB)) | ((uint32_t)e << WLO) | (l & ((1u << WLO) - 1u));
    }
};

// Twiddle index (high << spp) | (r >> (bit + 1)) of the butterfly at stage
// bit `bit` whose upper element is register e (r = r_of(l, e)).  The lane
// bits below the window drop out of the shift; in the phase that holds the
// window's top bits no lane bit is left, so the index is the same for every
// lane of a sub-problem.
template <int LOG_M, int PH, int EB>
__device__ __forceinline__ uint32_t tw_index(uint32_t l, int e, int bit, uint32_t high, int spp) {
    using Ph = Phase<LOG_M, PH, EB>;
    const uint32_t lhi = (Ph::WLO + EB >= LOG_M) ? 0u : (l >> Ph::WLO);
    return (high << spp) | (lhi << (Ph::WLO + EB - bit - 1)) | ((uint32_t)e >> (bit + 1 - Ph::WLO));
}

// Twiddles preloaded per register phase ahead of the exchange before it
// (PhaseTw below): by the transform passes with 8 or 16 residues per
// thread, and by the fused inner product (fp64 rows two digits or one per
// pass, 60-bit rows); larger budgets spill or cost waves per SIMD.
constexpr int TW_PRE_PASS3 = 8;
constexpr int TW_PRE_PASS4 = 3;
constexpr int TW_PRE_INNER_FP2 = 3;
constexpr int TW_PRE_INNER_FP1 = 1;
constexpr int TW_PRE_INNER_INT = 1;
constexpr int tw_pre_pass(int eb) { return eb == 3 ? TW_PRE_PASS3 : eb == 4 ? TW_PRE_PASS4 : 0; }
constexpr int tw_pre_inner(bool fp, int g) {
    return fp ? (g == 2 ? TW_PRE_INNER_FP2 : TW_PRE_INNER_FP1) : TW_PRE_INNER_INT;
}
// The twiddles of register phase PH for one thread.  At the stage whose
// butterflies span window bit pos, the upper elements e that agree in
// e >> (pos + 1) share one twiddle (tw_index drops the bits below), so the
// stage needs E >> (pos + 1) of them.  The first stages in execution order,
// up to PRE twiddles, are loaded by the constructor: a pass builds the set
// of its next phase before the LDS exchange that precedes that phase, so the
// loads are in flight during the exchange and its barrier (the fences of
// the exchange would keep the compiler from moving them there itself).  The
// later stages load at use.  The inverse transform's final stage with N^-1
// folded in (FOLD, phase 0, top bit) uses none.
template <int LOG_M, int PH, int EB, bool INV, bool FOLD, int PRE = 8>
struct PhaseTw {
    using Ph = Phase<LOG_M, PH, EB>;
    static constexpr int E = 1 << EB;
    static constexpr int P_HI = Ph::HB - Ph::WLO;  // window positions 0 .. P_HI
    static constexpr int MAXPRE = PRE;
    static constexpr int cnt(int pos) { return (INV && FOLD && PH == 0 && pos == P_HI) ? 0 : E >> (pos + 1); }
    struct Layout {
        int base[8];
        bool pre[8];
        int total;
    };
    static constexpr Layout layout() {
        Layout y{};
        int n = 0;
        bool open = true;
        for (int k = 0; k <= P_HI; ++k) {
            const int pos = INV ? k : P_HI - k;
            const int c = cnt(pos);
            if (open && n + c <= MAXPRE) {
                y.base[pos] = n;
                y.pre[pos] = true;
                n += c;
            } else {
                open = false;
                y.base[pos] = 0;
                y.pre[pos] = false;
            }
        }
        y.total = n;
        return y;
    }
    static constexpr Layout LY = layout();
    TwPair t[LY.total > 0 ? LY.total : 1];
    const TwPair* __restrict__ twt;
    uint32_t l, high, s0;

    __device__ __forceinline__ PhaseTw(const TwPair* __restrict__ tw, uint32_t l_, uint32_t high_, uint32_t s0_)
        : twt(tw), l(l_), high(high_), s0(s0_) {
#pragma unroll
        for (int pos = 0; pos <= P_HI; ++pos) {
            if (!LY.pre[pos]) continue;
#pragma unroll
            for (int m = 0; m < cnt(pos); ++m) t[LY.base[pos] + m] = load(pos, m << (pos + 1));
        }
    }
    __device__ __forceinline__ TwPair load(int pos, int e) const {
        const int bit = pos + Ph::WLO;
        const int spp = LOG_M - 1 - bit;
        return twt[(1u << (s0 + (uint32_t)spp)) + tw_index<LOG_M, PH, EB>(l, e, bit, high, spp)];
    }
    // the twiddle of the butterfly at window bit pos whose upper element is e
    __device__ __forceinline__ TwPair get(int pos, int e) const {
        if (LY.pre[pos]) return t[LY.base[pos] + (e >> (pos + 1))];
        return load(pos, e);
    }
};

// LOW (forward only): the inputs are already reduced (fp64 within q/2 + 1
// or below q; integers below 2q), so the first stage skips its reduction of
// X; the bounds of the later stages are those of reduced inputs.
template <int LOG_M, int PH, int EB, bool INV, bool FP, bool FOLD, int PRE, bool LOW = false>
__device__ __forceinline__ void run_phase(uint64_t (&x)[1 << EB], const PhaseTw<LOG_M, PH, EB, INV, FOLD, PRE>& tw,
                                          const DevMod& md) {
    static_assert(!LOW || (!INV && PH == 0), "reduced inputs enter the first forward phase");
    using Ph = Phase<LOG_M, PH, EB>;
    constexpr int E = 1 << EB;
    const uint64_t q = md.q, two_q = md.two_q;
    const double qd = md.qd, qinv = md.qinv;
    if constexpr (!INV) {
#pragma unroll
        for (int bit = Ph::HB; bit >= Ph::LB; --bit) {
            const int spp = LOG_M - 1 - bit;
            const int pos = bit - Ph::WLO;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (e & (1 << pos)) continue;
                const TwPair tp = tw.get(pos, e);
                const bool first = LOW && PH == 0 && spp == 0;  // folded after unrolling
                if constexpr (FP)
                    fwd_bfly_fp(x[e], x[e | (1 << pos)], tp, qd, qinv, spp % 3 == 0 && !first);
                else if (first || !int_fwd_reduces(LOG_M, spp))
                    fwd_bfly_low(x[e], x[e | (1 << pos)], tp.w, tp.wp, q, two_q);
                else
                    fwd_bfly_r8(x[e], x[e | (1 << pos)], tp.w, tp.wp, q, two_q);
            }
        }
    } else {
#pragma unroll
        for (int bit = Ph::LB; bit <= Ph::HB; ++bit) {
            const int pos = bit - Ph::WLO;
            if (FOLD && PH == 0 && bit == Ph::HB) {
                // stage 0 with N^-1 folded in (integer path: outputs fully reduced)
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & (1 << pos)) continue;
                    uint64_t X = x[e], Y = x[e | (1 << pos)];
                    if constexpr (FP) {
                        const double a = as_f(X), b2 = as_f(Y);
                        x[e] = as_u(fmulmod(a + b2, md.n_inv_d, md.n_inv_q, qd));
                        x[e | (1 << pos)] = as_u(fmulmod(a - b2, md.last_inv_d, md.last_inv_q, qd));
                    } else {
                        uint64_t u = X + Y;
                        u = u >= two_q ? u - two_q : u;
                        x[e] = shoup(u, md.n_inv, md.n_inv_sh, q);
                        x[e | (1 << pos)] = shoup(X + two_q - Y, md.last_inv, md.last_inv_sh, q);
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if (e & (1 << pos)) continue;
                    const TwPair tp = tw.get(pos, e);
                    if constexpr (FP)
                        inv_bfly_fp(x[e], x[e | (1 << pos)], tp, qd, qinv, bit % 3 != 2);
                    else
                        inv_bfly(x[e], x[e | (1 << pos)], tp.w, tp.wp, q, two_q);
                }
            }
        }
    }
}

// One register phase loading each twiddle at its use (a single-phase pass:
// with no exchange in the way the compiler schedules the loads itself).
template <int LOG_M, int PH, int EB, bool INV, bool FP, bool FOLD, bool LOW = false>
__device__ __forceinline__ void run_phase(uint64_t (&x)[1 << EB], uint32_t l, uint32_t high, uint32_t s0,
                                          const TwPair* __restrict__ twt, const DevMod& md) {
    const PhaseTw<LOG_M, PH, EB, INV, FOLD, 0> tw(twt, l, high, s0);
    run_phase<LOG_M, PH, EB, INV, FP, FOLD, 0, LOW>(x, tw, md);
}

// LDS word of element r of sub-problem c: c S + r + P (r >> 4), or, where
// the 8-byte words of a 16-lane group cannot all be spread over distinct
// bank pairs by a padding, c S + (r ^ h(r)) with h(r) = ((r >> XA) & 7) |
// (((r >> XB) & 1) << 3): the low four bits of r are permuted by higher
// ones (a bijection within each sub-problem).  The padded form is affine in
// the register index e of every arrangement (so ds_read/ds_write take
// immediate offsets).  The parameters are chosen per (M, residues per
// thread) by an exhaustive model of the LDS serving 16 lanes x 8 bytes per
// cycle over every access pattern of the pass -- each register phase's
// arrangement under both lane mappings, the staging order and the
// element-pair order of the staged store: with 16 residues per thread every
// row-pass pattern is conflict-free (radix 6 and 7 keep a two-way conflict
// on one), and with 8 the swizzled forms make the row passes of radix 7-12
// conflict-free where any padding leaves two-way conflicts (radix 9 and 10
// keep one two-way conflict pattern as column passes).
template <int LOG_M, int EB> struct LdsPad;
template <int EB> struct LdsPad<4, EB> { static constexpr uint32_t S = 17, P = 0, XA = 0, XB = 0; };
template <> struct LdsPad<6, 4> { static constexpr uint32_t S = 69, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<6, 3> { static constexpr uint32_t S = 73, P = 2, XA = 0, XB = 0; };
template <> struct LdsPad<7, 4> { static constexpr uint32_t S = 145, P = 2, XA = 0, XB = 0; };
template <> struct LdsPad<7, 3> { static constexpr uint32_t S = 129, P = 0, XA = 4, XB = 4; };
template <int EB> struct LdsPad<8, EB> { static constexpr uint32_t S = 273, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<8, 3> { static constexpr uint32_t S = 257, P = 0, XA = 4, XB = 5; };
template <int EB> struct LdsPad<9, EB> { static constexpr uint32_t S = 546, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<9, 3> { static constexpr uint32_t S = 514, P = 0, XA = 4, XB = 6; };
template <int EB> struct LdsPad<10, EB> { static constexpr uint32_t S = 1092, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<10, 3> { static constexpr uint32_t S = 1026, P = 0, XA = 4, XB = 4; };
template <int EB> struct LdsPad<11, EB> { static constexpr uint32_t S = 2176, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<11, 3> { static constexpr uint32_t S = 2048, P = 0, XA = 4, XB = 5; };
template <int EB> struct LdsPad<12, EB> { static constexpr uint32_t S = 4352, P = 1, XA = 0, XB = 0; };
template <> struct LdsPad<12, 3> { static constexpr uint32_t S = 4096, P = 0, XA = 4, XB = 6; };
template <int LOG_M, int EB>
constexpr uint32_t lds_words() { return (4096u >> LOG_M) * LdsPad<LOG_M, EB>::S; }
template <int LOG_M, int EB>
__device__ __forceinline__ uint32_t lds_at(uint32_t c, uint32_t r) {
    using L = LdsPad<LOG_M, EB>;
    if constexpr (L::XA != 0)
        return c * L::S + (r ^ (((r >> L::XA) & 7u) | (((r >> L::XB) & 1u) << 3)));
    else
        return c * L::S + r + L::P * (r >> 4);
}

template <int LOG_M, int PH, int EB>
__device__ __forceinline__ void lds_read(uint64_t (&x)[1 << EB], const uint64_t* lds, uint32_t c, uint32_t l) {
#pragma unroll
    for (int e = 0; e < (1 << EB); ++e) x[e] = lds[lds_at<LOG_M, EB>(c, Phase<LOG_M, PH, EB>::r_of(l, e))];
}
template <int LOG_M, int PH, int EB>
__device__ __forceinline__ void lds_write(const uint64_t (&x)[1 << EB], uint64_t* lds, uint32_t c, uint32_t l) {
#pragma unroll
    for (int e = 0; e < (1 << EB); ++e) lds[lds_at<LOG_M, EB>(c, Phase<LOG_M, PH, EB>::r_of(l, e))] = x[e];
}

// Where thread-index bit b lands in the word index c M + r of register
// phase PH (COL: c = tid mod C, l = tid / C; otherwise c = tid / T, l =
// tid mod T; r = Phase::r_of(l, e)).
template <int LOG_M, int EB, bool COL>
constexpr int tid_bit_pos(int ph, int b) {
    constexpr int LT = LOG_M - EB;  // log2 of the threads per sub-problem
    constexpr int LC = 12 - LOG_M;  // log2 of the sub-problems per workgroup
    const int hb = LOG_M - 1 - EB * ph;
    const int wlo = hb - (EB - 1) >= 0 ? hb - (EB - 1) : 0;
    int lb = 0;
    if (COL) {
        if (b < LC) return LOG_M + b;
        lb = b - LC;
    } else {
        if (b >= LT) return LOG_M + (b - LT);
        lb = b;
    }
    return lb < wlo ? lb : lb + EB;
}
// Whether the exchange between register phases pa and pb stays inside each
// wave: every wave reads back exactly the words it wrote (its wave-index
// bits land on the same word-index bits in both phases, and its lane bits
// and element window cover the same set).  Such an exchange needs no
// workgroup barrier: a wave's LDS instructions execute in order, so its
// reads see its own earlier writes, and no other wave touches those words.
template <int LOG_M, int EB, bool COL>
constexpr bool wave_local_exchange(int pa, int pb) {
    constexpr int LNT = 12 - EB;  // log2 of the threads per workgroup
    if (LNT <= 6) return true;
    for (int b = 6; b < LNT; ++b)
        if (tid_bit_pos<LOG_M, EB, COL>(pa, b) != tid_bit_pos<LOG_M, EB, COL>(pb, b)) return false;
    auto varying = [](int ph) {
        const int hb = LOG_M - 1 - EB * ph;
        const int wlo = hb - (EB - 1) >= 0 ? hb - (EB - 1) : 0;
        uint32_t m = ((1u << EB) - 1u) << wlo;
        for (int b = 0; b < 6; ++b) m |= 1u << tid_bit_pos<LOG_M, EB, COL>(ph, b);
        return m;
    };
    return varying(pa) == varying(pb);
}
// Orders a wave's LDS writes before its following reads without a
// workgroup barrier (the compiler must not move memory accesses across it).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The register phases of one pass in execution order (forward: 0, 1, ...;
// inverse: the reverse), with an LDS exchange between consecutive phases.
// Each thread writes back to the words it read last, so one barrier per
// exchange suffices; an exchange that stays inside each wave needs none.
template <int LOG_M, int EB, bool INV, bool FP, bool FOLD, int K, bool COL = false, int PRE = 0>
__device__ __forceinline__ void run_phases(uint64_t (&x)[1 << EB], uint64_t* lds, uint32_t c, uint32_t l,
                                           uint32_t high, uint32_t s0, const TwPair* __restrict__ twt,
                                           const DevMod& md) {
    constexpr int NPH = (LOG_M + EB - 1) / EB;
    if constexpr (K < NPH) {
        constexpr int PH = INV ? NPH - 1 - K : K;
        // the phase's twiddle loads go out before the exchange
        const PhaseTw<LOG_M, PH, EB, INV, FOLD, PRE> tw(twt, l, high, s0);
        if constexpr (K > 0) {
            constexpr int PREV = INV ? PH + 1 : PH - 1;
            lds_write<LOG_M, PREV, EB>(x, lds, c, l);
            if constexpr (wave_local_exchange<LOG_M, EB, COL>(PREV, PH))
                wave_lds_sync();
            else
                __syncthreads();
            lds_read<LOG_M, PH, EB>(x, lds, c, l);
        }
        run_phase<LOG_M, PH, EB, INV, FP, FOLD, PRE>(x, tw, md);
        run_phases<LOG_M, EB, INV, FP, FOLD, K + 1, COL, PRE>(x, lds, c, l, high, s0, twt, md);
    }
}

// X -> X^kappa on an NTT-domain row (entry k holds the evaluation at
// psi^(2 brv(k) + 1)) is the gather out[k] = in[sigma(k)] with
// sigma(k) = brv(((2 brv(k) + 1) kappa mod 2N - 1) / 2).  In natural order
// the map is affine modulo N, so the low bits of the image depend only on
// the low bits of the argument; in bit-reversed order the high bits of
// sigma(k) depend only on the high bits of k: every aligned 4096-word tile
// of the result comes from one aligned tile of the input.  This stages
// destination tile `tile` of the result in LDS (in the pass's LDS layout):
// the source tile is read coalesced and word k of it is written at
// pi(k) = sigma^-1(k) (kappa_inv in place of kappa), converted to the fp64
// form if to_fp.  Ends with a barrier.
__device__ __forceinline__ uint32_t galois_index(uint32_t k, uint32_t kap, uint32_t log_n) {
    const uint32_t e = 2u * brev_n(k, log_n) + 1u;
    const uint32_t e2 = (e * kap) & ((2u << log_n) - 1u);  // 2N divides 2^32: the low product bits suffice
    return brev_n((e2 - 1u) >> 1, log_n);
}
template <int LOG_M, int EB>
__device__ __forceinline__ void galois_tile_to_lds(const uint64_t* __restrict__ src, uint32_t tile, uint32_t log_n,
                                                   uint64_t kappa, uint64_t kappa_inv, uint64_t* lds, bool to_fp) {
    constexpr uint32_t NT = 4096 >> EB;
    constexpr int E = 1 << EB;
    constexpr uint32_t M = 1u << LOG_M;
    const uint32_t st = galois_index(tile << 12, (uint32_t)kappa, log_n) >> 12;
    const uint64_t* __restrict__ s = src + ((size_t)st << 12);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t idx = threadIdx.x + NT * (uint32_t)k;
        const uint32_t d = galois_index((st << 12) + idx, (uint32_t)kappa_inv, log_n) - (tile << 12);
        const uint64_t v = s[idx];
        lds[lds_at<LOG_M, EB>(d / M, d % M)] = to_fp ? fp_from_u64(v) : v;
    }
    __syncthreads();
}

// One pass over stages s0 .. s0 + LOG_M - 1 of a 4096-element tile.
// COL (stages below log_n - LOG_M leave low index bits: the M elements of a
// sub-problem are 2^lbits apart): consecutive lanes take consecutive
// sub-problems, so every register arrangement is a coalesced global access
// and the pass loads and stores directly.  Row passes (lbits = 0, each
// sub-problem contiguous): consecutive lanes walk along a sub-problem.  With
// STAGE, a side whose arrangement gives runs shorter than 16 words goes
// through LDS in address order; without, it is accessed directly, and the
// arrangement in which each thread owns 16 consecutive words (the window's
// lowest stages) moves 16 bytes per lane per access.
// Limbs with DevMod::fp run the fp64 butterflies: the first pass of a
// transform converts its u64 input, later passes exchange the doubles through
// HBM, and the final pass writes canonical u64.  Integer limbs keep u64.
// PERM (row passes only): X -> X^kappa of NttEpilogue folded in.  Inverse
// (the transform's first pass): the input of polynomial p is row i of
// ep.perm_src[p] through the permutation.  Forward with EPI: the first
// polynomial of item z also adds row i of ep.perm_src[z] through the
// permutation (the ROTATE's X^kappa image of c0).
template <int LOG_M, int EB, bool INV, bool COL, bool FINAL, bool STAGE, bool EPI, bool PERM = false>
__global__ __launch_bounds__(4096 >> EB) void k_ntt_pass(PolyBatch b, const DevMod* __restrict__ mods,
                                                         const TwPair* __restrict__ tw, uint32_t log_n, uint32_t s0,
                                                         uint32_t first_pass, NttEpilogue ep) {
    static_assert(!PERM || (!COL && (INV || EPI)), "the permutation is folded into row passes");
    constexpr int M = 1 << LOG_M;
    constexpr int E = 1 << EB;          // residues per thread
    constexpr uint32_t NT = 4096 >> EB;  // threads per workgroup
    constexpr int T = M / E;             // threads per sub-problem
    constexpr int C = NT / T;            // sub-problems per workgroup
    constexpr int NPH = (LOG_M + EB - 1) / EB;
    constexpr int PH_IN = INV ? NPH - 1 : 0;
    constexpr int PH_OUT = INV ? 0 : NPH - 1;
    using PIN = Phase<LOG_M, PH_IN, EB>;
    using POUT = Phase<LOG_M, PH_OUT, EB>;
    constexpr bool DIRECT_IN = COL || !STAGE || PIN::WLO >= 4;
    constexpr bool DIRECT_OUT = COL || !STAGE || POUT::WLO >= 4;
    // a row-pass arrangement where thread l owns words E l .. E l + E - 1
    constexpr bool VEC_IN = !COL && PIN::WLO == 0;
    constexpr bool VEC_OUT = !COL && POUT::WLO == 0;
    __shared__ uint64_t lds[lds_words<LOG_M, EB>()];

    const uint32_t tid = threadIdx.x;
    const uint32_t job = blockIdx.y;
    const uint32_t limb = job / b.n_polys;
    const uint32_t poly = job - limb * b.n_polys;
    const uint32_t row = pb_row(b, poly, limb);
    const uint32_t mi = pb_mod(b, row);
    uint64_t* __restrict__ data = b.ptr[poly] + ((size_t)row << log_n);
    const DevMod md = mods[mi];
    const bool fp = md.fp != 0;
    const TwPair* __restrict__ twt = tw + ((size_t)mi << log_n);

    // a row pass has no index bits below its window (s0 + LOG_M = log_n)
    const uint32_t lbits = COL ? log_n - s0 - LOG_M : 0u;
    const uint32_t lmask = (1u << lbits) - 1u;
    const uint32_t sp0 = blockIdx.x * C;
    const uint32_t c = C == 1 ? 0u : (COL ? tid % C : tid / T);
    const uint32_t l = C == 1 ? tid : (COL ? tid / C : tid % T);
    const uint32_t high = (sp0 + c) >> lbits;
    // global index of element r of the workgroup's sub-problem cc
    auto gidx = [&](uint32_t cc, uint32_t r) -> size_t {
        const uint32_t sp = sp0 + cc;
        return ((((size_t)(sp >> lbits) << LOG_M) | r) << lbits) | (sp & lmask);
    };

    uint64_t x[E];
    const bool convert_in = fp && first_pass;
    const uint64_t* src = first_pass ? data + b.src_delta : data;  // may alias data (in place)
    if constexpr (PERM && INV) {
        galois_tile_to_lds<LOG_M, EB>(ep.perm_src[poly] + ((size_t)row << log_n), blockIdx.x, log_n, ep.kappa,
                                      ep.kappa_inv, lds, convert_in);
        lds_read<LOG_M, PH_IN, EB>(x, lds, c, l);
    } else if constexpr (DIRECT_IN && VEC_IN) {
        const ulonglong2* __restrict__ srcv = reinterpret_cast<const ulonglong2*>(src + gidx(c, (uint32_t)E * l));
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const ulonglong2 v = srcv[e];
            x[2 * e] = convert_in ? fp_from_u64(v.x) : v.x;
            x[2 * e + 1] = convert_in ? fp_from_u64(v.y) : v.y;
        }
    } else if constexpr (DIRECT_IN) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint64_t v = src[gidx(c, PIN::r_of(l, e))];
            x[e] = convert_in ? fp_from_u64(v) : v;
        }
    } else {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t idx = tid + NT * k;
            const uint32_t cc = idx / M, r = idx % M;
            const uint64_t v = src[gidx(cc, r)];
            lds[lds_at<LOG_M, EB>(cc, r)] = convert_in ? fp_from_u64(v) : v;
        }
        __syncthreads();
        lds_read<LOG_M, PH_IN, EB>(x, lds, c, l);
    }

    // the final inverse pass (s0 = 0) folds N^-1 into stage 0
    if (fp)
        run_phases<LOG_M, EB, INV, true, FINAL, 0, COL, tw_pre_pass(EB)>(x, lds, c, l, high, s0, twt, md);
    else
        run_phases<LOG_M, EB, INV, false, FINAL, 0, COL, tw_pre_pass(EB)>(x, lds, c, l, high, s0, twt, md);

    const uint64_t q = md.q, two_q = md.two_q;
    const double qd = md.qd, qinv = md.qinv;
    auto finish = [&](uint64_t v) -> uint64_t {
        if constexpr (FINAL) {
            if (fp) {
                v = fp_to_u64(v, qd, qinv);
            } else if constexpr (!INV) {
                v = v >= two_q ? v - two_q : v;
                v = v >= q ? v - q : v;
            }
        }
        return v;
    };
    // ModDown / RESCALE epilogue operands (uniform per workgroup)
    [[maybe_unused]] const uint32_t bsel = poly & 1u;
    [[maybe_unused]] uint64_t* __restrict__ out_row =
        EPI ? ep.out[poly >> 1] + ((size_t)(bsel * ep.level + row) << log_n) : nullptr;
    [[maybe_unused]] const TwPair pinv = EPI ? (fp ? ep.pinv_fp[row] : ep.pinv[row]) : TwPair{0, 0};
    [[maybe_unused]] const uint64_t* __restrict__ acc_src = nullptr;
    [[maybe_unused]] const uint64_t* __restrict__ add_src = nullptr;
    [[maybe_unused]] const uint64_t* __restrict__ add2_src = nullptr;
    if constexpr (EPI) {
        acc_src = ep.d_acc[bsel] == PFT_EPI_ITEM_ACC
                      ? ep.acc_item[poly >> 1] + ((size_t)(bsel * ep.acc_level + row) << log_n)
                      : data + ep.d_acc[bsel];
        if (ep.d_add[bsel] != PFT_EPI_NO_ADD) add_src = data + ep.d_add[bsel];
        if (ep.d_add2[bsel] != PFT_EPI_NO_ADD) add2_src = data + ep.d_add2[bsel];
    }
    // Epilogue stores of the E elements pos(k) with register forms val(k)
    // (integer-valued doubles within 4.5q for fp64 limbs; finish() reduces
    // integer limbs).  Every load of a chunk is issued before the first
    // result is formed, so their latencies overlap.
    // PAIRS: positions come in adjacent pairs (pos(2m + 1) = pos(2m) + 1 with
    // pos(2m) even), moved as 16-byte accesses.
    // padd / has_p: a further addend (the permuted one of PERM), uniform per workgroup.
    [[maybe_unused]] auto epi_store = [&](auto pos, auto val, auto pairs, auto padd, bool has_p) {
        constexpr bool PAIRS = decltype(pairs)::value;
        constexpr int CH = E < 8 ? E : 8;
        auto ld = [&](const uint64_t* __restrict__ p, const uint32_t (&jj)[CH], uint64_t (&v)[CH]) {
            if constexpr (PAIRS) {
#pragma unroll
                for (int k = 0; k < CH; k += 2) {
                    const ulonglong2 t = *reinterpret_cast<const ulonglong2*>(p + jj[k]);
                    v[k] = t.x;
                    v[k + 1] = t.y;
                }
            } else {
#pragma unroll
                for (int k = 0; k < CH; ++k) v[k] = p[jj[k]];
            }
        };
#pragma unroll
        for (int k0 = 0; k0 < E; k0 += CH) {
            uint32_t jj[CH];
            uint64_t a[CH], u[CH], w[CH], r[CH], pv[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) jj[k] = pos(k0 + k);
            ld(acc_src, jj, a);
            if (add_src) ld(add_src, jj, u);
            if (add2_src) ld(add2_src, jj, w);
            if (has_p) {
#pragma unroll
                for (int k = 0; k < CH; ++k) pv[k] = padd(k0 + k);
            }
            if (fp) {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
#pragma clang fp contract(off)
                    // (acc - conv) P^-1 with |acc - conv| < 5.5q: within 2q; the
                    // addends (< q each) keep it within 5q before the final reduction
                    double y = fmulmod(as_f(fp_from_u64(a[k])) - as_f(val(k0 + k)), as_f(pinv.w), as_f(pinv.wp), qd);
                    if (add_src) y += as_f(fp_from_u64(u[k]));
                    if (add2_src) y += as_f(fp_from_u64(w[k]));
                    if (has_p) y += as_f(fp_from_u64(pv[k]));
                    r[k] = fp_to_u64(as_u(y), qd, qinv);
                }
            } else {
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    uint64_t v = shoup(a[k] + q - finish(val(k0 + k)), pinv.w, pinv.wp, q);
                    if (add_src) v = add_mod(v, u[k], q);
                    if (add2_src) v = add_mod(v, w[k], q);
                    if (has_p) v = add_mod(v, pv[k], q);
                    r[k] = v;
                }
            }
            if constexpr (PAIRS) {
#pragma unroll
                for (int k = 0; k < CH; k += 2) {
                    ulonglong2 t;
                    t.x = r[k];
                    t.y = r[k + 1];
                    *reinterpret_cast<ulonglong2*>(out_row + jj[k]) = t;
                }
            } else {
#pragma unroll
                for (int k = 0; k < CH; ++k) out_row[jj[k]] = r[k];
            }
        }
    };
    if constexpr (DIRECT_OUT && VEC_OUT && !EPI) {
        ulonglong2* __restrict__ dst = reinterpret_cast<ulonglong2*>(data + gidx(c, (uint32_t)E * l));
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            ulonglong2 v;
            v.x = finish(x[2 * e]);
            v.y = finish(x[2 * e + 1]);
            dst[e] = v;
        }
    } else if constexpr (DIRECT_OUT) {
        if constexpr (EPI)
            epi_store([&](int e) { return (uint32_t)gidx(c, POUT::r_of(l, e)); }, [&](int e) { return x[e]; },
                      std::false_type{}, [](int) { return 0ull; }, false);
        else
#pragma unroll
            for (int e = 0; e < E; ++e) data[gidx(c, POUT::r_of(l, e))] = finish(x[e]);
    } else {
        lds_write<LOG_M, PH_OUT, EB>(x, lds, c, l);
        __syncthreads();
        auto at = [&](int k) {
            const uint32_t idx = tid + NT * k;
            return std::pair<uint32_t, uint32_t>(idx / M, idx % M);
        };
        if constexpr (EPI) {
            // element pairs 2 (tid + NT m) and its successor: adjacent in the
            // row (a row pass has no index bits below its window)
            auto at2 = [&](int k) {
                const uint32_t idx = 2u * (tid + NT * (uint32_t)(k >> 1)) + (uint32_t)(k & 1);
                return std::pair<uint32_t, uint32_t>(idx / M, idx % M);
            };
            if constexpr (!COL && PERM) {
                // the transform's values leave the LDS first, then the
                // permuted addend (first polynomial of an item) is staged there
                uint64_t v[E];
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const auto p = at2(k);
                    v[k] = lds[lds_at<LOG_M, EB>(p.first, p.second)];
                }
                const bool has_p = bsel == 0 && ep.kappa != 0;
                if (has_p) {
                    __syncthreads();
                    galois_tile_to_lds<LOG_M, EB>(ep.perm_src[poly >> 1] + ((size_t)row << log_n), blockIdx.x, log_n,
                                                  ep.kappa, ep.kappa_inv, lds, false);
                }
                epi_store([&](int k) { const auto p = at2(k); return (uint32_t)gidx(p.first, p.second); },
                          [&](int k) { return v[k]; }, std::true_type{},
                          [&](int k) { const auto p = at2(k); return lds[lds_at<LOG_M, EB>(p.first, p.second)]; },
                          has_p);
            } else if constexpr (!COL) {
                epi_store([&](int k) { const auto p = at2(k); return (uint32_t)gidx(p.first, p.second); },
                          [&](int k) { const auto p = at2(k); return lds[lds_at<LOG_M, EB>(p.first, p.second)]; },
                          std::true_type{}, [](int) { return 0ull; }, false);
            } else {
                epi_store([&](int k) { const auto p = at(k); return (uint32_t)gidx(p.first, p.second); },
                          [&](int k) { const auto p = at(k); return lds[lds_at<LOG_M, EB>(p.first, p.second)]; },
                          std::false_type{}, [](int) { return 0ull; }, false);
            }
        } else if constexpr (!COL) {
            // adjacent element pairs of the row as 16-byte stores
#pragma unroll
            for (int m = 0; m < E / 2; ++m) {
                const uint32_t idx = 2u * (tid + NT * (uint32_t)m);
                const uint32_t cc = idx / M, r = idx % M;
                ulonglong2 v;
                v.x = finish(lds[lds_at<LOG_M, EB>(cc, r)]);
                v.y = finish(lds[lds_at<LOG_M, EB>(cc, r + 1)]);
                *reinterpret_cast<ulonglong2*>(data + gidx(cc, r)) = v;
            }
        } else {
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const auto p = at(k);
                data[gidx(p.first, p.second)] = finish(lds[lds_at<LOG_M, EB>(p.first, p.second)]);
            }
        }
    }
}

template <int LOG_M, int EB, bool INV, bool COL, bool FINAL>
void launch_k(const PolyBatch& b, const DevTables& t, uint32_t log_n, uint32_t s0, uint32_t first_pass, bool stage,
              const NttEpilogue* epi, hipStream_t st) {
    const dim3 grid((1u << log_n) / 4096u, b.n_polys * b.n_limbs);
    const TwPair* tw = INV ? t.tw_inv : t.tw_fwd;
    const NttEpilogue ep = epi ? *epi : NttEpilogue{};
    if constexpr (!INV && !COL && FINAL) {
        // the epilogue reads acc and the addend and writes out beside the
        // transformed value: always through the coalesced staged store
        if (epi) {
            if (epi->kappa)
                hipLaunchKernelGGL((k_ntt_pass<LOG_M, EB, INV, COL, FINAL, true, true, true>), grid, dim3(4096 >> EB),
                                   0, st, b, t.mods, tw, log_n, s0, first_pass, ep);
            else
                hipLaunchKernelGGL((k_ntt_pass<LOG_M, EB, INV, COL, FINAL, true, true>), grid, dim3(4096 >> EB), 0, st,
                                   b, t.mods, tw, log_n, s0, first_pass, ep);
            return;
        }
    }
    if constexpr (INV && !COL) {
        // the first pass of an inverse transform reading its input through
        // X -> X^kappa (staged through LDS on its input side)
        if (epi && epi->kappa && first_pass) {
            hipLaunchKernelGGL((k_ntt_pass<LOG_M, EB, INV, COL, FINAL, true, false, true>), grid, dim3(4096 >> EB), 0,
                               st, b, t.mods, tw, log_n, s0, first_pass, ep);
            return;
        }
    }
    if (COL || stage)
        hipLaunchKernelGGL((k_ntt_pass<LOG_M, EB, INV, COL, FINAL, true, false>), grid, dim3(4096 >> EB), 0, st, b,
                           t.mods, tw, log_n, s0, first_pass, ep);
    else if constexpr (!COL)
        hipLaunchKernelGGL((k_ntt_pass<LOG_M, EB, INV, COL, FINAL, false, false>), grid, dim3(4096 >> EB), 0, st, b,
                           t.mods, tw, log_n, s0, first_pass, ep);
}

// One pass.  A column pass (low index bits remain below the window) needs at
// least 16 sub-problems per workgroup for coalescing, so radices above 8 only
// run as the last window.  Going forward the last window is the final pass;
// going back the s0 = 0 window is.
template <int LOG_M, bool INV>
void launch_pass(const PolyBatch& b, const DevTables& t, uint32_t log_n, uint32_t s0, bool final_pass, bool stage,
                 bool e8, const NttEpilogue* epi, hipStream_t st, ProfHook* g_prof) {
    const int kid = INV ? PK_NTT_INV : PK_NTT_FWD;
    const uint32_t first_pass = INV ? (s0 + LOG_M == log_n) : (s0 == 0);
    const bool col = s0 + LOG_M < log_n;
    const bool staged = col || stage || (epi && !INV && final_pass);
    if (g_prof) g_prof->begin(kid);
    auto go = [&](auto eb) {
        constexpr int EB = decltype(eb)::value;
        if (col) {
            if constexpr (LOG_M <= 8) launch_k<LOG_M, EB, INV, true, INV>(b, t, log_n, s0, first_pass, true, nullptr, st);
        } else if (final_pass) {
            if constexpr (!INV || LOG_M == 12)
                launch_k<LOG_M, EB, INV, false, true>(b, t, log_n, s0, first_pass, stage, epi, st);
        } else {
            if constexpr (INV) launch_k<LOG_M, EB, INV, false, false>(b, t, log_n, s0, first_pass, stage, epi, st);
        }
    };
    if (e8)
        go(std::integral_constant<int, 3>{});
    else
        go(std::integral_constant<int, 4>{});
    if (g_prof) {
        const double elems = (double)b.n_polys * b.n_limbs * (double)(1u << log_n);
        // method bytes: the transform's input (read by its first pass) and
        // output (written by its final pass), 8 bytes per residue each; the
        // words between two passes are the layout's cost, not the method's.
        // N/2 butterflies per stage.
        const bool fused = epi && !INV && final_pass && !col;
        const bool perm = epi && epi->kappa && !col && (INV ? first_pass != 0 : fused);
        const uint32_t variant = 1u + (LOG_M | (col ? 32u : 0u) | (final_pass ? 64u : 0u) | (staged ? 128u : 0u) |
                                       (e8 ? 256u : 0u) | (fused ? 512u : 0u) | (perm ? 1024u : 0u));
        // the ModDown epilogue reads acc (and the addends) and writes out in
        // place of the transform's own store
        double extra = 0.0;  // addends: half of the rows (one polynomial) each
        if (fused) {
            for (int bb = 0; bb < 2; ++bb)
                extra += (epi->d_add[bb] != PFT_EPI_NO_ADD ? 4.0 : 0.0) + (epi->d_add2[bb] != PFT_EPI_NO_ADD ? 4.0 : 0.0);
            if (perm) extra += 4.0;  // the permuted addend of the first polynomial
        }
        const double in_b = first_pass ? 8.0 : 0.0, out_b = final_pass ? 8.0 : 0.0;
        const double bytes = elems * (in_b + (fused ? 16.0 + extra : out_b));
        g_prof->end(kid, bytes, 0.5 * elems * LOG_M, variant);
    }
}

// A base conversion of hybrid key switching fused with the first pass
// (stages 0-3, a radix-16 column pass) of the forward transform of every row
// it produces.  ModUp (DOWN false): digit j = blockIdx.y of item z =
// blockIdx.z, inputs the digit's rows of d, targets every row outside the
// digit (q-limbs, then special primes), output ext_j.  ModDown (DOWN true):
// polynomial b = blockIdx.y, inputs the K special rows of acc_b, targets the
// q-limbs 0..level-1, output conv_b.  The workgroup converts the 256
// coefficients u0 + u + t N/16 (u, t < 16): the same exact contraction on the
// matrix cores and fold as the stand-alone conversion kernels, for up to 16
// target rows at a time, into LDS; then thread (target, u) takes the 16
// values t of its column through the four stages exactly as the first
// transform pass does (on fp64 rows the fold's reduced double is already the
// butterflies' input form) and stores them in that pass's output form, so the
// transform continues with its second pass.
//
// IFUSE: the input rows come from an inverse transform whose final pass (a
// radix-16 column pass, stages 3-0 with N^-1 folded in) has not run; the
// workgroup applies it to its 16 columns of each input row exactly as that
// pass would (the same butterflies, the same conversion to canonical u64)
// and stages the result in LDS before splitting the digits.
template <uint32_t NKB, bool DOWN, bool IFUSE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_bconv_col_b(
    WsRef ws, uint64_t off_in, uint64_t off_out, uint32_t level, KsConsts kc, const DevMod* __restrict__ mods,
    const TwPair* __restrict__ tw, const TwPair* __restrict__ tw_inv, uint32_t log_n) {
    constexpr uint32_t ROWP = 272;  // LDS words per target row (256 coefficients + padding)
    __shared__ uint64_t ybuf[16 * ROWP];
    __shared__ BconvRed s_red[64];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, half = lane >> 5, wave = tid >> 6;
    const uint32_t S = 1u << (log_n - 4);
    const uint32_t u0 = blockIdx.x * 16u;
    const uint32_t j = blockIdx.y;  // digit (ModUp) or polynomial (ModDown)
    const uint32_t rows = level + kc.K;
    // ModUp: the digit's limbs [i0, i0 + na) are the inputs and are skipped as targets
    const uint32_t i0 = DOWN ? level : j * kc.alpha;
    const uint32_t na = DOWN ? kc.K : min(i0 + kc.alpha, level) - i0;
    const uint32_t T = DOWN ? level : rows - na;
    const size_t cbase = ((size_t)(level - 1) * kc.dnum + j) * kc.alpha;
    uint64_t* item = ws.base + (size_t)blockIdx.z * ws.stride;
    const uint64_t* __restrict__ in = item + off_in + (DOWN ? ((size_t)j * rows << log_n) : 0);
    uint64_t* __restrict__ out = item + off_out + ((size_t)j * (DOWN ? level : rows) << log_n);
    if constexpr (IFUSE) {
        // the final inverse pass of each input row's 16 columns, into LDS
        // rows 0..na-1 at column 16 t + u
        const uint32_t ii = tid >> 4, u = tid & 15u;
        if (ii < na) {
            const uint32_t mi = DOWN ? kc.L + ii : i0 + ii;
            const DevMod md = mods[mi];
            const TwPair* __restrict__ twt = tw_inv + ((size_t)mi << log_n);
            const uint64_t* __restrict__ irow = in + ((size_t)(i0 + ii) << log_n) + u0 + u;
            uint64_t x[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = irow[(size_t)e * S];
            if (md.fp) {
                run_phase<4, 0, 4, true, true, true>(x, 0u, 0u, 0u, twt, md);
#pragma unroll
                for (int e = 0; e < 16; ++e) x[e] = fp_to_u64(x[e], md.qd, md.qinv);
            } else {
                run_phase<4, 0, 4, true, false, true>(x, 0u, 0u, 0u, twt, md);
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) ybuf[ii * ROWP + 16u * e + u] = x[e];
        }
        __syncthreads();
    }
    // input digits of this lane's coefficient in each of the wave's two
    // 32-column blocks: column ci = 32 cb + (lane & 31) = 16 t + u
    uint32_t ci[2];
    long bop[2][NKB];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        ci[h] = 32u * (2u * wave + (uint32_t)h) + (lane & 31u);
        const uint32_t pos = u0 + (ci[h] & 15u) + (ci[h] >> 4) * S;
#pragma unroll
        for (uint32_t kb = 0; kb < NKB; ++kb) {
            const uint32_t ii = 2 * kb + half;
            uint64_t x = 0;
            if (ii < na) {
                const TwPair hv = DOWN ? kc.down_phatinv[ii] : kc.modup_hatinv[cbase + ii];
                const uint64_t qi = mods[DOWN ? kc.L + ii : i0 + ii].q;
                const uint64_t v = IFUSE ? ybuf[ii * ROWP + ci[h]] : in[((size_t)(i0 + ii) << log_n) + pos];
                x = shoup(v, hv.w, hv.wp, qi);
            }
            bop[h][kb] = split_digits(x);
        }
    }
    const uint32_t kbs = DOWN ? kc.down_kb : kc.up_kb;
    const uint64_t* __restrict__ aop =
        (DOWN ? kc.down_aop : kc.up_aop + ((size_t)(level - 1) * kc.dnum + j) * kc.up_rt * kc.up_kb * 64) + lane;
    const uint32_t tiles = (T + 3) / 4;
    // target tt: its row and modulus index
    auto row_of = [&](uint32_t tt) { return DOWN ? tt : (tt < i0 ? tt : tt + na); };
    auto mod_of = [&](uint32_t t) { return t < level ? t : kc.L + (t - level); };
    // the fold constants of every target (T <= L + K <= 64) into LDS in
    // target order, so that a fold finds its own at s_red[tt]; the barrier
    // also orders the LDS input reads above before the first target batch
    // overwrites those rows
    {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(kc.red);
        uint64_t* dst = reinterpret_cast<uint64_t*>(s_red);
        constexpr uint32_t WPR = sizeof(BconvRed) / 8;
        for (uint32_t w = tid; w < T * WPR; w += blockDim.x) dst[w] = src[mod_of(row_of(w / WPR)) * WPR + w % WPR];
        __syncthreads();
    }
    long av[NKB];
#pragma unroll
    for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[kb * 64];
    for (uint32_t tb0 = 0; tb0 < T; tb0 += 16) {
        const uint32_t nt = min(16u, T - tb0);
        for (uint32_t rt = 0; rt * 4 < nt; ++rt) {
            const uint32_t g = tb0 / 4 + rt;  // row tile of the constant operands
            // the two column blocks one after the other (one accumulator tile live)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const v16i zero = {};
                v16i acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[0], bop[h][0], zero, 0, 0, 0);
#pragma unroll
                for (uint32_t kb = 1; kb < NKB; ++kb)
                    acc = __builtin_amdgcn_mfma_i32_32x32x16_i8(av[kb], bop[h][kb], acc, 0, 0, 0);
                if (h == 1 && g + 1 < tiles) {
#pragma unroll
                    for (uint32_t kb = 0; kb < NKB; ++kb) av[kb] = (long)aop[((g + 1) * kbs + kb) * 64];
                }
#pragma unroll
                for (int uu = 0; uu < 2; ++uu) {
                    const uint32_t tt = 4 * g + 2 * half + (uint32_t)uu;
                    if (tt < T) {
                        int z[8];
                        if (uu == 0) tile_digits<0>(acc, z); else tile_digits<1>(acc, z);
                        // fp64 rows keep the fold's double (the pass's input form)
                        ybuf[(tt - tb0) * ROWP + ci[h]] = fold_digits<true>(z, s_red[tt]);
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t tl = tid >> 4, u = tid & 15u;
        if (tl < nt) {
            const uint32_t t = row_of(tb0 + tl);
            const uint32_t mi = mod_of(t);
            const DevMod md = mods[mi];
            const TwPair* __restrict__ twt = tw + ((size_t)mi << log_n);
            uint64_t x[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) x[e] = ybuf[tl * ROWP + 16u * e + u];
            // the fold's values are reduced (within q/2 + 1, or below q)
            if (md.fp) {
                run_phase<4, 0, 4, false, true, false, true>(x, 0u, 0u, 0u, twt, md);
            } else {
                run_phase<4, 0, 4, false, false, false, true>(x, 0u, 0u, 0u, twt, md);
            }
            uint64_t* __restrict__ orow = out + ((size_t)t << log_n) + u0 + u;
#pragma unroll
            for (int e = 0; e < 16; ++e) orow[(size_t)e * S] = x[e];
        }
        __syncthreads();
    }
}

// RESCALE's expansion fused with the first pass (stages 0-3, a radix-16
// column pass) of the forward transform of its rows: thread (row k, column u)
// reads the 16 values t of column u0 + u + t N/16 of last_b (polynomial b's
// limb level-1 in coefficient form), forms ((c + h) mod q_last) - h mod q_k
// (h = (q_last - 1)/2 rounding, 0 floor; q_last < q_k) and takes the column
// through the four stages exactly as the first transform pass does (fp64
// rows converted on entry); row k of tmp_b continues at the second pass.
__global__ __launch_bounds__(256) void k_rescale_col_b(WsRef ws, uint64_t off_last, uint64_t off_tmp, uint32_t level,
                                                       uint32_t mode, const DevMod* __restrict__ mods,
                                                       const TwPair* __restrict__ tw, uint32_t log_n) {
    const uint32_t S = 1u << (log_n - 4);
    const uint32_t u0 = blockIdx.x * 16u;
    const uint32_t nl = level - 1;
    const uint32_t groups = (nl + 15) / 16;
    const uint32_t b = blockIdx.y / groups;
    const uint32_t k = (blockIdx.y - b * groups) * 16u + (threadIdx.x >> 4), u = threadIdx.x & 15u;
    if (k >= nl) return;  // no barrier in this kernel
    const uint64_t ql = mods[level - 1].q;
    const uint64_t h = mode == 0 ? (ql - 1) / 2 : 0;
    uint64_t* item = ws.base + (size_t)blockIdx.z * ws.stride;
    const uint64_t* __restrict__ last = item + off_last + ((size_t)b << log_n) + u0 + u;
    const DevMod md = mods[k];
    uint64_t x[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        uint64_t r = last[(size_t)e * S] + h;
        r = r >= ql ? r - ql : r;
        x[e] = r >= h ? r - h : r + md.q - h;
    }
    const TwPair* __restrict__ twt = tw + ((size_t)k << log_n);
    if (md.fp) {
#pragma unroll
        for (int e = 0; e < 16; ++e) x[e] = fp_from_u64(x[e]);
        run_phase<4, 0, 4, false, true, false, true>(x, 0u, 0u, 0u, twt, md);  // canonical inputs
    } else {
        run_phase<4, 0, 4, false, false, false, true>(x, 0u, 0u, 0u, twt, md);
    }
    uint64_t* __restrict__ orow = item + off_tmp + ((size_t)(b * nl + k) << log_n) + u0 + u;
#pragma unroll
    for (int e = 0; e < 16; ++e) orow[(size_t)e * S] = x[e];
}

// Forward register phase PH applied to G independent tiles at once: each
// twiddle is loaded once and serves the butterflies of every tile.
template <int LOG_M, int PH, int EB, int G, bool FP, int PRE>
__device__ __forceinline__ void run_phase_g(uint64_t (&x)[G][1 << EB],
                                            const PhaseTw<LOG_M, PH, EB, false, false, PRE>& tw, const DevMod& md) {
    using Ph = Phase<LOG_M, PH, EB>;
    constexpr int E = 1 << EB;
    const uint64_t q = md.q, two_q = md.two_q;
    const double qd = md.qd, qinv = md.qinv;
#pragma unroll
    for (int bit = Ph::HB; bit >= Ph::LB; --bit) {
        const int spp = LOG_M - 1 - bit;
        const int pos = bit - Ph::WLO;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e & (1 << pos)) continue;
            const TwPair tp = tw.get(pos, e);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if constexpr (FP)
                    fwd_bfly_fp(x[g][e], x[g][e | (1 << pos)], tp, qd, qinv, spp % 3 == 0);
                else if (!int_fwd_reduces(LOG_M, spp))
                    fwd_bfly_low(x[g][e], x[g][e | (1 << pos)], tp.w, tp.wp, q, two_q);
                else
                    fwd_bfly_r8(x[g][e], x[g][e | (1 << pos)], tp.w, tp.wp, q, two_q);
            }
        }
    }
}
// The forward register phases of one pass for G tiles, each exchanging
// through its own LDS region (one barrier per exchange for all of them).
template <int LOG_M, int EB, int G, bool FP, int K, int PRE>
__device__ __forceinline__ void run_phases_g(uint64_t (&x)[G][1 << EB], uint64_t* lds, uint32_t c, uint32_t l,
                                             uint32_t high, uint32_t s0, const TwPair* __restrict__ twt,
                                             const DevMod& md) {
    constexpr int NPH = (LOG_M + EB - 1) / EB;
    constexpr uint32_t W = lds_words<LOG_M, EB>();
    if constexpr (K < NPH) {
        // the phase's twiddle loads go out before the exchange
        const PhaseTw<LOG_M, K, EB, false, false, PRE> tw(twt, l, high, s0);
        if constexpr (K > 0) {
#pragma unroll
            for (int g = 0; g < G; ++g) lds_write<LOG_M, K - 1, EB>(x[g], lds + g * W, c, l);
            if constexpr (wave_local_exchange<LOG_M, EB, false>(K - 1, K))
                wave_lds_sync();
            else
                __syncthreads();
#pragma unroll
            for (int g = 0; g < G; ++g) lds_read<LOG_M, K, EB>(x[g], lds + g * W, c, l);
        }
        run_phase_g<LOG_M, K, EB, G, FP, PRE>(x, tw, md);
        run_phases_g<LOG_M, EB, G, FP, K + 1, PRE>(x, lds, c, l, high, s0, twt, md);
    }
}

// The key inner product of hybrid key switching fused with the last pass of
// the forward transform of ModUp's rows.  Where the conversion kernel has
// already applied the first pass (a radix-16 column pass), each extended row
// needs one row pass of LOG_M = log_n - 4 stages over 4096-word tiles.  A
// workgroup takes one tile of row t of one item and every digit j: x_j is d
// itself where t is one of digit j's own rows (d is in the NTT domain
// already) or ext_j[t] taken through the row pass in registers; the product
// with the key tile is accumulated, and only the two accumulator tiles
// acc_b[t] = sum_j x_j key_{j,b}[t] (b = 0, 1) are written.  The extended
// digits are read once instead of being written back by the row pass and
// read again by a separate inner-product kernel.  The products are taken in
// the arrangement the pass ends in (each thread holds E consecutive words of
// its sub-problem), so d, the key and the accumulators move as 16-byte
// accesses per lane and no LDS staging is needed.
//
// G digits go through the row pass together (G = 2: each twiddle load and
// each LDS barrier serves two tiles, and the two tiles' butterflies are
// independent instruction streams); a leftover digit takes the pass alone.
//
// Block order: blocks are issued to the eight XCDs round-robin; block id
// 8 k + x runs item k mod n of the (row, tile) pair 8 floor(k / n) + x, so
// the items sharing one key tile run on one XCD at about the same time and
// the tile comes from HBM about once per launch, then from that XCD's L2.
//
// FP (rows with q < 2^50, the key holding integer-valued doubles): x is
// brought within q/2, each product formed by fmulmod against the quotient
// w (1/q) (|term| < 0.9q, so the sum over at most 8 digits stays below
// 2^53), the sums converted to canonical residues.  Otherwise x is brought
// below q and the Montgomery products with the key (stored times 2^64) are
// summed without REDC's final subtraction (terms below 2q, at most 8 of
// them: below 16q < 2^64), the sums reduced below q once at the end.  The
// rows of one kind form one launch (ri.row).
template <int LOG_M, int EB, bool FP, int G>
__global__ __launch_bounds__(4096 >> EB) __attribute__((amdgpu_waves_per_eu(4)))
void k_row_inner(RowInner ri, const DevMod* __restrict__ mods, const TwPair* __restrict__ tw, uint32_t log_n) {
    constexpr int M = 1 << LOG_M;
    constexpr int E = 1 << EB;
    constexpr uint32_t NT = 4096 >> EB;
    constexpr int T = M / E;
    constexpr int C = NT / T;
    constexpr int NPH = (LOG_M + EB - 1) / EB;
    using PIN = Phase<LOG_M, 0, EB>;
    using POUT = Phase<LOG_M, NPH - 1, EB>;
    static_assert(PIN::WLO >= 4, "the row pass reads its input directly");
    static_assert(POUT::WLO == 0, "each thread ends with E consecutive words");
    static_assert(G == 1 || G == 2, "one or two tiles per row pass");
    __shared__ uint64_t lds[G * lds_words<LOG_M, EB>()];

    const uint32_t bid = blockIdx.x;
    const uint32_t kx = bid >> 3;
    const uint32_t z = kx % ri.n_items;
    const uint32_t pair = (kx / ri.n_items) * 8u + (bid & 7u);
    if (pair >= ri.tiles * ri.n_rows) return;  // whole workgroup, before any barrier
    const uint32_t tile = pair % ri.tiles;
    const uint32_t t = ri.row[pair / ri.tiles];

    const uint32_t tid = threadIdx.x;
    const uint32_t mi = t < ri.level ? t : ri.L + (t - ri.level);
    const DevMod md = mods[mi];
    const uint64_t q = md.q, two_q = md.two_q;
    const double qd = md.qd, qinv = md.qinv;
    const TwPair* __restrict__ twt = tw + ((size_t)mi << log_n);
    const uint32_t s0 = log_n - LOG_M;
    const uint32_t sp0 = tile * (uint32_t)C;
    const uint32_t c = C == 1 ? 0u : tid / T;
    const uint32_t l = C == 1 ? tid : tid % T;
    uint64_t* __restrict__ item = ri.base + (size_t)z * ri.stride;
    // this thread's E consecutive words of the row: [w0, w0 + E)
    const size_t w0 = ((size_t)(sp0 + c) << LOG_M) + (size_t)l * E;

    auto load_vec = [&](const uint64_t* __restrict__ p, uint64_t (&v)[E]) {
        const ulonglong2* __restrict__ pv = reinterpret_cast<const ulonglong2*>(p + w0);
#pragma unroll
        for (int e = 0; e < E / 2; ++e) {
            const ulonglong2 u = pv[e];
            v[2 * e] = u.x;
            v[2 * e + 1] = u.y;
        }
    };
    uint64_t acc0[E], acc1[E];  // FP: doubles; otherwise residues below q
#pragma unroll
    for (int e = 0; e < E; ++e) acc0[e] = acc1[e] = 0;  // also the bits of +0.0
    // the key tile key_{j,b}[t] of this thread's words
    auto load_key = [&](uint32_t j, int b, uint64_t (&k)[E]) {
        load_vec(ri.key + ((size_t)((2 * j + b) * ri.krows + mi) << log_n), k);
    };
    // acc_b += x k
    auto mac = [&](const uint64_t (&x)[E], const uint64_t (&k)[E], uint64_t (&acc)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (FP) {
#pragma clang fp contract(off)
                const double a = as_f(k[e]);
                acc[e] = as_u(as_f(acc[e]) + fmulmod(as_f(x[e]), a, a * qinv, qd));
            } else {
                // REDC without its final subtraction: each term lies in [0, 2q)
                const uint64_t lo = x[e] * k[e], m = lo * md.mont_neg_qinv;
                acc[e] += mulhi64(x[e], k[e]) + mulhi64(m, q) + (lo != 0 ? 1u : 0u);
            }
        }
    };
    auto accumulate = [&](const uint64_t (&x)[E], uint32_t j) {
        uint64_t k0[E], k1[E];
        load_key(j, 0, k0);
        load_key(j, 1, k1);
        mac(x, k0, acc0);
        mac(x, k1, acc1);
    };
    // ext_j[t] (after the conversion kernel's column pass) into x
    auto load_ext = [&](uint32_t j, uint64_t (&x)[E]) {
        const uint64_t* __restrict__ src = item + ri.off_ext + ((size_t)(j * ri.rows + t) << log_n);
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = src[((size_t)(sp0 + c) << LOG_M) | PIN::r_of(l, e)];
    };
    // an integer accumulator (at most 8 terms below 2q each: below 16q <
    // 2^64) brought below q
    [[maybe_unused]] auto settle_acc = [&](uint64_t v) -> uint64_t {
#pragma unroll
        for (int sh = 3; sh >= 0; --sh) {
            const uint64_t m = q << sh;
            v = v >= m ? v - m : v;
        }
        return v;
    };
    // the row pass's output brought within q/2 (FP) or below q
    auto settle = [&](uint64_t (&x)[E]) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if constexpr (FP) {
                x[e] = as_u(freduce(as_f(x[e]), qd, qinv));
            } else {
                const uint64_t v = x[e] >= two_q ? x[e] - two_q : x[e];
                x[e] = v >= q ? v - q : v;
            }
        }
    };
    // the twiddles and their addresses are the same for every digit; an
    // opaque zero offset of their base and opaque copies of the lane indices
    // keep the compiler from holding all of them in registers across the
    // digit loop (they are recomputed and reloaded per digit).  The offset,
    // not the pointer, is hidden, so the loads stay global (not flat) loads.
    // (Issuing the key loads ahead of the pass, to hide their latency behind
    // it, was measured slower: the extra live registers spill or crowd the
    // pass at four waves per SIMD.)
    auto row_pass_1 = [&](uint32_t j) {
        uint64_t x[E];
        load_ext(j, x);
        uint32_t zoff = 0, lj = l, cj = c;
        asm volatile("" : "+v"(zoff), "+v"(lj), "+v"(cj));
        const TwPair* __restrict__ twj = twt + zoff;
        run_phases<LOG_M, EB, false, FP, false, 0, false, tw_pre_inner(FP, G)>(x, lds, cj, lj, sp0 + c, s0, twj, md);
        __syncthreads();  // the next digit's exchanges reuse the LDS
        settle(x);
        accumulate(x, j);
    };
    [[maybe_unused]] auto row_pass_2 = [&](uint32_t j1, uint32_t j2) {
        uint64_t x[2][E];
        load_ext(j1, x[0]);
        load_ext(j2, x[1]);
        uint32_t zoff = 0, lj = l, cj = c;
        asm volatile("" : "+v"(zoff), "+v"(lj), "+v"(cj));
        const TwPair* __restrict__ twj = twt + zoff;
        run_phases_g<LOG_M, EB, 2, FP, 0, tw_pre_inner(FP, 2)>(x, lds, cj, lj, sp0 + c, s0, twj, md);
        __syncthreads();  // the next digits' exchanges reuse the LDS
        settle(x[0]);
        accumulate(x[0], j1);
        settle(x[1]);
        accumulate(x[1], j2);
    };

    // the digit whose own rows include t: d itself (no transform needed)
    if (t < ri.level) {
        const uint32_t jo = t / ri.alpha;
        uint64_t x[E];
        if (ri.kappa) {
            // d = X^kappa image of the input's row t: its tile staged in LDS
            galois_tile_to_lds<LOG_M, EB>(ri.perm_src[z] + ((size_t)t << log_n), tile, log_n, ri.kappa, ri.kappa_inv,
                                          lds, FP);
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = lds[lds_at<LOG_M, EB>(c, l * (uint32_t)E + (uint32_t)e)];
            __syncthreads();  // the digits' exchanges reuse the LDS
        } else {
            load_vec(item + ri.off_d + ((size_t)t << log_n), x);
            if constexpr (FP) {
#pragma unroll
                for (int e = 0; e < E; ++e) x[e] = fp_from_u64(x[e]);
            }
        }
        accumulate(x, jo);
    }
    // every other digit through the row pass, G at a time (uniform control
    // flow: t, level, alpha and beta are the same for the whole workgroup)
    uint32_t pend = ~0u;
    for (uint32_t j = 0; j < ri.beta; ++j) {
        if (t < ri.level && j == t / ri.alpha) continue;
        if constexpr (G == 1) {
            row_pass_1(j);
        } else {
            if (pend == ~0u) {
                pend = j;
                continue;
            }
            row_pass_2(pend, j);
            pend = ~0u;
        }
    }
    if (pend != ~0u) row_pass_1(pend);

    ulonglong2* __restrict__ o0 = reinterpret_cast<ulonglong2*>(item + ri.off_acc + ((size_t)t << log_n) + w0);
    ulonglong2* __restrict__ o1 =
        reinterpret_cast<ulonglong2*>(item + ri.off_acc + ((size_t)(ri.rows + t) << log_n) + w0);
#pragma unroll
    for (int e = 0; e < E / 2; ++e) {
        ulonglong2 u, v;
        if constexpr (FP) {
            u.x = fp_to_u64(acc0[2 * e], qd, qinv);
            u.y = fp_to_u64(acc0[2 * e + 1], qd, qinv);
            v.x = fp_to_u64(acc1[2 * e], qd, qinv);
            v.y = fp_to_u64(acc1[2 * e + 1], qd, qinv);
        } else {
            u.x = settle_acc(acc0[2 * e]);
            u.y = settle_acc(acc0[2 * e + 1]);
            v.x = settle_acc(acc1[2 * e]);
            v.y = settle_acc(acc1[2 * e + 1]);
        }
        o0[e] = u;
        o1[e] = v;
    }
}

template <bool INV>
void launch_radix(uint32_t radix, const PolyBatch& b, const DevTables& t, uint32_t log_n, uint32_t s0, bool fin,
                  bool stage, bool e8, const NttEpilogue* epi, hipStream_t st, ProfHook* prof) {
    switch (radix) {
        case 4: launch_pass<4, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 6: launch_pass<6, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 7: launch_pass<7, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 8: launch_pass<8, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 9: launch_pass<9, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 10: launch_pass<10, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 11: launch_pass<11, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        case 12: launch_pass<12, INV>(b, t, log_n, s0, fin, stage, e8, epi, st, prof); break;
        default: break;
    }
}

}  // namespace

bool ntt_supported(uint32_t log_n) { return log_n >= 12 && log_n <= 16; }

// Candidate schedules per log2 N, the default first: every radix split
// below, each with the row pass staged through LDS and direct, and each with
// 16 and with 8 residues per thread.  Windows are
// listed in forward order (stages 0.. first); every candidate has at most two
// passes, so each moves every residue through HBM at most twice.
int ntt_candidates(uint32_t log_n, NttSchedule* out, int max_out) {
    static const uint8_t c12[][2] = {{12, 0}, {8, 4}, {6, 6}, {4, 8}};
    static const uint8_t c13[][2] = {{7, 6}, {6, 7}, {4, 9}};
    static const uint8_t c14[][2] = {{7, 7}, {8, 6}, {6, 8}, {4, 10}};
    static const uint8_t c15[][2] = {{8, 7}, {7, 8}, {6, 9}, {4, 11}};
    static const uint8_t c16[][2] = {{8, 8}, {7, 9}, {6, 10}, {4, 12}};
    const uint8_t(*c)[2] = nullptr;
    int n = 0;
    switch (log_n) {
        case 12: c = c12; n = 4; break;
        case 13: c = c13; n = 3; break;
        case 14: c = c14; n = 4; break;
        case 15: c = c15; n = 4; break;
        case 16: c = c16; n = 4; break;
        default: return 0;
    }
    int k = 0;
    for (int e8 = 0; e8 < 2; ++e8)
        for (int direct = 0; direct < 2; ++direct)
            for (int i = 0; i < n; ++i) {
                if (k >= max_out) return k;
                NttSchedule s{};
                s.n_passes = c[i][1] ? 2 : 1;
                s.radix[0] = c[i][0];
                s.radix[1] = c[i][1];
                s.flags = (direct ? NTT_DIRECT_ROWS : 0u) | (e8 ? NTT_E8 : 0u);
                out[k++] = s;
            }
    return k;
}

bool ntt_schedule_valid(uint32_t log_n, const NttSchedule& s) {
    NttSchedule c[32];
    const int n = ntt_candidates(log_n, c, 32);
    for (int i = 0; i < n; ++i)
        if (c[i].n_passes == s.n_passes && c[i].radix[0] == s.radix[0] && c[i].radix[1] == s.radix[1] &&
            c[i].flags == s.flags)
            return true;
    return false;
}

template <bool DOWN, bool IFUSE>
static void launch_bconv_col(uint32_t nkb, dim3 grid, hipStream_t st, WsRef ws, uint64_t off_in, uint64_t off_out,
                             uint32_t level, const KsConsts& kc, const DevTables& t, uint32_t log_n) {
#define PFT_BCONV_COL(K)                                                                                     \
    case K:                                                                                                  \
        hipLaunchKernelGGL((k_bconv_col_b<K, DOWN, IFUSE>), grid, dim3(256), 0, st, ws, off_in, off_out, level, \
                           kc, t.mods, t.tw_fwd, t.tw_inv, log_n);                                           \
        break;
    switch (nkb) {
        PFT_BCONV_COL(1)
        PFT_BCONV_COL(2)
        PFT_BCONV_COL(3)
        PFT_BCONV_COL(4)
        PFT_BCONV_COL(5)
        PFT_BCONV_COL(6)
        default: break;
    }
#undef PFT_BCONV_COL
}

void launch_modup_col_b(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint32_t level, const KsConsts& kc,
                        const DevTables& t, uint32_t log_n, bool ifuse, hipStream_t st) {
    const uint32_t beta = (level + kc.alpha - 1) / kc.alpha;
    const uint32_t nkb = (std::min(kc.alpha, level) + 1) / 2;
    const dim3 grid((1u << log_n) / 256, beta, n);
    if (ifuse)
        launch_bconv_col<false, true>(nkb, grid, st, ws, off_d, off_ext, level, kc, t, log_n);
    else
        launch_bconv_col<false, false>(nkb, grid, st, ws, off_d, off_ext, level, kc, t, log_n);
}

void launch_moddown_col_b(uint32_t n, WsRef ws, uint64_t off_acc, uint64_t off_conv, uint32_t level,
                          const KsConsts& kc, const DevTables& t, uint32_t log_n, bool ifuse, hipStream_t st) {
    const dim3 grid((1u << log_n) / 256, 2, n);
    if (ifuse)
        launch_bconv_col<true, true>((kc.K + 1) / 2, grid, st, ws, off_acc, off_conv, level, kc, t, log_n);
    else
        launch_bconv_col<true, false>((kc.K + 1) / 2, grid, st, ws, off_acc, off_conv, level, kc, t, log_n);
}

void launch_rescale_col_b(uint32_t n, WsRef ws, uint64_t off_last, uint64_t off_tmp, uint32_t level, uint32_t mode,
                          const DevTables& t, uint32_t log_n, hipStream_t st) {
    const uint32_t groups = (level - 1 + 15) / 16;
    hipLaunchKernelGGL(k_rescale_col_b, dim3((1u << log_n) / 256, 2 * groups, n), dim3(256), 0, st, ws, off_last,
                       off_tmp, level, mode, t.mods, t.tw_fwd, log_n);
}

bool row_inner_supported(uint32_t log_n) {
    const uint32_t r = log_n - 4;
    return r >= 8 && r <= 12;
}

void launch_row_inner(uint32_t n, WsRef ws, uint64_t off_d, uint64_t off_ext, uint64_t off_acc, const uint64_t* key,
                      uint32_t level, const KsConsts& kc, const DevTables& t, const uint32_t* fp_rows,
                      uint32_t log_n, const uint64_t* const* perm_src, uint64_t kappa, uint64_t kappa_inv,
                      bool pair_digits, hipStream_t st, ProfHook* prof, uint32_t rows_sel) {
    RowInner ri{};
    if (kappa) {
        for (uint32_t z = 0; z < n; ++z) ri.perm_src[z] = perm_src[z];
        ri.kappa = kappa;
        ri.kappa_inv = kappa_inv;
    }
    ri.base = ws.base;
    ri.stride = ws.stride;
    ri.off_d = off_d;
    ri.off_ext = off_ext;
    ri.off_acc = off_acc;
    ri.key = key;
    ri.n_items = n;
    ri.level = level;
    ri.rows = level + kc.K;
    ri.alpha = kc.alpha;
    ri.beta = (level + kc.alpha - 1) / kc.alpha;
    // the integer accumulators hold at most 8 terms below 2q (callers check)
    if (ri.beta > 8) {
        fprintf(stderr, "launch_row_inner: %u digits, at most 8 supported\n", ri.beta);
        abort();
    }
    ri.L = kc.L;
    ri.krows = kc.L + kc.K;
    ri.tiles = (1u << log_n) >> 12;
    for (int fp = 1; fp >= 0; --fp) {
        if (!(rows_sel & (fp ? ROW_INNER_FP : ROW_INNER_INT))) continue;
        // the rows of one arithmetic kind, in chunks that fit the row list
        std::vector<uint16_t> rows;
        for (uint32_t r = 0; r < ri.rows; ++r) {
            const uint32_t mi = r < level ? r : kc.L + (r - level);
            if ((int)fp_rows[mi] == fp) rows.push_back((uint16_t)r);
        }
        for (size_t r0 = 0; r0 < rows.size(); r0 += PFT_ROW_LIST) {
            ri.n_rows = (uint32_t)std::min<size_t>(PFT_ROW_LIST, rows.size() - r0);
            for (uint32_t i = 0; i < ri.n_rows; ++i) ri.row[i] = rows[r0 + i];
            const uint32_t pairs = ri.tiles * ri.n_rows;
            const dim3 grid(8u * n * ((pairs + 7u) / 8u));
            // method bytes: d's own rows and both accumulators per item, the
            // key rows once (the extended rows are the pass boundary); work:
            // the row pass's butterflies and two products per digit input
            double bytes = 0.0, ops = 0.0;
            const double N = (double)(1u << log_n), lm = (double)(log_n - 4);
            for (uint32_t i = 0; i < ri.n_rows; ++i) {
                const double own = ri.row[i] < level ? 1.0 : 0.0;
                bytes += 8.0 * N * (n * (own + 2.0) + 2.0 * ri.beta);
                ops += N * n * (0.5 * lm * (ri.beta - own) + 2.0 * ri.beta);
            }
            const bool g2 = fp && pair_digits;
            if (prof) prof->begin(PK_KEY_INNER, st);
            auto go = [&](auto lm, auto eb) {
                constexpr int LM = decltype(lm)::value, EB = decltype(eb)::value;
                if (g2)
                    hipLaunchKernelGGL((k_row_inner<LM, EB, true, 2>), grid, dim3(4096 >> EB), 0, st, ri, t.mods,
                                       t.tw_fwd, log_n);
                else if (fp)
                    hipLaunchKernelGGL((k_row_inner<LM, EB, true, 1>), grid, dim3(4096 >> EB), 0, st, ri, t.mods,
                                       t.tw_fwd, log_n);
                else
                    hipLaunchKernelGGL((k_row_inner<LM, EB, false, 1>), grid, dim3(4096 >> EB), 0, st, ri, t.mods,
                                       t.tw_fwd, log_n);
            };
            // 8 residues per thread: with 16 the two accumulators and the
            // pass's registers exceed what four waves per SIMD allow
            auto by_eb = [&](auto lm) { go(lm, std::integral_constant<int, 3>{}); };
            switch (log_n - 4) {
                case 8: by_eb(std::integral_constant<int, 8>{}); break;
                case 9: by_eb(std::integral_constant<int, 9>{}); break;
                case 10: by_eb(std::integral_constant<int, 10>{}); break;
                case 11: by_eb(std::integral_constant<int, 11>{}); break;
                case 12: by_eb(std::integral_constant<int, 12>{}); break;
                default: break;
            }
            // variant: 1024 + radix, + 64 for the fp64 rows, + 128 with two digits per pass
            if (prof)
                prof->end(PK_KEY_INNER, bytes, ops, 1024u + (log_n - 4) + (fp ? 64u : 0u) + (g2 ? 128u : 0u), st);
        }
    }
}

void launch_ntt(const PolyBatch& b, const DevTables& t, uint32_t log_n, bool inverse, const NttSchedule& s,
                hipStream_t st, ProfHook* prof, const NttEpilogue* epi, uint32_t first) {
    if (b.n_polys == 0 || b.n_limbs == 0 || s.n_passes == 0 || s.n_passes > 3) return;
    uint32_t s0[4];
    uint32_t acc = 0;
    for (uint32_t p = 0; p < s.n_passes; ++p) {
        s0[p] = acc;
        acc += s.radix[p];
    }
    if (acc != log_n) return;
    const bool stage = (s.flags & NTT_DIRECT_ROWS) == 0;
    const bool e8 = (s.flags & NTT_E8) != 0;
    if (!inverse) {
        for (uint32_t p = first; p < s.n_passes; ++p)
            launch_radix<false>(s.radix[p], b, t, log_n, s0[p], p + 1 == s.n_passes, stage, e8,
                                p + 1 == s.n_passes ? epi : nullptr, st, prof);
    } else {
        // epi of an inverse transform: X -> X^kappa folded into its first pass
        for (uint32_t p = s.n_passes; p-- > first;)
            launch_radix<true>(s.radix[p], b, t, log_n, s0[p], p == 0, stage, e8,
                               p + 1 == s.n_passes && epi && epi->kappa ? epi : nullptr, st, prof);
    }
}
