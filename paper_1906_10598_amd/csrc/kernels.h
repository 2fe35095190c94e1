// kernels.h -- HIP kernels of the phase-tracking fit (gfx950).
//
// Objective (Eq. 2-2-4 over the model of Eq. 2-2-2): one launch evaluates
// every candidate of every block in the launch against every sample.  The
// grid is a list of work units; a unit is (block, sample tile, candidate
// group).  A workgroup of 256 lanes owns one tile of 256 * S samples: each
// lane holds S consecutive samples in registers (read from HBM once per
// generation and reused for all candidates of the group) and loops over
// the group's candidates.  For each (lane, candidate) an FP64 anchor -- the
// phase in turns and its Taylor coefficients at the lane's first sample,
// with a compensated product for the large linear term -- turns the
// per-sample phase into a 3-FMA local polynomial in the literal offset j.
// Lane partial sums go to LDS; each wave then reduces one candidate's 256
// partials with a fixed-order DPP/shuffle butterfly and writes one FP64
// partial per (candidate, tile).  Units are remapped so that all candidate
// groups of a tile run on the same XCD (consecutive workgroup ids are
// dealt round-robin to the eight XCDs, each with its own L2).
//
// DE (Sec. 1.2, Table 4, DE/rand/1/bin): one workgroup per block sums the
// partials in tile order, applies selection, finds the best member, runs
// the stop rule and draws the next trial population from Philox; every
// decision is taken on the device so a fit needs no host round trip.
#pragma once

#include <type_traits>

#include "device.h"

namespace pt {

// ---------------------------------------------------------------------------
// Accesses to data one workgroup writes and another reads inside one launch
// of the persistent kernel (population rows, partial sums, DE state).
// Variant 0: plain accesses, agent-scope acquire / release fences (L2
// invalidate / write-back).  Variant 1: coherent (agent-scope atomic) loads,
// so readers need no L2 invalidate.  Variant 2 (built): coherent loads and
// stores, so neither side needs cache maintenance; fences only order the
// wave.  All three give bit-identical fits; on the paper-scale block the fit
// takes 70, 52 and 48 ms with them.
// ---------------------------------------------------------------------------
#ifndef PT_SYNC_VARIANT
#define PT_SYNC_VARIANT 2
#endif
#if PT_SYNC_VARIANT >= 1
#define PT_ACQ_SCOPE "workgroup"
#else
#define PT_ACQ_SCOPE "agent"
#endif
#if PT_SYNC_VARIANT >= 2
#define PT_REL_SCOPE "workgroup"
#else
#define PT_REL_SCOPE "agent"
#endif

// Every buffer a kernel reaches through a descriptor is device (global)
// memory; accessing it through global-space pointers gives global_load /
// global_store instead of flat accesses, which also count against the LDS
// counter, so a wait for an LDS or scalar access would wait for them too.
#define PT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const PT_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
    *(PT_GLOBAL T*)p = v;
}

__device__ __forceinline__ double xld(const double* p) {
#if PT_SYNC_VARIANT >= 1
    return __hip_atomic_load((const PT_GLOBAL double*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
    return gld(p);
#endif
}
// Load of a word another launch wrote (COH = false: plain, cacheable; kernel
// boundaries order it) or that another workgroup of this launch may write
// (COH = true: xld).
template <bool COH>
__device__ __forceinline__ double ld(const double* p) {
    if constexpr (COH)
        return xld(p);
    else
        return gld(p);
}

__device__ __forceinline__ void xst(double* p, double v) {
#if PT_SYNC_VARIANT >= 2
    __hip_atomic_store((PT_GLOBAL double*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
    gst(p, v);
#endif
}
__device__ __forceinline__ void xsti(int* p, int v) {
#if PT_SYNC_VARIANT >= 2
    __hip_atomic_store((PT_GLOBAL int*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#else
    gst(p, v);
#endif
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
// Sums over the wave of N values at once, each ending in every lane: pairs,
// quads, eights and rows of 16 lanes by DPP lane moves (quad permutations,
// half-row and row mirrors), then the two halves of each 32 and of the wave
// by the lane-swap instructions; every step adds two values that both lanes
// of a pair hold, so all lanes end with the same bits.  The N chains run side
// by side.  (Register moves with a few cycles of latency, where a shuffle
// through the LDS crossbar costs a round trip per step.)
__device__ __forceinline__ double dpp_move(double v, int ctrl) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int a, b;
    switch (ctrl) {  // (the control is an immediate of the instruction)
    case 0:  // quad_perm [1, 0, 3, 2]: the other lane of the pair
        a = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
        b = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
        break;
    case 1:  // quad_perm [2, 3, 0, 1]: the other pair of the quad
        a = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
        b = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
        break;
    case 2:  // row_half_mirror: the other quad of the eight
        a = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
        b = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
        break;
    default:  // row_mirror: the other eight of the row
        a = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
        b = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
        break;
    }
    return __hiloint2double(b, a);
}
template <bool W32>
__device__ __forceinline__ double swap_add(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    // each lane gets its own value and its partner's (other row of the pair
    // of rows, or other half of the wave), in the same order on both sides
    const auto l = W32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                       : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = W32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                       : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
template <int N>
__device__ __forceinline__ void wave_sums(double (&v)[N]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        double o[N];
#pragma unroll
        for (int r = 0; r < N; ++r) o[r] = dpp_move(v[r], s);
#pragma unroll
        for (int r = 0; r < N; ++r) v[r] += o[r];
    }
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = swap_add<false>(v[r]);
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = swap_add<true>(v[r]);
}

__device__ __forceinline__ int find_block(const BlockDesc* __restrict__ descs, int nblk, int unit) {
    int lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].unit_begin <= unit) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Turn-domain coefficients of one candidate (see device.h).
struct Cand {
    double a0, a1, a2, a3, a4, A, Ad;  // Ad = Adot / fs: amplitude slope per sample
};

// Turn-domain value of population slot j (coefficient x): A; phi0 / 2 pi
// reduced to [-1/2, 1/2]; f0 / fs; f1 / (2 fs^2); f2 / (6 fs^3); Adot / fs;
// f3 / (24 fs^4).  One division serves every slot (slots 0 and 1 divide by
// 1); no contraction, so every caller rounds alike.
__device__ __forceinline__ double cand_value(int j, double x, double fs) {
#pragma clang fp contract(off)
    double den = 1.0;
    if (j == 2 || j == 5) den = fs;
    if (j == 3) den = 2.0 * fs * fs;
    if (j == 4) den = 6.0 * fs * fs * fs;
    if (j == 6) den = 24.0 * fs * fs * fs * fs;
    double q = x / den;
    if (j == 1) {
        const double t = x * 0.15915494309189533577;
        q = t - rint(t);
    }
    return q;
}
// Cand member written by slot j
__device__ __forceinline__ double& cand_member(Cand& c, int j) {
    double* m = &c.a0;  // a0, a1, a2, a3, a4, A, Ad
    constexpr unsigned kIdx = 5u | (0u << 3) | (1u << 6) | (2u << 9) | (3u << 12) | (6u << 15) | (4u << 18);
    return m[(kIdx >> (3 * j)) & 7u];
}

template <bool COH>
__device__ __forceinline__ Cand make_cand(const double* x, double fs) {
    Cand c;
    c.A = cand_value(0, ld<COH>(x + 0), fs);
    c.a0 = cand_value(1, ld<COH>(x + 1), fs);
    c.a1 = cand_value(2, ld<COH>(x + 2), fs);
    c.a2 = cand_value(3, ld<COH>(x + 3), fs);
    c.a3 = cand_value(4, ld<COH>(x + 4), fs);
    c.Ad = cand_value(5, ld<COH>(x + 5), fs);
    c.a4 = cand_value(6, ld<COH>(x + 6), fs);
    return c;
}

// Phase (turns) and its Taylor coefficients at sample offset m0: anchor
// b0 = frac(Phi(m0)) and Phi(m0 + j) = b0 + j (b1 + j (b2 + j (b3 + j b4))).
// The product a1 m0 (up to ~1e5 turns) is split exactly with an FMA so b0
// keeps ~1e-16 turns; m0^2 is exact for |m0| < 2^26.  With a4 = 0 every
// value equals the cubic's (the quartic terms enter as exact zeros).
struct Anchor {
    double b0, b1, b2, b3, b4;
};

__device__ __forceinline__ Anchor make_anchor(const Cand& c, double m0) {
    Anchor a;
    double p = c.a1 * m0;
    const double e = __fma_rn(c.a1, m0, -p);
    p -= rint(p);
    const double mm = m0 * m0;
    double q = __fma_rn(__fma_rn(c.a4, m0, c.a3), m0, c.a2) * mm;
    q -= rint(q);
    double b0 = (c.a0 + p) + (q + e);
    a.b0 = b0 - rint(b0);
    const double t3 = 3.0 * c.a3;
    // b2 = a2 + 3 a3 m0 + 6 a4 m0^2, b1 = a1 + 2 a2 m0 + 3 a3 m0^2 + 4 a4 m0^3, b3 = a3 + 4 a4 m0
    a.b2 = __fma_rn(__fma_rn(6.0 * c.a4, m0, t3), m0, c.a2);
    a.b1 = __fma_rn(__fma_rn(__fma_rn(4.0 * c.a4, m0, t3), m0, 2.0 * c.a2), m0, c.a1);
    a.b3 = __fma_rn(4.0 * c.a4, m0, c.a3);
    a.b4 = c.a4;
    return a;
}

// ---------------------------------------------------------------------------
// FP64 lane accumulation over S samples for one candidate.  The phase is
// stepped with forward differences of the local cubic, Phi(j + 1) =
// Phi(j) + d1(j), d1(j + 1) = d1(j) + d2(j), d2(j + 1) = d2(j) + 6 b3, with
// d1(0) = b1 + b2 + b3 and d2(0) = 2 b2 + 6 b3; each step continues from the
// exactly reduced phase r(j) = Phi(j) - rint(Phi(j)), so the running value
// stays within one turn (rounding ~1e-16 turns per step, S <= 32 steps).
// ---------------------------------------------------------------------------
template <int S, bool TAIL, bool SLOPE, bool COR = false, bool QUART = false>
__device__ __forceinline__ double lane_chi2_f64(const double (&sv)[S], const Anchor& an, double amp0,
                                                double ad, int valid) {
    // Samples are processed in groups of IL: the phase recurrence runs
    // through the group, then the IL cosine polynomials are evaluated in
    // lockstep (IL independent FMA chains hide the FP64 FMA latency) and
    // summed into IL accumulators that are combined at the end.
#ifndef PT_IL64
#define PT_IL64 4
#endif
#ifndef PT_COS64
#define PT_COS64 kCos64
#define PT_COS64_DEG kCosDeg64
#endif
    constexpr int IL = (S >= PT_IL64) ? PT_IL64 : S;
    static_assert(S % IL == 0, "samples per lane must be a multiple of the interleave");
    double acc[IL];
#pragma unroll
    for (int q = 0; q < IL; ++q) acc[q] = 0.0;
    double ph = an.b0;
    // forward differences of the local cubic, or quartic: d1(0) = b1 + b2 + b3
    // (+ b4), d2(0) = 2 b2 + 6 b3 (+ 14 b4), d3(0) = 6 b3 (+ 36 b4), d4 = 24 b4
    double d1 = (an.b1 + an.b2) + an.b3;
    double d2 = __fma_rn(6.0, an.b3, 2.0 * an.b2);
    double d3 = 6.0 * an.b3;
    double d4 = 0.0;
    if constexpr (QUART) {
        d1 += an.b4;
        d2 = __fma_rn(14.0, an.b4, d2);
        d3 = __fma_rn(36.0, an.b4, d3);
        d4 = 24.0 * an.b4;
    }
#pragma unroll
    for (int g = 0; g < S; g += IL) {
        double u[IL], p[IL];
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            const double r = ph - rint(ph);
            if (g + q + 1 < S) {
                ph = r + d1;
                d1 += d2;
                d2 += d3;
                if constexpr (QUART) d3 += d4;
            }
            u[q] = r * r;
            p[q] = PT_COS64[0];
        }
#pragma unroll
        for (int k = 1; k <= PT_COS64_DEG; ++k) {
#pragma unroll
            for (int q = 0; q < IL; ++q) p[q] = __fma_rn(p[q], u[q], PT_COS64[k]);
        }
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            const int j = g + q;
            if constexpr (COR) {
                // masked tail samples are zero, so they add nothing
                const double m = SLOPE ? __fma_rn(ad, (double)j, amp0) * p[q] : p[q];
                acc[q] = __fma_rn(sv[j], m, acc[q]);
            } else {
                const double amp = SLOPE ? __fma_rn(ad, (double)j, amp0) : amp0;
                const double rho = __fma_rn(-amp, p[q], sv[j]);
                if (TAIL) {
                    if (j < valid) acc[q] = __fma_rn(rho, rho, acc[q]);
                } else {
                    acc[q] = (g == 0) ? rho * rho : __fma_rn(rho, rho, acc[q]);
                }
            }
        }
    }
    double tot = 0.0;
#pragma unroll
    for (int q = 0; q < IL; ++q) tot += acc[q];
    return (COR && !SLOPE) ? amp0 * tot : tot;
}

// ---------------------------------------------------------------------------
// FP64 phasor lane accumulation.  A lane's chunk of S samples is expanded
// about its centre: with j = 0..S-1 the sample index in the chunk and
// C = S / 2, the phase is
//   Phi(j) = c0 + c1 (j - C) + c2 (j - C)^2 + (c3 (j - C)^3 + c4 (j - C)^4) turns.
// The host selects this path only where, for every candidate of the box,
//   (1) the dropped terms C^3 |c3| + C^4 |c4| stay below 1e-12 turns,
//   (2) theta = 2 pi |c2| C^2 satisfies theta^2 / 2 <= 1e-11,
//   (3) the local frequency c1 stays at least S * 2.2e-4 / (2 pi) turns away
//       from 0 and 1/2 (|sin 2 pi c1| >= S * 2.2e-4), and
//   (4) across a tile the local frequency moves by at most 6e-3 / (2 pi)
//       turns (the small-angle rotation below).
// Then exp(2 pi i Phi(j)) = u_j g_j with u_j = exp(2 pi i (c0 + c1 (j - C)))
// and g_j = exp(i theta_j), theta_j = 2 pi c2 (j - C)^2:
//   - both parts of u_j follow the real three-term (Chebyshev) recurrence
//     u_{j+1} = 2 cos(2 pi c1) u_j - u_{j-1}, one FMA each; its rounding
//     grows by at most j ulp / |sin 2 pi c1|, held below 1e-12 by (3);
//   - cos(2 pi Phi(j)) = Re(u_j) cos theta_j - Im(u_j) sin theta_j, taken as
//     Re(u_j) - Im(u_j) theta_j, whose error theta^2 / 2 is bounded by (2).
// Five FP64 operations per sample and candidate (two recurrence FMAs, the
// difference s - R, the correction FMA, square-accumulate) instead of a
// reduction and a degree-10 cosine.
//
// Per (lane, candidate) set-up.  The workgroup first forms, once per
// candidate, the phase and its Taylor coefficients B0..B4 at the centre of
// the tile's first chunk (RotConst, FP64 with the linear coefficient kept as
// a double-double B1h + B1l, B1h short enough that B1h n is exact for every
// lane offset n), and exp(2 pi i B1).  A lane at offset n = lane * S then
// needs only polynomial updates in n: its start phase
//   c0 - C c1 = B0 + B1 (n - C) + B2 n^2 + B3 n^3 + B4 n^4 - C delta,
//   delta = c1 - B1 = n (2 B2 + 3 B3 n + 4 B4 n^2),
// one sine / cosine polynomial of that (reduced) phase for u_0, and
// exp(2 pi i c1) = exp(2 pi i B1) exp(2 pi i delta) with a fourth-order
// series of the small angle 2 pi delta.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sincos_turns64(double r, double& c, double& sn) {
    const double u = r * r;
    double pc = kCos64[0], ps = kSin64[0];
#pragma unroll
    for (int k = 1; k <= kCosDeg64; ++k) {
        pc = __fma_rn(pc, u, kCos64[k]);
        ps = __fma_rn(ps, u, kSin64[k]);
    }
    c = pc;
    sn = r * ps;
}

struct RotConst {
    double B0, B1h, B1l, B2, B3, B4;  // turns: phase and Taylor coefficients at the first chunk's centre
    double D2, D3, D4;                // 2 B2, 3 B3, 4 B4 (frequency change with the lane offset)
    double T2, T3, T4;                // 2 pi g (B2, 3 B3, 6 B4) (g theta at a chunk centre)
    double Or, Oi;                    // exp(2 pi i B1)
    double g;                         // amplitude carried by the recurrence: A, or 1 with a slope
};

// Tile constants of one candidate; mt: offset of the tile's first sample
// from the reference sample.
template <int S, bool SLOPE>
__device__ __forceinline__ RotConst make_rot_const(const Cand& c, double mt) {
    constexpr double C = S / 2;
    const double M = mt + C;
    const Anchor a = make_anchor(c, M);
    RotConst k;
    k.B0 = a.b0;
    k.B2 = a.b2;
    k.B3 = a.b3;
    k.B4 = a.b4;
    // B1 = a1 + M (2 a2 + M (3 a3 + 4 a4 M)) as hi + lo (two-sum), then hi
    // split into 40 leading bits (B1h) and the rest (folded into B1l)
    const double sm = __fma_rn(__fma_rn(4.0 * c.a4, M, 3.0 * c.a3), M, 2.0 * c.a2) * M;
    const double hi = c.a1 + sm;
    const double bb = hi - c.a1;
    const double lo = (c.a1 - (hi - bb)) + (sm - bb);
    const double h40 = __longlong_as_double(__double_as_longlong(hi) & ~0x1FFFLL);
    k.B1h = h40;
    k.B1l = (hi - h40) + lo;
    double r = h40 - rint(h40);
    r += k.B1l;
    sincos_turns64(r, k.Or, k.Oi);
    k.D2 = 2.0 * k.B2;
    k.D3 = 3.0 * k.B3;
    k.D4 = 4.0 * k.B4;
    k.g = SLOPE ? 1.0 : c.A;
    const double G = 6.283185307179586477 * k.g;
    k.T2 = G * k.B2;
    k.T3 = G * (3.0 * k.B3);
    k.T4 = G * (6.0 * k.B4);
    return k;
}

// Lane sum of one candidate.  n: the lane's offset from the tile's first
// chunk (lane * S), n2 = n^2, nc = n - C; amp0, ad: amplitude at the chunk's
// first sample and its slope per sample (SLOPE).
template <int S, bool TAIL, bool SLOPE, bool COR>
__device__ __forceinline__ double lane_rot(const double (&sv)[S], const RotConst& k, double n, double n2,
                                           double nc, double amp0, double ad, int valid) {
    constexpr int C = S / 2;
    // start phase of the chunk's linear part and its frequency offset
    const double inner = __fma_rn(__fma_rn(k.D4, n, k.D3), n, k.D2);
    const double delta = n * inner;
    double p = k.B1h * nc;  // exact
    p -= rint(p);
    const double t = __fma_rn(__fma_rn(k.B4, n, k.B3), n, k.B2);
    const double q = __fma_rn(k.B1l, nc, __fma_rn(delta, -(double)C, n2 * t));
    double l0 = (k.B0 + p) + q;
    l0 -= rint(l0);
    double cr, ci;
    sincos_turns64(l0, cr, ci);  // u_0
    // exp(2 pi i c1) = exp(2 pi i B1) exp(i x): |x| <= 6e-3, series error <= x^6 / 720
    const double x = 6.283185307179586477 * delta;
    const double x2 = x * x;
    const double cx = __fma_rn(__fma_rn(x2, 1.0 / 24.0, -0.5), x2, 1.0);
    const double sx = x * __fma_rn(__fma_rn(x2, 1.0 / 120.0, -1.0 / 6.0), x2, 1.0);
    const double wr = __fma_rn(k.Or, cx, -(k.Oi * sx));
    const double wi = __fma_rn(k.Or, sx, k.Oi * cx);
    const double c2 = wr + wr;
    // u_{-1} = u_0 exp(-2 pi i c1) starts the recurrence; it carries R = g Re(u)
    // and W = g theta Im(u), so that g cos(2 pi Phi(j)) = R_j - W_j (j - C)^2 and
    // the residual is (s - R_j) + W_j (j - C)^2
    const double pr = __fma_rn(cr, wr, ci * wi);
    const double pi = __fma_rn(ci, wr, -(cr * wi));
    const double gth = __fma_rn(__fma_rn(k.T4, n, k.T3), n, k.T2);
    double r = k.g * cr, rp = k.g * pr, w = gth * ci, wp = gth * pi;
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) {
        if (j > 0) {
            const double nr = __fma_rn(c2, r, -rp);
            const double nw = __fma_rn(c2, w, -wp);
            rp = r;
            wp = w;
            r = nr;
            w = nw;
        }
        // (j - C)^2 is an immediate, so no per-sample constant is held in registers
        const double k2 = (double)((j - C) * (j - C));
        double& acc = (j & 1) ? acc1 : acc0;
        if constexpr (COR) {
            const double zr = j == C ? r : __fma_rn(-w, k2, r);
            const double m = SLOPE ? __fma_rn(ad, (double)j, amp0) * zr : zr;
            acc = __fma_rn(sv[j], m, acc);
        } else {
            double rho;
            if constexpr (SLOPE) {
                const double zr = j == C ? r : __fma_rn(-w, k2, r);
                rho = __fma_rn(-__fma_rn(ad, (double)j, amp0), zr, sv[j]);
            } else {
                const double d = sv[j] - r;
                rho = j == C ? d : __fma_rn(w, k2, d);
            }
            if (TAIL) {
                if (j < valid) acc = __fma_rn(rho, rho, acc);
            } else {
                acc = (j < 2) ? rho * rho : __fma_rn(rho, rho, acc);
            }
        }
    }
    return acc0 + acc1;
}

// ---------------------------------------------------------------------------
// Mixed precision lane accumulation: FP64 anchor, FP32 local offset.
// The linear part j * b1 is split: b1h keeps 18 significant bits so that
// j * b1h is exact in FP32 for j < 64 and its fractional part is exact; the
// remainder b0 + j (b1l + j (b2 + j b3)) is small-magnitude FP32.  cos, the
// residual and the lane sum are FP32.
// ---------------------------------------------------------------------------
template <int S, bool TAIL, bool SLOPE, bool COR = false, bool QUART = false>
__device__ __forceinline__ float lane_chi2_mixed(const float (&sv)[S], const Anchor& an, double amp0,
                                                 double ad, int valid) {
    constexpr int IL = 4;  // samples whose cosine chains run in lockstep
    static_assert(S % IL == 0, "samples per lane must be a multiple of 4");
    const float b1h = __int_as_float(__float_as_int((float)an.b1) & ~63);
    const float b1l = (float)(an.b1 - (double)b1h);
    const float b0 = (float)an.b0;
    const float b2 = (float)an.b2;
    const float b3 = (float)an.b3;
    const float b4 = (float)an.b4;
    const float A = (float)amp0;
    const float Ad = (float)ad;
    float acc[IL];
#pragma unroll
    for (int q = 0; q < IL; ++q) acc[q] = 0.0f;
#pragma unroll
    for (int g = 0; g < S; g += IL) {
        float u[IL], p[IL];
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            const int j = g + q;
            const float jj = (float)j;
            float ph;
            if (j == 0) {
                ph = b0;
            } else {
                float lin = jj * b1h;  // exact: b1h has 18 significant bits, j < 64
                lin -= rintf(lin);
                const float c3 = QUART ? __fmaf_rn(b4, jj, b3) : b3;
                const float sm = __fmaf_rn(__fmaf_rn(__fmaf_rn(c3, jj, b2), jj, b1l), jj, b0);
                ph = lin + sm;
            }
            const float r = ph - rintf(ph);
            u[q] = r * r;
            p[q] = kCos32[0];
        }
#pragma unroll
        for (int k = 1; k <= kCosDeg32; ++k) {
#pragma unroll
            for (int q = 0; q < IL; ++q) p[q] = __fmaf_rn(p[q], u[q], kCos32[k]);
        }
#pragma unroll
        for (int q = 0; q < IL; ++q) {
            const int j = g + q;
            if constexpr (COR) {
                const float m = SLOPE ? __fmaf_rn(Ad, (float)j, A) * p[q] : p[q];
                acc[q] = __fmaf_rn(sv[j], m, acc[q]);
            } else {
                const float amp = SLOPE ? __fmaf_rn(Ad, (float)j, A) : A;
                const float rho = __fmaf_rn(-amp, p[q], sv[j]);
                if (TAIL) {
                    if (j < valid) acc[q] = __fmaf_rn(rho, rho, acc[q]);
                } else {
                    acc[q] = (g == 0) ? rho * rho : __fmaf_rn(rho, rho, acc[q]);
                }
            }
        }
    }
    const float tot = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    return (COR && !SLOPE) ? A * tot : tot;
}

// ---------------------------------------------------------------------------
// One work unit of the objective: the 256 * S samples of `tile` against the
// CPG candidates of `group`.  Writes partials[cand * ntiles + tile].
// T: sample type; S: samples per lane; CPG: candidates per workgroup;
// MODE: arithmetic (see objective_unit); SLOPE: amplitude slope active.  sv holds the
// lane's samples (loaded by load_lane); cs / red are LDS scratch.
// ---------------------------------------------------------------------------
// The loads are branch-free: every lane reads S / G 16-byte groups (G
// samples each) at start indices clamped to [0, n - G] (n >= 8 >= G), so
// every address is in range and no load waits for another at a branch.
// Only a lane reaching past the last sample sees clamped data; finish_lane
// shifts its group into place and zeroes what lies past the end.
template <typename T, int S>
__device__ __forceinline__ void load_lane_raw(const BlockDesc* __restrict__ d, int tile, T (&w)[S]) {
    constexpr int G = 16 / (int)sizeof(T);
    static_assert(S % G == 0, "samples per lane must be a multiple of a 16-byte group");
    typedef T group_t __attribute__((ext_vector_type(G), aligned(sizeof(T))));
    const int64_t n = d->n;
    const int64_t n0 = (int64_t)tile * (kThreads * S) + (int64_t)threadIdx.x * S;
    const T* __restrict__ sp = static_cast<const T*>(d->samples);
#pragma unroll
    for (int g = 0; g < S / G; ++g) {
        const int64_t b = min(n0 + G * g, n - G);
        const group_t x = *(const PT_GLOBAL group_t*)(sp + b);
#pragma unroll
        for (int e = 0; e < G; ++e) w[G * g + e] = x[e];
    }
}

// sv from the raw groups; full: the whole tile lies inside the block;
// valid: samples of this lane inside the block (S when full).
template <typename V, typename T, int S>
__device__ __forceinline__ void finish_lane(const BlockDesc* __restrict__ d, int tile, const T (&w)[S],
                                            V (&sv)[S], bool& full, int& valid) {
    constexpr int G = 16 / (int)sizeof(T);
    const int64_t n = d->n;
    const int64_t tile0 = (int64_t)tile * (kThreads * S);
    const int64_t n0 = tile0 + (int64_t)threadIdx.x * S;
    full = tile0 + kThreads * S <= n;
#pragma unroll
    for (int j = 0; j < S; ++j) sv[j] = (V)w[j];
    valid = S;
    if (!full) {
        const int64_t rem = n - n0;
        valid = rem <= 0 ? 0 : (rem >= S ? S : (int)rem);
#pragma unroll
        for (int g = 0; g < S / G; ++g) {
            const int64_t s0 = n0 + G * g;
            const int64_t sh = s0 - min(s0, n - G);  // where the group's first sample landed
#pragma unroll
            for (int e = 0; e < G; ++e) {
                T x = w[G * g + e];
#pragma unroll
                for (int t = 1; e + t < G; ++t) x = sh == t ? w[G * g + e + t] : x;
                sv[G * g + e] = s0 + e < n ? (V)x : (V)0;
            }
        }
    }
}

template <typename V, typename T, int S>
__device__ __forceinline__ void load_lane(const BlockDesc* __restrict__ d, int tile, V (&sv)[S], bool& full,
                                          int& valid) {
    T w[S];
    load_lane_raw<T, S>(d, tile, w);
    finish_lane<V, T, S>(d, tile, w, sv, full, valid);
}

// Lane sum of the per-sample paths (MODE 0 FP64, 1 mixed) for one candidate:
// chi-square (tail samples masked) or correlation (masked samples are zero,
// so one loop serves both), cubic or quartic phase.
template <int MODE, int S, bool SLOPE, bool QUART, typename V>
__device__ __forceinline__ double lane_sum(const V (&sv)[S], const Anchor& an, double amp0, double ad, int valid,
                                          bool cor, bool full) {
    if constexpr (MODE == 1) {
        if (cor) return (double)lane_chi2_mixed<S, false, SLOPE, true, QUART>(sv, an, amp0, ad, valid);
        return full ? (double)lane_chi2_mixed<S, false, SLOPE, false, QUART>(sv, an, amp0, ad, valid)
                    : (double)lane_chi2_mixed<S, true, SLOPE, false, QUART>(sv, an, amp0, ad, valid);
    } else {
        if (cor) return lane_chi2_f64<S, false, SLOPE, true, QUART>(sv, an, amp0, ad, valid);
        return full ? lane_chi2_f64<S, false, SLOPE, false, QUART>(sv, an, amp0, ad, valid)
                    : lane_chi2_f64<S, true, SLOPE, false, QUART>(sv, an, amp0, ad, valid);
    }
}

// The candidates of one work unit into LDS before its evaluation: cs (and,
// for the phasor path, the tile constants rc) from the population rows, or --
// rows == nullptr -- rc from candidates the caller has already put into cs
// (past a barrier).  Ends with a barrier.  COH: the rows may be written
// inside the launch (persistent kernel).
template <int S, int CPG, int MODE, bool SLOPE, bool COH = false>
__device__ __forceinline__ void unit_setup(const BlockDesc* __restrict__ d, int tile, int group, Cand* cs,
                                           RotConst* rc, const double* trows) {
    const int cbase = group * CPG;
    const int ncand = min(CPG, d->P - cbase);
    const int tid = threadIdx.x;
    const double mt = (double)((int64_t)tile * (kThreads * S)) - d->ref;  // the tile's first sample
    if (trows != nullptr) {
        if (tid < ncand) {
            const Cand cc = make_cand<COH>(trows + (size_t)(cbase + tid) * kStride, d->fs);
            cs[tid] = cc;
            if constexpr (MODE == 2) rc[tid] = make_rot_const<S, SLOPE>(cc, mt);
        }
        __syncthreads();
    } else if constexpr (MODE == 2) {
        if (tid < ncand) rc[tid] = make_rot_const<S, SLOPE>(cs[tid], mt);
        __syncthreads();
    }
}

// MODE: 0 = FP64 with per-sample cosine polynomial, 1 = mixed precision,
// 2 = FP64 phasor recurrence.  The group's candidates are in cs (and rc)
// (unit_setup); part: the partial sums to write.  red: LDS for the lane
// sums (CPG x kThreads doubles).  COHST: the partials are read inside the
// launch (coherent stores); the leading-step form reads them only in the
// next launch, whose boundary orders plain stores.
template <int S, int CPG, int MODE, bool SLOPE, typename V, bool COHST = true>
__device__ __forceinline__ void objective_unit(const BlockDesc* __restrict__ d, int tile, int group,
                                               const V (&sv)[S], bool full, int valid, const Cand* cs,
                                               const RotConst* rc, double (*red)[kThreads], double* part) {
    const int cbase = group * CPG;
    const int ncand = min(CPG, d->P - cbase);
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const bool cor = d->objective != 0;
    const bool quart = d->quartic != 0;
    const double mt = (double)((int64_t)tile * (kThreads * S)) - d->ref;  // the tile's first sample
    const double m0 = mt + (double)(tid * S);                             // the lane's first sample
    // A wave none of whose lanes holds a chunk that is partly past the block's
    // end runs the loop of full chunks, and its lanes wholly past the end drop
    // their sums at the end (the same values as masking every sample); only
    // the wave holding the block's one partial chunk, if any, masks per sample.
    const bool wave_full = full || __ballot(valid != 0 && valid != S) == 0;
    auto keep = [&](int c, double acc) { red[c][tid] = (full || cor || valid != 0) ? acc : 0.0; };

    if constexpr (MODE == 2) {
        // the phasor path: tile constants plus per-lane polynomial updates (the
        // anchor carries the cubic and quartic terms; inside the chunk they are
        // part of the dropped terms the host bounds).  One loop per variant:
        // with the variant chosen inside the loop the compiler computes the
        // recurrence once ahead of the branch and holds the whole chunk's
        // values live.
        const double n = (double)(tid * S), n2 = n * n, nc = n - (double)(S / 2);
        auto run = [&](auto tail, auto corr) {
            for (int c = 0; c < ncand; ++c) {
                const RotConst k = rc[c];
                const double ad = SLOPE ? cs[c].Ad : 0.0;
                const double amp0 = SLOPE ? __fma_rn(ad, m0, cs[c].A) : 0.0;
                keep(c, lane_rot<S, decltype(tail)::value, SLOPE, decltype(corr)::value>(sv, k, n, n2, nc, amp0,
                                                                                         ad, valid));
            }
        };
        if (cor)
            run(std::false_type{}, std::true_type{});
        else if (wave_full)
            run(std::false_type{}, std::false_type{});
        else
            run(std::true_type{}, std::false_type{});
    } else {
        for (int c = 0; c < ncand; ++c) {
            const Cand cc = cs[c];
            const Anchor an = make_anchor(cc, m0);
            const double amp0 = SLOPE ? __fma_rn(cc.Ad, m0, cc.A) : cc.A;
            double acc;
            if (quart)
                acc = lane_sum<MODE, S, SLOPE, true>(sv, an, amp0, cc.Ad, valid, cor, wave_full);
            else
                acc = lane_sum<MODE, S, SLOPE, false>(sv, an, amp0, cc.Ad, valid, cor, wave_full);
            keep(c, acc);
        }
    }
    __syncthreads();
    // one FP64 partial per (candidate, tile): wave w takes candidates w,
    // w + 4, ..., adds each one's four wave-slices lane by lane, then runs the
    // fixed-order shuffle butterfly of all of them side by side (rows past
    // the group's candidates are read, clamped, and not stored)
    constexpr int kW = kThreads / 64, kPer = (CPG + kW - 1) / kW;
    double v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = min(wave + r * kW, CPG - 1);
        double x = red[c][lane];
#pragma unroll
        for (int q = 1; q < kW; ++q) x += red[c][lane + 64 * q];
        v[r] = x;
    }
    wave_sums(v);
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int c = wave + r * kW;
        if (lane == 0 && c < ncand) {
            double* dst = part + (size_t)(cbase + c) * d->ntiles + tile;
            if constexpr (COHST)
                xst(dst, v[r]);
            else
                gst(dst, v[r]);
        }
    }
}


// ---------------------------------------------------------------------------
// Objective of every candidate from its tile partials, by the whole
// workgroup (NT = blockDim.x threads): k = max(1, NT / P) threads per
// candidate each sum a strided subset of the tiles in a fixed order, then
// thread c adds its candidate's k subtotals in order.  The order depends
// only on (P, NT, ntiles), so every caller with the same geometry gets
// bit-identical sums.  red: NT doubles of LDS.  Returns the objective of
// candidate threadIdx.x (meaningful for threadIdx.x < P) after a barrier.
// ---------------------------------------------------------------------------
template <bool COH, int kB = 32>
__device__ __forceinline__ double reduce_partials(const BlockDesc* __restrict__ d, const double* partials,
                                                  double* red) {
    const int P = d->P, T = d->ntiles, NT = blockDim.x, t = threadIdx.x;
    const int k = NT >= P ? NT / P : 1;
    if (t < P * k) {
        const int c = t / k, part = t - c * k;
        const double* pr = partials + (size_t)c * T + part;
        const int cnt = part < T ? (T - part + k - 1) / k : 0;  // tiles part, part + k, ... < T
        double s = 0.0;
        // batches of kB loads in flight (one memory round trip per batch), then
        // added one by one in tile order
        for (int base = 0; base < cnt; base += kB) {
            double v[kB];
#pragma unroll
            for (int q = 0; q < kB; ++q) v[q] = base + q < cnt ? ld<COH>(pr + (size_t)(base + q) * k) : 0.0;
#pragma unroll
            for (int q = 0; q < kB; ++q)
                if (base + q < cnt) s += v[q];
        }
        red[t] = s;
    }
    __syncthreads();
    double tot = 0.0;
    if (t < P) {
        for (int q = 0; q < k; ++q) tot += red[t * k + q];
        // correlation objective, Eq. (2-2-5): F = 1 / (arctan(C) + pi/2)
        if (d->objective != 0) tot = 1.0 / (atan(tot) + 1.5707963267948966192);
    }
    return tot;
}

// out[p] = objective of candidate p (bare evaluation, no DE state); one
// workgroup of the DE step's size, NT doubles of dynamic LDS.
#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ void k_reduce_out(const BlockDesc* __restrict__ descs, double* __restrict__ out) {
    extern __shared__ double red[];
    const BlockDesc* d = descs;
    const double v = reduce_partials<false>(d, d->partials, red);
    if ((int)threadIdx.x < d->P) out[threadIdx.x] = v;
}
#endif

// ---------------------------------------------------------------------------
// DE: initial population (generation 0), one workgroup per block.
// x_j = lo_j + u (hi_j - lo_j), u = (w + 1/2) / 2^32 from the INIT stream.
// ---------------------------------------------------------------------------
// Initial population of one block (generation 0) and its DE state.
__device__ __forceinline__ void init_block(const BlockDesc* __restrict__ d) {
    const int i = threadIdx.x;
    if (i < d->P) {
        double x[kStride];
#pragma unroll
        for (int j = 0; j < kSlots; ++j) x[j] = d->lo[j];
#pragma unroll
        for (int j = kSlots; j < kStride; ++j) x[j] = 0.0;
        U4 w{0, 0, 0, 0};
        for (int a = 0; a < d->D; ++a) {
            if ((a & 3) == 0) w = draw4(d->seed, d->stream, (uint32_t)i, 0u, kTagInit, (uint32_t)(a >> 2));
            const double u = unit_from(word(w, a & 3));
            const int j = d->act[a];
            x[j] = __fma_rn(u, d->hi[j] - d->lo[j], d->lo[j]);
        }
        double* pr = d->pop + (size_t)i * kStride;
        double* tr = d->trial + (size_t)i * kStride;
#pragma unroll
        for (int j = 0; j < kStride; ++j) {
            pr[j] = x[j];
            tr[j] = x[j];
        }
    }
    if (i == 0) {
        DeState s;
        s.gen = 0;
        s.done = 0;
        s.flags = 0;
        s.best = 0;
        s.best_f = __builtin_inf();
        s.arrive = 0;
        s.ready = 0;
        s.slot = 0;
        s.pad = 0;
        s.old = 0.0;
        *d->st = s;
        if (d->st2 != nullptr) {
            // leading-step form: launch 1 runs the DE step of generation 0
            s.gen = 1;
            *d->st2 = s;
        }
    }
    if (d->sync != nullptr)
        for (int k = i; k < kSyncInts; k += blockDim.x) d->sync[k] = 0;  // gen_begin is 0 here
}

#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ void k_de_init(const BlockDesc* __restrict__ descs, int* __restrict__ err) {
    if (err != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *err = 0;
    init_block(descs + blockIdx.x);
}
#endif

// (f, index) pair order of the argmin: smaller objective, then smaller index.
__device__ __forceinline__ bool better(double fa, int ia, double fb, int ib) {
    return ib >= 0 && (ia < 0 || fb < fa || (fb == fa && ib < ia));
}

// Random decisions of member i's trial for generation gn (DE/rand/1/bin,
// Table 4): r1, r2, r3 distinct and != i, and the active coordinates the
// binomial crossover takes from the mutant (u < CR, or the forced jrand) as a
// bit mask over act[].  Every number comes from the fit's Philox stream at
// (i, gn); none depends on the population, so the draws can be made before
// the selection they feed.
struct Draws {
    int r1, r2, r3;
    unsigned cross;
};

// Draws from the Philox words of member i: w (the mutation call) and u0, u1
// (the crossover calls of active coordinates 0-3 and 4-7).
__device__ __forceinline__ Draws draws_from(const U4& w, const U4& u0, const U4& u1, int i, int P, int D,
                                            double CR) {
    Draws r;
    int r1 = index_from(w.x, P - 1);
    if (r1 >= i) ++r1;
    const int lo2 = min(i, r1), hi2 = max(i, r1);
    int r2 = index_from(w.y, P - 2);
    if (r2 >= lo2) ++r2;
    if (r2 >= hi2) ++r2;
    int e0 = i, e1 = r1, e2 = r2, t;
    if (e0 > e1) { t = e0; e0 = e1; e1 = t; }
    if (e1 > e2) { t = e1; e1 = e2; e2 = t; }
    if (e0 > e1) { t = e0; e0 = e1; e1 = t; }
    int r3 = index_from(w.z, P - 3);
    if (r3 >= e0) ++r3;
    if (r3 >= e1) ++r3;
    if (r3 >= e2) ++r3;
    const int jr = index_from(w.w, D);
    unsigned cross = 0;
#pragma unroll
    for (int a = 0; a < kSlots; ++a) {
        const uint32_t x = word(a < 4 ? u0 : u1, a & 3);
        if (a < D && (unit_from(x) < CR || a == jr)) cross |= 1u << a;
    }
    r.r1 = r1;
    r.r2 = r2;
    r.r3 = r3;
    r.cross = cross;
    return r;
}

__device__ __forceinline__ Draws trial_draws(const BlockDesc* __restrict__ d, int i, uint32_t gn) {
    const U4 w = draw4(d->seed, d->stream, (uint32_t)i, gn, kTagMut, 0u);
    const U4 u0 = draw4(d->seed, d->stream, (uint32_t)i, gn, kTagXover, 0u);
    U4 u1{0, 0, 0, 0};
    if (d->D > 4) u1 = draw4(d->seed, d->stream, (uint32_t)i, gn, kTagXover, 1u);
    return draws_from(w, u0, u1, i, d->P, d->D, d->CR);
}

// The same draws made by the eight lanes of an octet (lanes 8c .. 8c + 7 of
// one wave, all active, all for member i): lane k of the octet evaluates one
// Philox call (k = 0 the mutation call, k = 1, 2 the crossover calls), the
// octet exchanges the words and every lane derives the draws.  One Philox
// chain per lane instead of three in a row; bit-identical to trial_draws.
__device__ __forceinline__ Draws trial_draws_octet(const BlockDesc* __restrict__ d, int i, uint32_t gn) {
    const int lane = (int)(threadIdx.x & 63u), k = lane & 7, base = lane & ~7;
    const U4 mine = draw4(d->seed, d->stream, (uint32_t)i, gn, k == 0 ? kTagMut : kTagXover,
                          (uint32_t)(k == 0 ? 0 : k - 1));
    auto from = [&](int src) {
        U4 v;
        v.x = (uint32_t)__shfl((int)mine.x, base + src, 64);
        v.y = (uint32_t)__shfl((int)mine.y, base + src, 64);
        v.z = (uint32_t)__shfl((int)mine.z, base + src, 64);
        v.w = (uint32_t)__shfl((int)mine.w, base + src, 64);
        return v;
    };
    const U4 w = from(0), u0 = from(1), u1 = from(2);
    return draws_from(w, u0, u1, i, d->P, d->D, d->CR);
}

// Quotients of small non-negative integers by an FP32 reciprocal instead of
// the integer division sequence (tens of dependent instructions on the
// chain before the leading step's loads).
// floor(a / b) for 0 <= a <= 4096, b >= 1: the fractional part of
// (a + 1/2) / b lies in [1/(2b), 1 - 1/(2b)], and the reciprocal (1 ulp)
// and the product (1/2 ulp) move the quotient by less than 2^-11 / b.
__device__ __forceinline__ int div_small(int a, int b) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}
// floor(a / b) for 0 <= a < 2^23, b >= 1: the FP32 estimate is within one
// of the quotient, and one remainder test corrects it.
__device__ __forceinline__ int div_mid(int a, int b) {
    int q = (int)((float)a * __builtin_amdgcn_rcpf((float)b));
    const int r = a - q * b;
    q += r >= b ? 1 : 0;
    q -= r < 0 ? 1 : 0;
    return q;
}

// Draws of one member packed into the pad slot (slot 7) of its trial row
// (P <= 256, at most 7 active coordinates): r1, r2, r3 in bytes 0-2, the
// crossover mask in byte 3 of the low word; the high word holds the stop
// flag the launch reading the row needs (the fit has stopped).
__device__ __forceinline__ unsigned long long pack_draws(const Draws& w, bool done) {
    return (unsigned long long)((unsigned)w.r1 | ((unsigned)w.r2 << 8) | ((unsigned)w.r3 << 16) | (w.cross << 24)) |
           ((unsigned long long)done << 32);
}
__device__ __forceinline__ Draws unpack_draws(unsigned long long u) {
    return Draws{(int)(u & 255u), (int)((u >> 8) & 255u), (int)((u >> 16) & 255u), (unsigned)((u >> 24) & 255u)};
}

// Trial vector y of member i from the selected population xs (P x kSlots,
// LDS) and its draws: v = x_r1 + F (x_r2 - x_r3) with the half-way bound
// rule on the crossed coordinates, x_i elsewhere.
__device__ __forceinline__ void apply_trial(const BlockDesc* __restrict__ d, const double* xs, int i,
                                            const Draws& r, double (&y)[kStride]) {
#pragma unroll
    for (int j = 0; j < kSlots; ++j) y[j] = xs[i * kSlots + j];
#pragma unroll
    for (int j = kSlots; j < kStride; ++j) y[j] = 0.0;
    for (int a = 0; a < d->D; ++a) {
        if (!((r.cross >> a) & 1u)) continue;
        const int j = d->act[a];
        const double x1 = xs[r.r1 * kSlots + j];
        double v = __fma_rn(d->F, xs[r.r2 * kSlots + j] - xs[r.r3 * kSlots + j], x1);
        if (v < d->lo[j]) v = (d->lo[j] + x1) * 0.5;
        if (v > d->hi[j]) v = (d->hi[j] + x1) * 0.5;
        y[j] = v;
    }
}

// Best member of the selected population: argmin of fsel (thread i holds
// member i's value, -1 index past P), lowest index on ties; every thread
// gets the result.  fr / ix: NT doubles / ints of LDS.
__device__ __forceinline__ void argmin_members(int P, double fsel, double* fr, int* ix, int& best, double& bf) {
    const int NT = blockDim.x, i = threadIdx.x;
    if (P <= 64) {
        // wave 0: the smallest value, then the lowest lane holding it (the
        // lowest index on ties; a member whose objective is NaN is never best
        // unless all are)
        if (i < 64) {
            const double f = i < P ? fsel : __builtin_inf();
            double m = f;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
            const unsigned long long hit = __ballot(i < P && f == m);
            const int id = hit ? __ffsll(hit) - 1 : 0;
            const double fb = __shfl(f, id, 64);
            if (i == 0) {
                fr[0] = fb;
                ix[0] = id;
            }
        }
        __syncthreads();
    } else {
        fr[i] = fsel;
        ix[i] = i < P ? i : -1;
        __syncthreads();
        for (int off = NT >> 1; off > 0; off >>= 1) {
            if (i < off && better(fr[i], ix[i], fr[i + off], ix[i + off])) {
                fr[i] = fr[i + off];
                ix[i] = ix[i + off];
            }
            __syncthreads();
        }
    }
    best = ix[0];
    bf = fr[0];
}

// ---------------------------------------------------------------------------
// DE: one generation step per block (blockDim = NT >= P, power of two).
//   1. f(trial_i) = sum of tile partials (reduce_partials)
//   2. selection: x_i <- trial_i iff f(trial_i) <= f(x_i)  (gen 0: accept)
//   3. best = argmin, lowest index on ties; hist[g] = best value
//   4. stop rule: VTR, window rule, generation cap
//   5. trial_i of generation g + 1: r1, r2, r3 distinct and != i, jrand,
//      v = x_r1 + F (x_r2 - x_r3) with the half-way bound rule, binomial
//      crossover with rate CR and the forced coordinate jrand.
// Member rows and the state are fetched before the reduction so their
// latency overlaps it.  Dynamic LDS: P * kSlots + 2 NT doubles + NT ints.
// ---------------------------------------------------------------------------
// ROWS_COH: population rows and DE state may be written inside the launch
// (persistent kernel); PART_COH: the partial sums may (fused or persistent).
template <bool ROWS_COH, bool PART_COH>
__device__ __forceinline__ void de_step_body(const BlockDesc* __restrict__ d, double* lds) {
    DeState* st = d->st;
    const int P = d->P, NT = blockDim.x, i = threadIdx.x;
    double* xs = lds;                              // P x kSlots
    double* red = xs + (size_t)P * kSlots;         // NT
    double* fr = red + NT;                         // NT
    int* ix = reinterpret_cast<int*>(fr + NT);     // NT
    __shared__ int s_done, s_gen, s_stop;
    __shared__ double s_old;

    double tr[kSlots], po[kSlots], fo = 0.0;
    if (i < P) {
        const double* a = d->trial + (size_t)i * kStride;
        const double* b = d->pop + (size_t)i * kStride;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) {
            tr[j] = ld<ROWS_COH>(a + j);
            po[j] = ld<ROWS_COH>(b + j);
        }
        fo = ld<ROWS_COH>(d->fpop + i);
    }
    if (i == 0) {
        // Atomic (vector, agent-scope) loads: inside the persistent kernel these
        // words are rewritten by other workgroups, so they must not come from
        // the scalar cache.
        const int g0 = __hip_atomic_load(&st->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_done = __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_gen = g0;
        s_old = (d->rel_tol > 0.0 && d->window > 0 && g0 >= d->window)
                    ? __hip_atomic_load(d->hist + (g0 - d->window), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                    : 0.0;
    }
    const double ft = reduce_partials<PART_COH>(d, d->partials, red);  // contains a barrier
    if (s_done) return;
    const int g = s_gen;

    // selection (generation 0 accepts the initial population); the global
    // stores wait until after the last barrier, which would otherwise wait
    // for them
    double fsel = __builtin_inf();
    bool take = false;
    if (i < P) {
        take = g == 0 || ft <= fo;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) xs[i * kSlots + j] = take ? tr[j] : po[j];
        fsel = take ? ft : fo;
    }

    // argmin, lowest index on ties
    int best;
    double bf;
    argmin_members(P, fsel, fr, ix, best, bf);

    int flags = 0;
    if (i == 0) {
        if (bf <= d->vtr) flags |= 4;  // PT_FLAG_VTR
        if (d->rel_tol > 0.0 && d->window > 0 && g >= d->window && s_old - bf <= d->rel_tol * bf)
            flags |= 1;  // PT_FLAG_CONVERGED
        if (!flags && g >= d->max_gens) flags |= 2;  // PT_FLAG_MAXGEN
        s_stop = flags != 0;
    }
    __syncthreads();
    if (take) {
        double* prow = d->pop + (size_t)i * kStride;
#pragma unroll
        for (int j = 0; j < kSlots; ++j) xst(prow + j, tr[j]);
        xst(d->fpop + i, ft);
    }
    if (i == 0) {
        xst(d->hist + g, bf);
        xsti(&st->best, best);
        xst(&st->best_f, bf);
        if (flags) {
            xsti(&st->flags, flags);
            xsti(&st->done, 1);
        } else {
            xsti(&st->gen, g + 1);
        }
    }
    if (s_stop || i >= P) return;

    double y[kStride];
    apply_trial(d, xs, i, trial_draws(d, i, (uint32_t)(g + 1)), y);
    double* trow = d->trial + (size_t)i * kStride;
#pragma unroll
    for (int j = 0; j < kStride; ++j) xst(trow + j, y[j]);
}

#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ __launch_bounds__(1024) void k_de_step(const BlockDesc* __restrict__ descs) {
    extern __shared__ double lds[];
    de_step_body<false, false>(descs + blockIdx.x, lds);
}
#endif

// ---------------------------------------------------------------------------
// Inputs of a leading step: the slot it reads (tile partials, population
// rows, trial rows and population objectives of slot p ^ 1) and P and
// ntiles.  A one-block launch passes them as kernel arguments, which arrive
// in scalar registers at wave launch, so the step's loads do not wait for the
// descriptor; otherwise lead_in_of reads them from the descriptor.
struct LeadIn {
    const double* part;
    const double* rows;
    const double* trial;
    const double* fpop;
    int P, T;
};

__device__ __forceinline__ LeadIn lead_in_of(const BlockDesc* __restrict__ d, int L) {
    const int p = L & 1;
    const double *pop0 = d->pop, *pop1 = d->pop2, *tr0 = d->trial, *tr1 = d->trial2;
    const double *fp0 = d->fpop, *fp1 = d->fpop2, *pa0 = d->partials, *pa1 = d->partials2;
    return LeadIn{p ? pa0 : pa1, p ? pop0 : pop1, p ? tr0 : tr1, p ? fp0 : fp1, d->P, d->ntiles};
}

// Leading DE step (fits with P <= 256, blockDim = 256).  Launch L of a fit
// (L a kernel argument) evaluates the trial population of generation L.
// Before that, every objective workgroup of the launch repeats the DE step
// of generation L - 1 for itself -- the objectives of all P trials from
// their tile partials, and the selection -- and draws the trials of its own
// candidate group (BOOK = false).  One more workgroup per block (BOOK =
// true) runs the same step with the rest of it: the best member, the
// best-so-far history and the stop rule, and it stores the selected
// population, its objectives and the state the next launch reads.
// Objective workgroups do not wait for the stop rule: after a stop they
// evaluate one generation that nothing reads.  No workgroup waits for
// another and none reads what another writes in the same launch: launch
// parity p reads the state of slot p and the rows, objectives and partials
// of slot p ^ 1 (all written by the previous launch) and writes the
// opposite slots (BlockDesc).  Reduction order, selection, argmin and random
// draws are those of de_step_body, so fits are bit-identical to the other
// launch forms.  The random draws of the group's trials depend on L only,
// so they are made while the step's loads are in flight.  A fit takes
// max_gens + 2 launches: the last one runs only the DE step of generation
// max_gens, which stops the fit.  After a stop, each further launch copies
// the final state to the other slot, so every later launch sees it.
//
// Returns false when there is nothing to evaluate (BOOK, or the fit has
// stopped); otherwise the group's candidates are in cs, past a barrier, and
// conv (the conversion of the lane's samples, raw, loaded by the step) has
// run on every wave but the trial wave, which runs it next.
// lds: the DE step's dynamic LDS plus P * kSlots doubles (2 P kSlots + 2 *
// 256 doubles + 256 ints).  Workgroups of kThreads threads (k_objective's):
// a compile-time count keeps the launch's geometry out of the chain of
// dependent loads before the step's data loads.
// ---------------------------------------------------------------------------
// The wave that builds a group's trials.  The others convert their lanes'
// samples (conv) meanwhile, and the trial wave does while wave 0 makes the
// tile constants; neither conversion waits for the samples before the
// selection is done.
constexpr int kTrialWave = 1;
static_assert(kThreads >= 128, "the trial wave is the second wave");

template <int CPG, bool BOOK, bool PRE, typename RT, int RS, typename Conv>
__device__ __forceinline__ bool de_lead(const BlockDesc* __restrict__ d, int L, int tile, int group, Cand* cs,
                                        double* lds, const LeadIn& in, RT (&raw)[RS], Conv&& conv) {
    const int p = L & 1;
    constexpr int NT = kThreads;
    const int P = in.P, i = threadIdx.x;
    double* xs = lds;                              // P x kSlots: trial rows, then the selected rows
    double* red = xs + (size_t)P * kSlots;         // NT
    double* fr = red + NT;                         // NT
    int* ix = reinterpret_cast<int*>(fr + NT);     // NT
    double* xp = reinterpret_cast<double*>(ix + NT);  // P x kSlots: population rows
    __shared__ int s_done, s_stop;
    __shared__ double s_old;
    // the slot the step reads (in); the state and the outputs from the
    // descriptor, both slots' pointers read unconditionally and then selected
    // (through a parity-selected field address they would cost one more
    // dependent scalar round trip)
    const double* rows_in = in.rows;  // slot p ^ 1
    const double* trial_in = in.trial;
    const double* fpop_in = in.fpop;
    const double* part_in = in.part;
    const int cbase = group * CPG;
    const int ncand = min(CPG, P - cbase);

    // 1. every load of the step, issued together: the tile partials (k threads
    //    per member summing tiles part, part + k, ... as reduce_partials does),
    //    the population rows and objectives, the state
    // loads per thread in one batch: 17 covers P = 40 up to 102 tiles (400 000
    // samples at 16 per lane) in one memory round trip; 24 would cost the
    // kernel its fourth wave per SIMD (143 VGPRs instead of 115)
    constexpr int kB = 17;
    const int T = in.T;
    // (T < 2^21: a block holds fewer than 2^31 samples, a tile at least 2^10)
    const int k = NT >= P ? div_small(NT, P) : 1;
    const int pm = div_small(i, k), part = i - pm * k;
    const int cnt = (i < P * k && part < T) ? div_mid(T - part + k - 1, k) : 0;
    // this thread's trial coordinate (candidate c = i / 8 of the group, slot
    // j = i % 8): its bounds, read first (per-lane indices into the
    // descriptor, so vector loads; issued after the step's loads they would
    // wait for them)
    const int c = (i & 63) >> 3, j = i & 7;
    const int jc = j < kSlots ? j : kSlots - 1;
    const double lo_j = gld(&d->lo[jc]), hi_j = gld(&d->hi[jc]);
    const double* pr = part_in + (size_t)pm * T + part;
    double v[kB];
    // (no load sits in a branch: out-of-range ones read a valid address and
    // are discarded, so none waits for another)
#pragma unroll
    for (int q = 0; q < kB; ++q) {
        const double x = gld(q < cnt ? pr + (size_t)q * k : part_in);
        v[q] = q < cnt ? x : 0.0;
    }
    // rows: element e = member * kSlots + slot, kR per thread (P <= 73 in one round)
    constexpr int kR = 2;
    const int ne = P * kSlots;
    double rt[kR], rp[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int e = min(i + r * NT, ne - 1);
        const int mem = e / kSlots;
        const size_t off = (size_t)mem * kStride + (e - mem * kSlots);
        rt[r] = gld(trial_in + off);
        rp[r] = gld(rows_in + off);
    }
    // the member a thread selects: for P <= 64 in an objective workgroup the
    // trial wave's lanes select (so the trials need no barrier after the
    // selection, only the wave's own order), otherwise thread i selects i
    const bool one = !BOOK && P <= 64;
    const int sm = one ? (i & 63) : i;
    const bool selects = one ? (i >> 6) == kTrialWave && sm < P : i < P;
    const double fo = gld(fpop_in + min(sm, P - 1));
    // PRE: this lane's trial draws, made by the previous launch's bookkeeping
    // workgroup and kept in the pad slot of the trial rows this step reads
    // (and, in the high word, whether the fit has stopped: no dependent
    // loads through the descriptor's state pointer)
    unsigned long long dpk = 0ull;
    if constexpr (PRE)
        dpk = gld(reinterpret_cast<const unsigned long long*>(trial_in + (size_t)min(cbase + c, P - 1) * kStride +
                                                              kSlots));
    // what comes from the descriptor, behind the step's loads: the lane's
    // samples (needed only by the objective after the step), the state and
    // the slots the step writes
    if constexpr (!BOOK) load_lane_raw<RT, RS>(d, tile, raw);
    // every descriptor field the rest of the launch reads, fetched in the
    // scalar round trip the samples' address needs anyway (read later, after
    // a barrier, each line of the descriptor would be one more round trip;
    // the empty asm only makes the compiler hold them here)
    if constexpr (PRE)
        asm volatile("" ::"s"(d->ref), "s"(d->F), "s"(d->objective), "s"(d->quartic), "s"(d->amask),
                     "s"(d->trial), "s"(d->trial2), "s"(d->partials), "s"(d->partials2));
    DeState *st0 = d->st, *st1 = d->st2;
    double *pop0 = d->pop, *pop1 = d->pop2, *tr0 = d->trial, *tr1 = d->trial2;
    double *fp0 = d->fpop, *fp1 = d->fpop2;
    const DeState* st_in = p ? st1 : st0;
    DeState* st_out = p ? st0 : st1;
    double* rows_out = p ? pop1 : pop0;  // slot p
    double* trial_out = p ? tr1 : tr0;
    double* fpop_out = p ? fp1 : fp0;
    const int st_done = PRE ? 0 : gld(&st_in->done);
    const double st_old = BOOK ? gld(&st_in->old) : 0.0;

    // 2. while they are in flight: the random draws of this thread's trial
    //    coordinate (candidate c = i / 8 of the group, slot j = i % 8); the
    //    bookkeeping workgroup makes every member's draws of the next launch,
    //    to store them with the stop flag in the pad slot of the trial rows
    //    that launch reads (PRE)
    const int wave = i >> 6;
    const bool tw = !BOOK && L > 0 && c < ncand && wave == kTrialWave;
    // this thread's coordinate's place among the active slots
    const unsigned am = (unsigned)d->amask;
    const int a_j = ((am >> j) & 1u) ? __builtin_popcount(am & ((1u << j) - 1u)) : -1;
    const double Fm = d->F, fs = d->fs;
    Draws dr{0, 0, 0, 0u};
    if constexpr (BOOK) {
        if (i < P) dr = trial_draws(d, i, (uint32_t)(L + 1));
    } else if constexpr (!PRE) {
        // (every lane of the wave makes the octet draws, so that the octets'
        // exchanges see all their lanes; only those with tw use them)
        if (L > 0 && wave == kTrialWave) dr = trial_draws_octet(d, cbase + c, (uint32_t)L);
    }

    // 3. objectives of all P trials, in reduce_partials' order
    double sp = 0.0;
#pragma unroll
    for (int q = 0; q < kB; ++q)
        if (q < cnt) sp += v[q];
    for (int base = kB; base < cnt; base += kB) {
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const double x = gld(base + q < cnt ? pr + (size_t)(base + q) * k : part_in);
            v[q] = base + q < cnt ? x : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kB; ++q)
            if (base + q < cnt) sp += v[q];
    }
    if (i < P * k) red[i] = sp;
#pragma unroll
    for (int r = 0; r < kR; ++r) {
        const int e = i + r * NT;
        if (e < ne) {
            xs[e] = rt[r];
            xp[e] = rp[r];
        }
    }
    for (int e = i + kR * NT; e < ne; e += NT) {  // P > 73
        const int mem = e / kSlots;
        const size_t off = (size_t)mem * kStride + (e - mem * kSlots);
        xs[e] = gld(trial_in + off);
        xp[e] = gld(rows_in + off);
    }
    // the stop state: the bookkeeping workgroup needs it here; objective
    // workgroups only after the selection (its loads, two dependent round
    // trips through the descriptor, then have that much longer to arrive)
    if (BOOK && i == 0) {
        s_done = st_done;
        s_old = st_old;
    }
    __syncthreads();
    double ft = 0.0;
    if (selects) {
        // the member's k subtotals added in order, read eight at a time (one
        // LDS round trip per eight rather than per subtotal)
        for (int b = 0; b < k; b += 8) {
            double w[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) w[q] = red[sm * k + min(b + q, k - 1)];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (b + q < k) ft += w[q];
        }
        // correlation objective, Eq. (2-2-5): F = 1 / (arctan(C) + pi/2)
        if (d->objective != 0) ft = 1.0 / (atan(ft) + 1.5707963267948966192);
    }
    // (the bookkeeping workgroup's pad-slot stores, at each of its exits)
    auto store_pad = [&](bool done) {
        if (BOOK && i < P)
            gst(reinterpret_cast<unsigned long long*>(trial_out + (size_t)i * kStride + kSlots), pack_draws(dr, done));
    };
    if (BOOK && s_done) {
        store_pad(true);
        if (i == 0) {
            const DeState s = *st_in;
            xsti(&st_out->gen, s.gen);
            xsti(&st_out->done, s.done);
            xsti(&st_out->flags, s.flags);
            xsti(&st_out->best, s.best);
            xst(&st_out->best_f, s.best_f);
            xsti(&st_out->slot, s.slot);
        }
        return false;
    }
    if (L == 0) {
        // generation 0: the initial population as stored (slot 0); no step
        if (BOOK) {
            store_pad(false);
            return false;
        }
        if (i < ncand) cs[i] = make_cand<false>(trial_out + (size_t)(cbase + i) * kStride, d->fs);
        if (i == 0) s_done = st_done;  // (0 for PRE: a fit starts unstopped)
        if (wave != kTrialWave) conv();
        __syncthreads();
        return !s_done;
    }
    const int g = L - 1;

    // 4. selection (generation 0 accepts the initial population)
    double fsel = __builtin_inf();
    if (selects) {
        const bool take = g == 0 || ft <= fo;
        if (!take) {
#pragma unroll
            for (int q = 0; q < kSlots; ++q) xs[sm * kSlots + q] = xp[sm * kSlots + q];
        }
        fsel = take ? ft : fo;
    }
    if constexpr (!BOOK) {
        // a stopped fit evaluates nothing (the selection above wrote only
        // LDS); every thread holds the same stop flag
        const int done = PRE ? (int)(dpk >> 32) : st_done;
        if (one) {
            if (done) return false;
            // the trial wave's own selected rows: its LDS accesses stay in
            // program order, which the wave-scope fences keep the compiler to
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            if (i == 0) s_done = done;
            __syncthreads();  // selected rows complete
            if (s_done) return false;
        }
        if (wave != kTrialWave) conv();
        if constexpr (PRE) dr = unpack_draws(dpk);
        // 5. the group's trials, one coordinate per thread (apply_trial's
        //    arithmetic), straight into the candidates' turn-domain form
        if (tw) {
            const int m = cbase + c;
            double y = 0.0;
            if (j < kSlots) {
                y = xs[m * kSlots + j];
                if (a_j >= 0 && ((dr.cross >> a_j) & 1u)) {
                    const double x1 = xs[dr.r1 * kSlots + j];
                    double vm = __fma_rn(Fm, xs[dr.r2 * kSlots + j] - xs[dr.r3 * kSlots + j], x1);
                    if (vm < lo_j) vm = (lo_j + x1) * 0.5;
                    if (vm > hi_j) vm = (hi_j + x1) * 0.5;
                    y = vm;
                }
                cand_member(cs[c], j) = cand_value(j, y, fs);
            }
            // (the pad slot carries the next launch's draws, stored by the
            // bookkeeping workgroup)
            if (tile == 0 && j < kSlots) gst(trial_out + (size_t)m * kStride + j, y);
        }
        __syncthreads();
        return true;
    }

    // bookkeeping: best member, stop rule, stores
    int best;
    double bf;
    argmin_members(P, fsel, fr, ix, best, bf);  // contains a barrier
    if (i == 0) {
        int flags = 0;
        if (bf <= d->vtr) flags |= 4;  // PT_FLAG_VTR
        if (d->rel_tol > 0.0 && d->window > 0 && g >= d->window && s_old - bf <= d->rel_tol * bf)
            flags |= 1;  // PT_FLAG_CONVERGED
        if (!flags && g >= d->max_gens) flags |= 2;  // PT_FLAG_MAXGEN
        s_stop = flags;
    }
    __syncthreads();
    const int flags = s_stop;
    if (i < P) {
        double* r = rows_out + (size_t)i * kStride;
#pragma unroll
        for (int q = 0; q < kSlots; ++q) gst(r + q, xs[i * kSlots + q]);
#pragma unroll
        for (int q = kSlots; q < kStride; ++q) gst(r + q, 0.0);
        gst(fpop_out + i, fsel);
    }
    store_pad(flags != 0);
    if (i == 0) {
        xst(d->hist + g, bf);
        // the window rule of the next step compares with hist[g + 1 - window]
        double old = 0.0;
        if (!flags && d->rel_tol > 0.0 && d->window > 0 && g + 1 >= d->window)
            old = d->window == 1 ? bf : gld(d->hist + (g + 1 - d->window));
        // the next launch evaluates generation g + 2 after the step of g + 1
        xsti(&st_out->gen, flags ? g : g + 2);
        xsti(&st_out->done, flags != 0);
        xsti(&st_out->flags, flags);
        xsti(&st_out->best, best);
        xst(&st_out->best_f, bf);
        xsti(&st_out->slot, p);
        xst(&st_out->old, old);
    }
    return false;
}

// ---------------------------------------------------------------------------
// Persistent fit kernel: every generation of every block of a launch in one
// cooperative grid.  Workgroup w owns a fixed list of work units (those of
// its XCD's contiguous range of units, round-robin over the XCD's
// workgroups); with at most one unit per workgroup its samples stay in
// registers for the whole fit.  Per block there is no grid-wide barrier:
// each finished unit bumps the block's arrival counter, the workgroup that
// completes a generation runs that block's DE step and publishes the next
// trial population by raising the block's ready counter, and a workgroup
// about to evaluate generation g of a block waits until ready >= g.
//
// Synchronisation words live in BlockDesc::sync (kSyncInts ints per block,
// one 128-byte line per counter): a unit's arrival is counted in its XCD
// range's counter, the last arrival of a range counts the range in the
// block counter, and the DE step publishes the ready generation to one copy
// per XCD range, so no counter or polled word serves more than one XCD's
// workgroups.  Launches may start at any generation (gen_begin) and run
// `steps` generations; counters restart at every launch.
//
// Progress: every workgroup processes generation g of all its units before
// any unit of generation g + 1, so the workgroups at the lowest generation
// only ever wait for DE steps whose units are all finished; with all
// workgroups resident (cooperative launch) the grid always drains.  Waits
// are bounded by spin_ticks of the constant-rate clock as a safety net: on
// expiry the kernel sets *err and every workgroup leaves.
// ---------------------------------------------------------------------------
constexpr int kPersistLds = 256 * kSlots + 2 * 256 + 128;  // doubles: DE step (P <= 256) or one unit

// Poll with relaxed agent-scope loads (no cache maintenance per poll), then
// one acquire fence once the value is reached.  Called by one thread.
__device__ __forceinline__ bool spin_until_ge(int* p, int want, int* err, uint64_t spin_ticks) {
    const uint64_t t0 = wall_clock64();
    for (;;) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, PT_ACQ_SCOPE);
            return true;
        }
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > spin_ticks) {
            __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

// Number of units of block d that fall in XCD range x ([x Ux, (x + 1) Ux)).
__device__ __forceinline__ int units_in_range(const BlockDesc* d, int x, int Ux, int total_units) {
    const int ub = d->unit_begin, ue = ub + d->ntiles * d->ngroups;
    const int rb = x * Ux, re = min(total_units, rb + Ux);
    return max(0, min(ue, re) - max(ub, rb));
}

// Objective kernel: one work unit per workgroup (fused = 0; 1 and >= 2 add
// the DE step, see below).  Units are remapped so
// that the candidate groups of a tile run on one XCD (workgroup ids are dealt
// round-robin to the 8 XCDs, so XCD x runs units [x Ux, (x + 1) Ux), Ux =
// gridDim / 8).
//
// fused != 0 (fits with P <= 256): the DE step of each block runs in the
// same launch, in the workgroup that finishes the block's last unit.  Every
// workgroup counts its finished unit on the block's counter for its XCD
// range; the one completing a range counts the range on the block's range
// counter; the one completing that runs de_step_body (the same code, thread
// count and reduction order as k_de_step, so fits are bit-identical to the
// two-launch form) and clears the counters for the next launch.  No
// workgroup waits for another.  Partial sums are coherent stores and loads
// (xst / xld), so the fences only order each wave's accesses around its
// counter update.
//
// fused = 2 + k (fits with P <= 256): the leading-step form (de_lead), launch
// L = gen_begin + k of each block (gen_begin is 0 for a fit, a block's own
// offset in the serving loop): every objective workgroup first runs the DE
// step of generation L - 1 for itself, then evaluates its candidates of
// generation L; the grid has one more unit per block (after the objective
// units) that keeps the block's DE state.
//
// Dynamic LDS for fused != 0: the DE step's (P * kSlots + 2 * 256 doubles +
// 256 ints), and P * kSlots doubles more for fused >= 2.
// LEAD: the instance for the leading-step form (fused >= 2 only), 1 reading
// the step's inputs from the descriptor, 2 from the kernel arguments (one
// block); the other forms use the instance without it (LEAD = 0), which
// needs fewer registers.
template <typename T, int S, int CPG, int MODE, bool SLOPE, int LEAD>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_objective(
    int fused, int nblk, int total_units, int lp, const double* __restrict__ l_part, const double* __restrict__ l_rows,
    const double* __restrict__ l_trial, const double* __restrict__ l_fpop, const BlockDesc* __restrict__ descs) {
    // workgroups (a multiple of 8); the one-block leading form launches the
    // units plus one, rounded up to 8, and derives it from its arguments (the
    // grid size is otherwise one more kernel-argument load before the step)
    const int nwg = LEAD == 2 ? (total_units + 1 + 7) & ~7 : (int)gridDim.x;
    const int bid = blockIdx.x;
    const int Ux = nwg >> 3;
    const int unit = (bid & 7) * Ux + (bid >> 3);
    __shared__ Cand cs[CPG];
    __shared__ RotConst rc[MODE == 2 ? CPG : 1];
    extern __shared__ double de_lds[];
    if (unit >= total_units) {
        // leading-step form: unit total_units + b keeps block b's DE state
        if constexpr (LEAD) {
            if (unit < total_units + nblk) {
                float none[1] = {0.0f};
                const BlockDesc* db = descs + (unit - total_units);
                const int Lb = db->gen_begin + fused - 2;
                de_lead<CPG, true, false>(db, Lb, 0, 0, cs, de_lds, lead_in_of(db, Lb), none, [] {});
            }
        }
        return;
    }
    const BlockDesc* __restrict__ d = LEAD == 2 ? descs : descs + find_block(descs, nblk, unit);
    int tile, group, L = 0;
    LeadIn lin{};
    if constexpr (LEAD == 2) {
        // one block (launch index fused - 2, first unit 0) whose step inputs
        // came as kernel arguments, lp = P | ntiles << 9: nothing here waits
        // for the descriptor before the step's loads are issued
        // (the host takes this form only for fewer than 2^23 units, the
        // range of div_mid)
        const int P = lp & 511, ng = (P + CPG - 1) / CPG;
        tile = div_mid(unit, ng);
        group = unit - tile * ng;
        L = fused - 2;
        lin = LeadIn{l_part, l_rows, l_trial, l_fpop, P, lp >> 9};
    } else {
        // leading-step form: every descriptor field read before the step's
        // data loads, fetched together (left to the compiler, they came in
        // three dependent scalar round trips).  The empty asm only makes the
        // compiler hold them all in scalar registers here; it emits nothing.
        if constexpr (LEAD)
            asm volatile("" ::"s"(d->samples), "s"(d->n), "s"(d->P), "s"(d->ntiles), "s"(d->ngroups),
                         "s"(d->unit_begin), "s"(d->gen_begin), "s"(d->st), "s"(d->st2), "s"(d->pop),
                         "s"(d->pop2), "s"(d->trial), "s"(d->trial2), "s"(d->fpop), "s"(d->fpop2),
                         "s"(d->partials), "s"(d->partials2), "s"(d->F), "s"(d->objective));
        // (the leading-step form reads its stop state inside de_lead, which
        // must also run after a stop to copy the state forward)
        if (!LEAD && d->st != nullptr && d->st->done) return;
        const int local = unit - d->unit_begin;
        tile = local / d->ngroups;
        group = local - tile * d->ngroups;
        if constexpr (LEAD) {
            L = d->gen_begin + fused - 2;  // the block's launch index (gen_begin: its offset)
            lin = lead_in_of(d, L);
        }
    }

    __shared__ double red[CPG][kThreads];
    __shared__ int s_last;
    using V = typename std::conditional<MODE == 1, float, double>::type;
    V sv[S];
    bool full;
    int valid;
    if constexpr (LEAD) {
        // the samples' loads overlap the DE step's, and the step converts
        // them into sv where each wave would otherwise idle
        T raw[S];  // loaded inside de_lead, behind the step's own loads
        auto conv = [&] { finish_lane<V, T, S>(d, tile, raw, sv, full, valid); };
        if (!de_lead<CPG, false, LEAD == 2>(d, L, tile, group, cs, de_lds, lin, raw, conv)) return;
        if ((int)(threadIdx.x >> 6) == kTrialWave) conv();  // while wave 0 makes the tile constants
        unit_setup<S, CPG, MODE, SLOPE>(d, tile, group, cs, rc, nullptr);
        objective_unit<S, CPG, MODE, SLOPE, V, false>(d, tile, group, sv, full, valid, cs, rc, red,
                                                      (L & 1) ? d->partials2 : d->partials);
    } else {
        load_lane<V, T, S>(d, tile, sv, full, valid);
        unit_setup<S, CPG, MODE, SLOPE>(d, tile, group, cs, rc, d->trial);
        objective_unit<S, CPG, MODE, SLOPE>(d, tile, group, sv, full, valid, cs, rc, red, d->partials);
        if (!fused) return;

        int* sync = d->sync;
        const int xcd = bid & 7;
        __syncthreads();  // every wave's partial stores are issued
        // (one counter per block instead of per XCD range: fits 30 % slower on MI355X,
        // the same-address atomics from all XCDs serialise)
        if (threadIdx.x == 0) {
            const int nx = units_in_range(d, xcd, Ux, total_units);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, PT_REL_SCOPE);
            const int old =
                __hip_atomic_fetch_add(sync + xcd * kSyncLine, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool last = false;
            if (old == nx - 1) {
                int nranges = 0;
                for (int x = 0; x < 8; ++x) nranges += units_in_range(d, x, Ux, total_units) > 0;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, PT_ACQ_SCOPE);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, PT_REL_SCOPE);
                const int old2 =
                    __hip_atomic_fetch_add(sync + 16 * kSyncLine, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                last = old2 == nranges - 1;
                if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, PT_ACQ_SCOPE);
            }
            s_last = last;
        }
        __syncthreads();
        if (!s_last) return;
        de_step_body<false, true>(d, de_lds);
        __syncthreads();
        if (threadIdx.x < 8) __hip_atomic_store(sync + threadIdx.x * kSyncLine, 0, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        if (threadIdx.x == 8) __hip_atomic_store(sync + 16 * kSyncLine, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}


template <typename T, int S, int CPG, int MODE, bool SLOPE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_fit_persistent(
    const BlockDesc* __restrict__ descs, int nblk, int total_units, int steps, int resident,
    int* __restrict__ err, uint64_t spin_ticks) {
    __shared__ double lds[kPersistLds];
    __shared__ int s_ok, s_done, s_last;
    Cand* cs = reinterpret_cast<Cand*>(lds);
    double(*red)[kThreads] = reinterpret_cast<double(*)[kThreads]>(lds + 64);
    RotConst* rc = reinterpret_cast<RotConst*>(lds + 64 + kMaxCpg * kThreads);
    static_assert(64 + kMaxCpg * kThreads + kMaxCpg * sizeof(RotConst) / sizeof(double) <= kPersistLds,
                  "persistent kernel LDS holds the candidates, the lane sums and the phasor constants");

    const int G = gridDim.x, w = blockIdx.x;
    const int xcd = w & 7, k = w >> 3, Gx = G >> 3;
    const int Ux = (total_units + 7) >> 3;
    const int u_begin = xcd * Ux, u_end = min(total_units, u_begin + Ux);

    using V = typename std::conditional<MODE == 1, float, double>::type;
    V sv[S];
    bool full = true;
    int valid = S;
    if (resident && u_begin + k < u_end) {
        const int u = u_begin + k;
        const BlockDesc* d = descs + find_block(descs, nblk, u);
        load_lane<V, T, S>(d, (u - d->unit_begin) / d->ngroups, sv, full, valid);
    }

    // step s evaluates generation gen_begin + s of every block (the initial
    // population when that is 0)
    for (int step = 0; step < steps; ++step) {
        bool any = false;
        for (int u = u_begin + k; u < u_end; u += Gx) {
            const BlockDesc* __restrict__ d = descs + find_block(descs, nblk, u);
            const int g = d->gen_begin + step;
            if (g > d->max_gens) continue;
            const int local = u - d->unit_begin;
            const int tile = local / d->ngroups;
            const int group = local - tile * d->ngroups;
            int* sync = d->sync;
            __syncthreads();  // everyone is done with the shared flags of the last unit
            if (threadIdx.x == 0) {
                const bool ok = spin_until_ge(sync + (8 + xcd) * kSyncLine, g, err, spin_ticks);
                s_ok = ok;
                s_done = ok ? __hip_atomic_load(&d->st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1;
            }
            __syncthreads();
            if (!s_ok) return;
            if (s_done) continue;
            any = true;
            if (!resident) load_lane<V, T, S>(d, tile, sv, full, valid);
            unit_setup<S, CPG, MODE, SLOPE, true>(d, tile, group, cs, rc, d->trial);
            objective_unit<S, CPG, MODE, SLOPE>(d, tile, group, sv, full, valid, cs, rc, red, d->partials);
            // The workgroup barrier makes every wave's partial stores visible
            // at the XCD's L2; one release fence then publishes them device-wide
            // before the arrival is counted.  Arrivals are counted per XCD
            // range first, so no counter sees more than one XCD's workgroups.
            __syncthreads();
            if (threadIdx.x == 0) {
                // counters restart at every launch (k_de_init / k_sync_reset)
                const int done_steps = step + 1;
                const int nx = units_in_range(d, xcd, Ux, total_units);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, PT_REL_SCOPE);
                const int old = __hip_atomic_fetch_add(sync + xcd * kSyncLine, 1, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                bool last = false;
                if (old == nx * done_steps - 1) {
                    int nranges = 0;
                    for (int x = 0; x < 8; ++x) nranges += units_in_range(d, x, Ux, total_units) > 0;
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, PT_ACQ_SCOPE);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, PT_REL_SCOPE);
                    const int old2 = __hip_atomic_fetch_add(sync + 16 * kSyncLine, 1, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT);
                    last = old2 == nranges * done_steps - 1;
                    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, PT_ACQ_SCOPE);
                }
                s_last = last;
            }
            __syncthreads();
            if (s_last) {
                de_step_body<true, true>(d, lds);
                __syncthreads();
                if (threadIdx.x == 0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, PT_REL_SCOPE);
                    for (int x = 0; x < 8; ++x)
                        if (units_in_range(d, x, Ux, total_units) > 0)
                            __hip_atomic_store(sync + (8 + x) * kSyncLine, g + 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (!any) return;  // every block of this workgroup is done or past its cap
    }
}

// Restart the persistent kernel's per-launch counters of every block and
// set its ready copies to the generation the launch starts from.
#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ void k_sync_reset(const BlockDesc* __restrict__ descs) {
    const BlockDesc* d = descs + blockIdx.x;
    if (d->sync == nullptr) return;
    for (int k = threadIdx.x; k < kSyncInts; k += blockDim.x)
        d->sync[k] = (k >= 8 * kSyncLine && k < 16 * kSyncLine) ? d->gen_begin : 0;
}
#endif

// Initial population of the blocks flagged fresh (BlockDesc::fresh != 0);
// the others keep their running state.  Used by the serving loop.
#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ void k_de_init_fresh(const BlockDesc* __restrict__ descs) {
    const BlockDesc* d = descs + blockIdx.x;
    if (d->fresh) init_block(d);
}
#endif

// ---------------------------------------------------------------------------
// Final record of each block: best member, objective, generations, flags
// (adds AT_BOUND: an active non-phase coordinate within 1e-6 of its box
// width from a bound).
// ---------------------------------------------------------------------------
struct FitRecord {
    double x[kSlots];
    double f;
    int gens;
    int flags;
};

#ifndef PT_INSTANCE_TU  // (the instance translation units hold only templates)
__global__ void k_finalize(const BlockDesc* __restrict__ descs, FitRecord* __restrict__ out) {
    const BlockDesc* d = descs + blockIdx.x;
    // leading-step form: the final state is the slot whose stop flag is set
    DeState s = *d->st;
    if (d->st2 != nullptr && !s.done) s = *d->st2;
    const double* pop = s.slot ? d->pop2 : d->pop;
    if (s.slot) {
        // leave the final population in slot 0, where the host reads it
        for (int k = threadIdx.x; k < d->P * kStride; k += blockDim.x) d->pop[k] = pop[k];
        for (int k = threadIdx.x; k < d->P; k += blockDim.x) d->fpop[k] = d->fpop2[k];
    }
    if (threadIdx.x != 0) return;
    FitRecord r;
    const double* xb = pop + (size_t)s.best * kStride;
    int flags = s.flags;
    for (int j = 0; j < kSlots; ++j) r.x[j] = xb[j];
    for (int a = 0; a < d->D; ++a) {
        const int j = d->act[a];
        if (j == 1) continue;
        const double w = d->hi[j] - d->lo[j];
        if (xb[j] - d->lo[j] <= 1e-6 * w || d->hi[j] - xb[j] <= 1e-6 * w) flags |= 8;
    }
    r.f = s.best_f;
    r.gens = s.gen;
    r.flags = flags;
    out[blockIdx.x] = r;
}
#endif

}  // namespace pt
