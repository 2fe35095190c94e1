// device.h -- types and device helpers shared by the phase-tracking kernels.
//
// Notation follows Sec. 2.2 of arXiv:1906.10598: the phase of a candidate
// is phi(t) = phi0 + 2 pi (f0 t + f1 t^2 / 2 + f2 t^3 / 6) with t measured
// from the block's reference sample.  On the device the phase is carried in
// turns (phi / 2 pi) as a polynomial in the sample offset m = n - ref:
//     Phi(m) = a0 + a1 m + a2 m^2 + a3 m^3 + a4 m^4,
//     a0 = phi0 / 2 pi, a1 = f0 / fs, a2 = f1 / (2 fs^2), a3 = f2 / (6 fs^3),
//     a4 = f3 / (24 fs^4) (the fourth Taylor order of Sec. 3.2.1; 0 for a cubic),
// which is the same polynomial (Eq. 2-2-3 with c_i = 2 pi a_i fs^i).  Turns
// make the reduction to one period exact: r = Phi - rint(Phi).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cospoly.h"

namespace pt {

constexpr int kSlots = 7;        // A, phi0, f0, f1, f2, Adot, f3
constexpr int kStride = 8;       // doubles per population row (64-byte rows)
constexpr int kThreads = 256;    // objective workgroup size (4 wave64)
constexpr int kMaxCpg = 8;       // largest candidates-per-workgroup instantiated

// Per-block DE state, written only by the DE kernels.
struct DeState {
    int gen;       // generation of the population in `trial` (0 = initial); leading-step form:
                   // the generation the launch reading this slot evaluates; at a stop, the last
                   // generation selected
    int done;      // nonzero once the stop rule has fired
    int flags;     // PT_FLAG_* bits
    int best;      // index of the best member
    double best_f;
    int arrive;    // persistent kernel: work units finished, all generations
    int ready;     // persistent kernel: DE steps completed (trial of `ready` is set)
    int slot;      // population slot (0: pop / fpop, 1: pop2 / fpop2) of the selected population
    int pad;
    double old;    // leading-step form: best-so-far value the window rule of the next step compares with
};

// Everything a kernel needs to know about one block of a launch.
struct BlockDesc {
    const void* samples;
    int64_t n;
    double fs;
    double ref;
    int dtype;        // 0 = FP32, 1 = FP64
    int P;            // population size
    int D;            // active dimensions
    int ntiles;       // sample tiles of this block (objective kernel)
    int ngroups;      // candidate groups (objective kernel)
    int unit_begin;   // first objective work unit of this block
    int act[kSlots];  // active slots, increasing
    int window;
    int max_gens;
    int fresh;        // serving: the block's slot starts a new fit (k_de_init_fresh)
    double lo[kSlots];
    double hi[kSlots];
    double F, CR, vtr, rel_tol;
    uint64_t seed;
    uint64_t stream;
    double* pop;       // P x kStride, current population
    double* trial;     // P x kStride, population awaiting evaluation
    double* fpop;      // P
    double* partials;  // P x ntiles objective partial sums
    double* hist;      // max_gens + 1 best-so-far values
    DeState* st;       // may be null (bare objective evaluation)
    int* sync;         // persistent kernel: kSyncInts counters (see k_fit_persistent), or null
    int gen_begin;     // persistent kernel: generation whose trial is ready at launch; leading-step
                       // form: the block's launch index at the launch's first step (0 for a fit)
    int objective;     // 0 = chi-square (Eq. 2-2-4), 1 = correlation (Eq. 2-2-5)
    int quartic;       // nonzero: the phase has the fourth-order term f3 (slot 6)
    int amask;         // bit j set when slot j is active (the slots of act[0 .. D))
    // Leading-step launches (k_objective with fused >= 2) alternate between two
    // copies of the DE buffers: launch parity p reads the state of slot p and
    // the rows, objectives and partials of slot p ^ 1, and writes the others.
    // Slot 0 is pop / trial / fpop / partials / st, slot 1 these; null when
    // the fit does not use that form.
    double* pop2;
    double* trial2;
    double* fpop2;
    double* partials2;
    DeState* st2;
};

// Persistent-kernel synchronisation words of one block, one 128-byte line each:
// line x < 8: arrivals of the block's units in XCD range x; line 8 + x: copy of
// the block's ready generation polled by XCD range x; line 16: arrivals of
// XCD ranges.
constexpr int kSyncLine = 32;  // ints per 128-byte line
constexpr int kSyncInts = 17 * kSyncLine;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64 multiplies with the halves swapped and the key mixed in; the
// key is bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        U4 n;
        n.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        n.y = (uint32_t)p1;
        n.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        n.w = (uint32_t)p0;
        c = n;
    }
    return c;
}

enum : uint32_t { kTagInit = 1u, kTagMut = 2u, kTagXover = 3u };

// The fit's random stream: counter (member, generation, stream low word,
// tag << 16 | call), key (seed low word, seed high word ^ stream high word).
__device__ inline U4 draw4(uint64_t seed, uint64_t stream, uint32_t i, uint32_t g, uint32_t tag,
                           uint32_t call) {
    U4 c{i, g, (uint32_t)stream, (tag << 16) | call};
    return philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)(stream >> 32));
}

__device__ inline double unit_from(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
__device__ inline int index_from(uint32_t w, int m) {
    return (int)(((uint64_t)w * (uint64_t)m) >> 32);
}
__device__ inline uint32_t word(const U4& v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// cos(2 pi r) for |r| <= 1/2 as a polynomial in u = r^2 (coefficients from
// gen_cospoly.py).  FP64: degree 10; FP32: degree 6.
__device__ __forceinline__ double cos_turns64(double u) {
    double p = kCos64[0];
#pragma unroll
    for (int k = 1; k <= kCosDeg64; ++k) p = __fma_rn(p, u, kCos64[k]);
    return p;
}
__device__ __forceinline__ float cos_turns32(float u) {
    float p = kCos32[0];
#pragma unroll
    for (int k = 1; k <= kCosDeg32; ++k) p = __fmaf_rn(p, u, kCos32[k]);
    return p;
}

}  // namespace pt
