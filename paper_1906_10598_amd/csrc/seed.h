// seed.h -- initial-range estimation of Sec. 3.1.1 on the device.
//
// The initial search box comes from short pieces of the block: the
// frequency at the block centre from the spectrum of a centred snippet, the
// frequency rate from a central difference of three equally spaced
// snippets, and the amplitude from the same spectrum.  One workgroup per
// snippet:
//   1. the M samples (M a power of two) go to LDS in bit-reversed order and
//      an in-place radix-2 decimation-in-time FFT runs there (log2 M stages,
//      one barrier each; twiddles from sincospi of the exact ratio j / half);
//   2. the peak bin k* maximises |X_k|^2 over 1 <= k < M/2 (lowest k on
//      ties) by a wave-shuffle + LDS argmax;
//   3. the frequency is refined between bins with Candan's bias-corrected
//      interpolator for a rectangular window (IEEE Signal Proc. Lett. 2011):
//      d = tan(pi/M)/(pi/M) * Re[(X_{k-1} - X_{k+1}) / (2 X_k - X_{k-1} - X_{k+1})];
//   4. the amplitude is 2 |sum_n x_n exp(-2 pi i f n / fs)| / M at the refined
//      frequency (phase in turns, exactly reduced), and the noise variance is
//      mean(x^2) - A^2 / 2.
// The estimates are per snippet; the host forms f0, f1, f2 and the box.
#pragma once

#include "device.h"

namespace pt {

constexpr int kSeedThreads = 1024;
constexpr int kSeedMaxLog = 13;  // M <= 8192 (128 KiB of FP64 complex LDS)

struct SeedSnippet {
    double f;      // Hz
    double amp;    // amplitude
    double noise;  // noise standard deviation
    int bin;       // peak bin k*
    int pad;
};

struct SeedStarts {
    int64_t v[3];  // first sample of each snippet
};

// (power, bin) order of the peak search: larger power, then lower bin.
__device__ __forceinline__ bool seed_better(double p, int k, double q, int m) {
    return p > q || (p == q && k < m);
}

template <typename T>
__global__ __launch_bounds__(kSeedThreads) void k_seed_spectrum(const T* __restrict__ s, SeedStarts starts,
                                                                int logM, double fs,
                                                                SeedSnippet* __restrict__ out) {
    extern __shared__ double lds[];
    const int M = 1 << logM;
    double* re = lds;
    double* im = lds + M;
    __shared__ double wp[kSeedThreads / 64];
    __shared__ int wk[kSeedThreads / 64];
    __shared__ double wsum[3][kSeedThreads / 64];
    __shared__ double fb;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const T* x = s + starts.v[blockIdx.x];

    for (int n = tid; n < M; n += blockDim.x) {
        const int r = (int)(__brev((unsigned)n) >> (32 - logM));
        re[r] = (double)x[n];
        im[r] = 0.0;
    }
    __syncthreads();
    for (int half = 1; half < M; half <<= 1) {
        for (int b = tid; b < (M >> 1); b += blockDim.x) {
            const int j = b & (half - 1);
            const int i0 = ((b - j) << 1) + j;
            const int i1 = i0 + half;
            double sn, cs;
            sincospi((double)j / (double)half, &sn, &cs);  // w = exp(-i pi j / half)
            const double r1 = re[i1], m1 = im[i1];
            const double tr = __fma_rn(cs, r1, sn * m1);
            const double ti = __fma_rn(cs, m1, -(sn * r1));
            const double r0 = re[i0], m0 = im[i0];
            re[i1] = r0 - tr;
            im[i1] = m0 - ti;
            re[i0] = r0 + tr;
            im[i0] = m0 + ti;
        }
        __syncthreads();
    }

    // peak bin
    double bp = -1.0;
    int bk = 0x7fffffff;
    for (int k = 1 + tid; k < (M >> 1); k += blockDim.x) {
        const double p = __fma_rn(re[k], re[k], im[k] * im[k]);
        if (seed_better(p, k, bp, bk)) {
            bp = p;
            bk = k;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double q = __shfl_xor(bp, o);
        const int m = __shfl_xor(bk, o);
        if (seed_better(q, m, bp, bk)) {
            bp = q;
            bk = m;
        }
    }
    if (lane == 0) {
        wp[wave] = bp;
        wk[wave] = bk;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < nwave; ++w)
            if (seed_better(wp[w], wk[w], bp, bk)) {
                bp = wp[w];
                bk = wk[w];
            }
        // (non-finite samples leave no candidate: fall back to bin 1, in range)
        const int k = (bk >= 1 && bk < (M >> 1)) ? bk : 1;
        // Candan's interpolator; X_{k-1} and X_{k+1} exist for 1 <= k < M/2
        const double nr = re[k - 1] - re[k + 1], ni = im[k - 1] - im[k + 1];
        const double dr = 2.0 * re[k] - re[k - 1] - re[k + 1], di = 2.0 * im[k] - im[k - 1] - im[k + 1];
        const double den = __fma_rn(dr, dr, di * di);
        double d = 0.0;
        if (den > 0.0) {
            const double c = M_PI / (double)M;
            d = tan(c) / c * (__fma_rn(nr, dr, ni * di) / den);
        }
        fb = ((double)k + d) * fs / (double)M;
        wk[0] = k;
    }
    __syncthreads();

    // amplitude at the refined frequency, and the snippet's power
    const double f = fb;
    const double nu = f / fs;  // turns per sample
    double yr = 0.0, yi = 0.0, ss = 0.0;
    for (int n = tid; n < M; n += blockDim.x) {
        const double v = (double)x[n];
        double q = nu * (double)n;
        q -= rint(q);
        double sn, cs;
        sincospi(2.0 * q, &sn, &cs);
        yr = __fma_rn(v, cs, yr);
        yi = __fma_rn(-v, sn, yi);
        ss = __fma_rn(v, v, ss);
    }
    for (int o = 32; o > 0; o >>= 1) {
        yr += __shfl_xor(yr, o);
        yi += __shfl_xor(yi, o);
        ss += __shfl_xor(ss, o);
    }
    if (lane == 0) {
        wsum[0][wave] = yr;
        wsum[1][wave] = yi;
        wsum[2][wave] = ss;
    }
    __syncthreads();
    if (tid == 0) {
        yr = yi = ss = 0.0;
        for (int w = 0; w < nwave; ++w) {
            yr += wsum[0][w];
            yi += wsum[1][w];
            ss += wsum[2][w];
        }
        const double A = 2.0 * sqrt(__fma_rn(yr, yr, yi * yi)) / (double)M;
        const double var = ss / (double)M - 0.5 * A * A;
        SeedSnippet o;
        o.f = f;
        o.amp = A;
        o.noise = var > 0.0 ? sqrt(var) : 0.0;
        o.bin = wk[0];
        o.pad = 0;
        out[blockIdx.x] = o;
    }
}

}  // namespace pt
