/*
 * oracle.c -- plain FP64 CPU oracle for the phase-tracking fit.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h): used by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product.
 *
 * Built with -ffp-contract=off so that the only fused multiply-adds are the
 * explicit fma() calls the DE conventions name.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2 by
 * the two round multipliers, swaps the halves and mixes in the key; the key
 * is advanced by the two Weyl constants between rounds.
 * ------------------------------------------------------------------------- */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Counter layout of the DE stream: (candidate, generation, stream low word,
 * tag << 16 | call); key = (seed low word, seed high word ^ stream high word). */
void orc_draw_words(uint64_t seed, uint64_t stream, uint32_t i, uint32_t g,
                    uint32_t tag, uint32_t call, uint32_t out[4]) {
    uint32_t ctr[4] = {i, g, (uint32_t)stream, (tag << 16) | call};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ (uint32_t)(stream >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Uniform in (0,1): (w + 1/2) / 2^32, exact in FP64. */
static double word_to_unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* Index in [0, m): floor(w * m / 2^32), integer arithmetic. */
static int word_to_index(uint32_t w, int m) { return (int)(((uint64_t)w * (uint64_t)m) >> 32); }

/* ---------------------------------------------------------------------------
 * Objective, Eq. (2-2-4) with sigma_i = 1, model Eq. (2-2-2):
 *   s(t) = (c4 + c5 t) cos(c0 + c1 t + c2 t^2 + c3 t^3)
 * with c0 = phi0, c1 = 2 pi f0, c2 = pi f1, c3 = pi f2 / 3 (Eq. 2-2-3), i.e.
 *   phi(t) = phi0 + 2 pi (f0 t + f1 t^2 / 2 + f2 t^3 / 6),
 * extended by the fourth-order term 2 pi f3 t^4 / 24 (Sec. 3.2.1, n = 4),
 * t measured from the block's reference sample (Sec. 2.2: phase origin at
 * the block centre).  The phase is evaluated directly in radians and the
 * cosine is the C library's.
 * ------------------------------------------------------------------------- */
double orc_chi2(const double* s, int64_t n, double fs, double ref, const double* x) {
    const double A = x[0], phi0 = x[1], f0 = x[2], f1 = x[3], f2 = x[4], Adot = x[5], f3 = x[6];
    const double two_pi = 2.0 * M_PI;
    double sum = 0.0, comp = 0.0; /* Neumaier */
    for (int64_t k = 0; k < n; ++k) {
        double t = ((double)k - ref) / fs;
        double turns = f0 * t + 0.5 * f1 * t * t + f2 * t * t * t / 6.0 + f3 * t * t * t * t / 24.0;
        double phi = phi0 + two_pi * turns;
        double model = (A + Adot * t) * cos(phi);
        double r = s[k] - model;
        double v = r * r;
        double tsum = sum + v;
        if (fabs(sum) >= fabs(v))
            comp += (sum - tsum) + v;
        else
            comp += (v - tsum) + sum;
        sum = tsum;
    }
    return sum + comp;
}

double orc_cor(const double* s, int64_t n, double fs, double ref, const double* x) {
    const double A = x[0], phi0 = x[1], f0 = x[2], f1 = x[3], f2 = x[4], Adot = x[5], f3 = x[6];
    const double two_pi = 2.0 * M_PI;
    double sum = 0.0, comp = 0.0; /* Neumaier */
    for (int64_t k = 0; k < n; ++k) {
        double t = ((double)k - ref) / fs;
        double turns = f0 * t + 0.5 * f1 * t * t + f2 * t * t * t / 6.0 + f3 * t * t * t * t / 24.0;
        double phi = phi0 + two_pi * turns;
        double v = s[k] * ((A + Adot * t) * cos(phi));
        double tsum = sum + v;
        if (fabs(sum) >= fabs(v))
            comp += (sum - tsum) + v;
        else
            comp += (v - tsum) + sum;
        sum = tsum;
    }
    return 1.0 / (atan(sum + comp) + 0.5 * M_PI);
}

void orc_obj_pop(int kind, const double* s, int64_t n, double fs, double ref,
                 const double* pop, int P, double* out, int nthreads) {
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int p = 0; p < P; ++p) {
        const double* x = pop + (size_t)p * ORC_NSLOT;
        out[p] = kind == ORC_OBJ_COR ? orc_cor(s, n, fs, ref, x) : orc_chi2(s, n, fs, ref, x);
    }
    (void)nthreads;
}

void orc_chi2_pop(const double* s, int64_t n, double fs, double ref,
                  const double* pop, int P, double* out, int nthreads) {
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int p = 0; p < P; ++p) out[p] = orc_chi2(s, n, fs, ref, pop + (size_t)p * ORC_NSLOT);
    (void)nthreads;
}

/* ---------------------------------------------------------------------------
 * DE/rand/1/bin (Storn & Price 1997), the scheme the paper's Sec. 1.2
 * describes (random initial population in the box, mutation, crossover,
 * selection), with F and CR as in Table 4.
 * ------------------------------------------------------------------------- */

/* Active slots: those whose box has lo < hi; lo == hi fixes the slot. */
static int active_slots(const double* lo, const double* hi, int* act) {
    int D = 0;
    for (int j = 0; j < ORC_NSLOT; ++j)
        if (lo[j] < hi[j]) act[D++] = j;
    return D;
}

void orc_de_init(uint64_t seed, uint64_t stream, int P, const double* lo,
                 const double* hi, double* pop) {
    int act[ORC_NSLOT];
    int D = active_slots(lo, hi, act);
    for (int i = 0; i < P; ++i) {
        double* x = pop + (size_t)i * ORC_NSLOT;
        for (int j = 0; j < ORC_NSLOT; ++j) x[j] = lo[j];
        uint32_t w[4];
        for (int a = 0; a < D; ++a) {
            if (a % 4 == 0) orc_draw_words(seed, stream, (uint32_t)i, 0u, ORC_TAG_INIT, (uint32_t)(a / 4), w);
            double u = word_to_unit(w[a % 4]);
            int j = act[a];
            x[j] = fma(u, hi[j] - lo[j], lo[j]);
        }
    }
}

void orc_de_draws(uint64_t seed, uint64_t stream, int g, int i, int P, int D,
                  int* r1, int* r2, int* r3, int* jrand, double* U) {
    uint32_t w[4];
    orc_draw_words(seed, stream, (uint32_t)i, (uint32_t)g, ORC_TAG_MUT, 0u, w);
    /* r1: uniform over the P-1 members other than i. */
    int a = word_to_index(w[0], P - 1);
    if (a >= i) ++a;
    /* r2: uniform over the P-2 members other than i and r1. */
    int lo2 = i < a ? i : a, hi2 = i < a ? a : i;
    int b = word_to_index(w[1], P - 2);
    if (b >= lo2) ++b;
    if (b >= hi2) ++b;
    /* r3: uniform over the P-3 members other than i, r1 and r2. */
    int e[3] = {i, a, b};
    for (int p = 0; p < 2; ++p)          /* sort the three exclusions */
        for (int q = 0; q < 2 - p; ++q)
            if (e[q] > e[q + 1]) { int t = e[q]; e[q] = e[q + 1]; e[q + 1] = t; }
    int c = word_to_index(w[2], P - 3);
    for (int p = 0; p < 3; ++p)
        if (c >= e[p]) ++c;
    *r1 = a; *r2 = b; *r3 = c;
    *jrand = word_to_index(w[3], D);
    for (int k = 0; k < D; ++k) {
        if (k % 4 == 0) orc_draw_words(seed, stream, (uint32_t)i, (uint32_t)g, ORC_TAG_XOVER, (uint32_t)(k / 4), w);
        U[k] = word_to_unit(w[k % 4]);
    }
}

void orc_de_trial(const double* pop, int i, int r1, int r2, int r3, int jrand,
                  const double* U, int D, const int* act, double F, double CR,
                  const double* lo, const double* hi, double* trial) {
    const double* xi = pop + (size_t)i * ORC_NSLOT;
    const double* x1 = pop + (size_t)r1 * ORC_NSLOT;
    const double* x2 = pop + (size_t)r2 * ORC_NSLOT;
    const double* x3 = pop + (size_t)r3 * ORC_NSLOT;
    for (int j = 0; j < ORC_NSLOT; ++j) trial[j] = xi[j];
    for (int a = 0; a < D; ++a) {
        int j = act[a];
        /* mutant: base x_r1 plus the scaled difference x_r2 - x_r3 */
        double v = fma(F, x2[j] - x3[j], x1[j]);
        /* a coordinate that leaves the box goes half-way from the base
         * vector to the violated bound */
        if (v < lo[j]) v = (lo[j] + x1[j]) * 0.5;
        if (v > hi[j]) v = (hi[j] + x1[j]) * 0.5;
        /* binomial crossover; coordinate jrand always comes from the mutant */
        if (U[a] < CR || a == jrand) trial[j] = v;
    }
}

int orc_de_fit(const double* s, int64_t n, double fs, double ref,
               const orc_de_cfg* cfg, int nthreads, double* best_x,
               double* best_f, int* gens, int* flags, double* pop_out,
               double* fpop_out, double* hist) {
    const int P = cfg->P;
    if (P < 4 || cfg->max_gens < 0 || n < 1 || !(fs > 0)) return -1;
    int act[ORC_NSLOT];
    int D = active_slots(cfg->lo, cfg->hi, act);
    if (D < 1) return -1;

    double* pop = (double*)malloc(sizeof(double) * (size_t)P * ORC_NSLOT);
    double* trial = (double*)malloc(sizeof(double) * (size_t)P * ORC_NSLOT);
    double* f = (double*)malloc(sizeof(double) * (size_t)P);
    double* ft = (double*)malloc(sizeof(double) * (size_t)P);
    double* h = (double*)malloc(sizeof(double) * (size_t)(cfg->max_gens + 1));

    orc_de_init(cfg->seed, cfg->stream, P, cfg->lo, cfg->hi, pop);
    orc_obj_pop(cfg->objective, s, n, fs, ref, pop, P, f, nthreads);

    int best = 0;
    for (int p = 1; p < P; ++p)
        if (f[p] < f[best]) best = p;
    h[0] = f[best];
    int g = 0, fl = 0;
    if (f[best] <= cfg->vtr) fl |= ORC_FLAG_VTR;

    while (!fl && g < cfg->max_gens) {
        ++g;
        /* all trials of generation g are built from the population of g-1 */
        for (int i = 0; i < P; ++i) {
            int r1, r2, r3, jr;
            double U[ORC_NSLOT];
            orc_de_draws(cfg->seed, cfg->stream, g, i, P, D, &r1, &r2, &r3, &jr, U);
            orc_de_trial(pop, i, r1, r2, r3, jr, U, D, act, cfg->F, cfg->CR,
                         cfg->lo, cfg->hi, trial + (size_t)i * ORC_NSLOT);
        }
        orc_obj_pop(cfg->objective, s, n, fs, ref, trial, P, ft, nthreads);
        /* selection: the trial replaces its target when it is not worse */
        for (int i = 0; i < P; ++i) {
            if (ft[i] <= f[i]) {
                memcpy(pop + (size_t)i * ORC_NSLOT, trial + (size_t)i * ORC_NSLOT, sizeof(double) * ORC_NSLOT);
                f[i] = ft[i];
            }
        }
        best = 0;
        for (int p = 1; p < P; ++p)
            if (f[p] < f[best]) best = p;
        h[g] = f[best];
        if (f[best] <= cfg->vtr) fl |= ORC_FLAG_VTR;
        if (cfg->rel_tol > 0 && cfg->window > 0 && g >= cfg->window &&
            h[g - cfg->window] - h[g] <= cfg->rel_tol * h[g])
            fl |= ORC_FLAG_CONVERGED;
    }
    if (!fl) fl |= ORC_FLAG_MAXGEN;

    /* best vector pinned at a bound of the box (phase slot excluded: its box
     * is a full turn) -- the failure mode of an under-sized range */
    const double* xb = pop + (size_t)best * ORC_NSLOT;
    for (int a = 0; a < D; ++a) {
        int j = act[a];
        if (j == 1) continue;
        double w = cfg->hi[j] - cfg->lo[j];
        if (xb[j] - cfg->lo[j] <= 1e-6 * w || cfg->hi[j] - xb[j] <= 1e-6 * w) fl |= ORC_FLAG_AT_BOUND;
    }

    memcpy(best_x, xb, sizeof(double) * ORC_NSLOT);
    *best_f = f[best];
    *gens = g;
    *flags = fl;
    if (pop_out) memcpy(pop_out, pop, sizeof(double) * (size_t)P * ORC_NSLOT);
    if (fpop_out) memcpy(fpop_out, f, sizeof(double) * (size_t)P);
    if (hist) {
        for (int k = 0; k <= cfg->max_gens; ++k) hist[k] = k <= g ? h[k] : NAN;
    }
    free(pop); free(trial); free(f); free(ft); free(h);
    return 0;
}
