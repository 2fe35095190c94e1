/*
 * oracle.h -- plain FP64 CPU oracle for the phase-tracking fit.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes,
 * links or calls this code; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark use it.  It shares no source with the
 * HIP path.
 *
 * What it computes (paper: "The GPU-based Phase Tracking method for
 * Planetary Radio Science applications", arXiv:1906.10598):
 *   - the signal model of Sec. 2.2, Eq. (2-2-1)..(2-2-3): a cubic Taylor
 *     phase around the block centre and an amplitude with optional slope;
 *   - the chi-square objective of Eq. (2-2-4) with unit weights;
 *   - the Differential Evolution fit of Sec. 1.2 / Table 4 as the classic
 *     DE/rand/1/bin scheme of Storn & Price (1997);
 *   - Philox4x32-10 from Salmon et al., SC'11, as the counter-based
 *     generator both sides draw their DE randomness from.
 *
 * Parameter slots (all FP64): 0 = A (amplitude, sample units),
 * 1 = phi0 [rad], 2 = f0 [Hz], 3 = f1 [Hz/s], 4 = f2 [Hz/s^2],
 * 5 = Adot (amplitude slope, sample units per second),
 * 6 = f3 [Hz/s^3], the fourth-order Taylor term of Sec. 3.2.1 (phase term
 *     2 pi f3 t^4 / 24; fixed at 0 for the cubic model).
 * Time of sample n: t_n = (n - ref) / fs seconds, ref in sample units.
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NSLOT 7

/* Random-stream tags (high 16 bits of the fourth counter word). */
#define ORC_TAG_INIT 1u
#define ORC_TAG_MUT 2u
#define ORC_TAG_XOVER 3u

/* Result flags. */
#define ORC_FLAG_CONVERGED 1
#define ORC_FLAG_MAXGEN 2
#define ORC_FLAG_VTR 4
#define ORC_FLAG_AT_BOUND 8

/* Philox4x32 with 10 rounds (Salmon et al. 2011). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Four words of the DE stream for (seed, stream, candidate i, generation g,
 * tag, call index). */
void orc_draw_words(uint64_t seed, uint64_t stream, uint32_t i, uint32_t g,
                    uint32_t tag, uint32_t call, uint32_t out[4]);

/* chi^2 = sum_n (s_n - (A + Adot t_n) cos(phi(t_n)))^2, Eq. (2-2-2)/(2-2-4),
 * phi(t) = phi0 + 2 pi (f0 t + f1 t^2/2 + f2 t^3/6 + f3 t^4/24) (Eq. 2-2-1 to
 * order 3, or 4 with slot 6), Neumaier-compensated, one candidate. */
double orc_chi2(const double* s, int64_t n, double fs, double ref, const double* x);

/* Correlation objective of Eq. (2-2-5) with the constant-amplitude model of
 * Eq. (2-2-6): F = 1 / (arctan(C) + pi/2), C = sum_n s_n (A + Adot t_n)
 * cos(phi(t_n)) -- the unnormalised correlation, which makes F tend to
 * 1/pi at the optimum as the paper states.  Neumaier-summed C. */
double orc_cor(const double* s, int64_t n, double fs, double ref, const double* x);

#define ORC_OBJ_CHI2 0
#define ORC_OBJ_COR 1

/* Objective of P candidates (row-major P x ORC_NSLOT); candidates in parallel with
 * nthreads OpenMP threads (<= 0: library default).  Each candidate's sum is
 * sequential, so the result does not depend on the thread count. */
void orc_chi2_pop(const double* s, int64_t n, double fs, double ref,
                  const double* pop, int P, double* out, int nthreads);

/* Objective `kind` (ORC_OBJ_CHI2 / ORC_OBJ_COR) of P candidates. */
void orc_obj_pop(int kind, const double* s, int64_t n, double fs, double ref,
                 const double* pop, int P, double* out, int nthreads);

/* Mutation indices and crossover uniforms of target i in generation g. */
void orc_de_draws(uint64_t seed, uint64_t stream, int g, int i, int P, int D,
                  int* r1, int* r2, int* r3, int* jrand, double* U /* D */);

/* One DE/rand/1/bin trial vector from explicit draws (all ORC_NSLOT slots;
 * act[0..D-1] lists the active slots in increasing order). */
void orc_de_trial(const double* pop, int i, int r1, int r2, int r3, int jrand,
                  const double* U, int D, const int* act, double F, double CR,
                  const double* lo, const double* hi, double* trial);

/* Initial population (P x ORC_NSLOT) inside the box. */
void orc_de_init(uint64_t seed, uint64_t stream, int P, const double* lo,
                 const double* hi, double* pop);

typedef struct {
    int P;            /* population size, >= 4 */
    int max_gens;     /* generation cap */
    double F, CR;     /* mutation scale, crossover rate */
    uint64_t seed;    /* Philox key */
    uint64_t stream;  /* per-block stream id (counter word) */
    double vtr;       /* stop when best <= vtr */
    double rel_tol;   /* > 0: window stop rule */
    int window;       /* window length W of the stop rule */
    double lo[ORC_NSLOT], hi[ORC_NSLOT];
    int objective;    /* ORC_OBJ_CHI2 or ORC_OBJ_COR */
} orc_de_cfg;

/* Full DE fit.  Outputs: best vector (ORC_NSLOT), best objective, generations run,
 * flags, final population (P x ORC_NSLOT, may be NULL), its objectives (P, may be
 * NULL), best-so-far history (max_gens + 1 entries, may be NULL).
 * Returns 0, or -1 on invalid arguments. */
int orc_de_fit(const double* s, int64_t n, double fs, double ref,
               const orc_de_cfg* cfg, int nthreads, double* best_x,
               double* best_f, int* gens, int* flags, double* pop_out,
               double* fpop_out, double* hist);

#ifdef __cplusplus
}
#endif
#endif
