/*
 * phasetrack.h -- C ABI of the MI355X phase-tracking fit library
 * (libphasetrack.so).
 *
 * The library fits a block of real open-loop tracking samples s[n] to the
 * model of Sec. 2.2 of "The GPU-based Phase Tracking method for Planetary
 * Radio Science applications" (arXiv:1906.10598):
 *
 *     s(t) = (A + Adot t) cos(phi(t)),
 *     phi(t) = phi0 + 2 pi (f0 t + f1 t^2 / 2 + f2 t^3 / 6)          (Eq. 2-2-1..2-2-3)
 *              [+ 2 pi f3 t^4 / 24, the fourth Taylor order of Sec. 3.2.1]
 *
 * by minimising the unit-weight chi-square of Eq. (2-2-4) with Differential
 * Evolution (Sec. 1.2; control parameters of Table 4) in the DE/rand/1/bin
 * form.  Time is measured from a reference sample: t_n = (n - ref) / fs,
 * with ref = N / 2 (the block centre, Sec. 2.2) unless the caller gives one.
 * From the fitted phase it derives the observables of Sec. 3.1.3 and
 * Sec. 4: instantaneous phase and frequency (Eq. 3-1-1), border values
 * (Eq. 3-1-2), total-count phase and integration Doppler (Eq. 4-1-1,
 * 4-1-2) and line-of-sight acceleration (Eq. 4-2-1).
 *
 * Conventions shared by every entry point
 *   - Parameter vectors have PT_NSLOT = 7 FP64 slots in this order:
 *       0 A     amplitude, sample units
 *       1 phi0  phase at the reference sample [rad]
 *       2 f0    frequency [Hz]
 *       3 f1    frequency rate [Hz/s]
 *       4 f2    frequency acceleration [Hz/s^2]
 *       5 Adot  amplitude slope [sample units / s] (c5 of Eq. 2-2-2)
 *       6 f3    third frequency derivative [Hz/s^3]: the fourth-order phase
 *               term of Sec. 3.2.1 (perigee arcs); box [0, 0] for the cubic
 *     A slot whose box has lo == hi is fixed at lo and takes no part in the
 *     DE; the others are the active dimensions, in slot order.
 *   - Return value: PT_OK (0) or a negative pt_status.  No C++ exception
 *     and no abort crosses the ABI.  pt_last_error() returns a message for
 *     the last failure on the calling thread (static storage, valid until
 *     the next call on that thread).
 *   - Ownership: every pointer argument is caller-owned; the library never
 *     frees it and never keeps it after the call returns.  pt_ctx and
 *     pt_server objects are library-owned (create / destroy).
 *   - Device pointers are HIP device addresses on the context's device.
 *     hip_stream is a hipStream_t (NULL = the null stream); calls that take
 *     one enqueue their GPU work on it and return after the results they
 *     report have been copied back (they synchronise that stream).
 *   - A context is not thread-safe: one host thread at a time per pt_ctx.
 */
#ifndef PHASETRACK_H
#define PHASETRACK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PT_NSLOT 7
#define PT_MAX_POP 1024

typedef enum {
    PT_OK = 0,
    PT_EINVAL = -1,       /* invalid argument (message names it) */
    PT_ENOMEM = -2,       /* device or pinned-host allocation failed */
    PT_EDEVICE = -3,      /* HIP runtime error, or no usable device */
    PT_EBUSY = -4,        /* server: no slot / HBM budget for the block now */
    PT_EUNSUPPORTED = -5  /* valid request this build does not implement */
} pt_status;

typedef enum { PT_F32 = 0, PT_F64 = 1 } pt_dtype;

/* Objective (Sec. 2.2).  PT_OBJ_CHI2: unit-weight chi-square of Eq. (2-2-4)
 * over the model of Eq. (2-2-2).  PT_OBJ_COR: the correlation objective of
 * Eq. (2-2-5), F = 1 / (arctan(C) + pi/2) with the unnormalised correlation
 * C = sum_n s_n (A + Adot t_n) cos phi(t_n) over the constant-amplitude model
 * of Eq. (2-2-6) (fix A with lo == hi); F tends to 1/pi at the optimum. */
typedef enum { PT_OBJ_CHI2 = 0, PT_OBJ_COR = 1 } pt_objective_kind;

/* Arithmetic of the objective.  PT_PREC_FP64: phase, cosine, residual and
 * sums in FP64.  PT_PREC_MIXED: FP64 per-chunk phase anchor, FP32 local
 * phase offset (compensated), FP32 cosine and residual, FP32 chunk sums,
 * FP64 cross-chunk sum; DE selection compares FP64 values in both modes. */
typedef enum { PT_PREC_FP64 = 0, PT_PREC_MIXED = 1 } pt_precision;

/* pt_fit.flags bits.  CONVERGED: the window stop rule was met; MAXGEN: the
 * generation cap ended the fit; VTR: best <= vtr; AT_BOUND: an active
 * non-phase coordinate of the best member lies within 1e-6 of its box
 * width from a bound -- the signature of a search range that misses the
 * truth (Sec. 3.1.1). */
enum { PT_FLAG_CONVERGED = 1, PT_FLAG_MAXGEN = 2, PT_FLAG_VTR = 4, PT_FLAG_AT_BOUND = 8 };

typedef struct pt_ctx pt_ctx;

/* Search box (XCmin / XCmax of Table 4), per slot. */
typedef struct {
    double lo[PT_NSLOT];
    double hi[PT_NSLOT];
} pt_box;

/* DE control parameters (Table 4) and stop rule (Sec. 3.1.2).
 *   pop       population size P, 4 <= P <= PT_MAX_POP
 *   max_gens  generation cap (itermax), >= 0
 *   F         mutation scale, 0 < F <= 2
 *   CR        crossover rate, 0 <= CR <= 1
 *   seed      Philox4x32-10 key of the fit's random stream
 *   vtr       stop as soon as the best objective is <= vtr (-inf: never)
 *   rel_tol   > 0 selects the window rule: stop after generation g >= window
 *             when best[g - window] - best[g] <= rel_tol * best[g];
 *             <= 0: run exactly max_gens generations (fixed iteration
 *             count, the paper's production choice)
 *   window    window length W of that rule (>= 1 when rel_tol > 0)
 *   precision pt_precision
 *   objective pt_objective_kind */
typedef struct {
    int32_t pop;
    int32_t max_gens;
    double F;
    double CR;
    uint64_t seed;
    double vtr;
    double rel_tol;
    int32_t window;
    int32_t precision;
    int32_t objective;  /* pt_objective_kind */
    int32_t reserved;   /* 0 */
} pt_de_settings;

/* One block of samples.
 *   samples   n samples of type dtype; device pointer when on_device != 0,
 *             else host pointer (copied to the device by the call)
 *   n         number of samples, >= 8
 *   fs        sample rate [Hz], > 0
 *   ref       reference sample (time origin) in sample units; NaN selects
 *             n / 2, the block centre
 *   stream    id of the block's DE random stream (Philox counter word 2 and
 *             high key word); give each (track, block) its own
 *   box       search box */
typedef struct {
    const void* samples;
    int64_t n;
    int32_t dtype;
    int32_t on_device;
    double fs;
    double ref;
    uint64_t stream;
    pt_box box;
} pt_block;

/* Result of one block fit, with the per-block output record of the
 * paper's Appendix 1.
 *   coef         best member (PT_NSLOT slots, as found inside the box)
 *   objective    chi-square at coef (RSS)
 *   generations  generations run after the initial population
 *   flags        PT_FLAG_* bits
 *   ref          reference sample used
 *   t_left, t_right   block borders relative to the reference [s]:
 *                (0 - ref) / fs and (n - ref) / fs
 *   phase_centre phi(0) mod 2 pi [rad] (c0 of Appendix 1)
 *   phase_left, phase_right  phi at the borders, mod 2 pi [rad] (Eq. 3-1-2)
 *   freq_left, freq_right    instantaneous frequency at the borders [Hz]
 *   total_phase  phi(t_right) - phi(t_left) [rad] (Eq. 4-1-2 term) */
typedef struct {
    double coef[PT_NSLOT];
    double objective;
    int32_t generations;
    int32_t flags;
    double ref;
    double t_left, t_right;
    double phase_centre;
    double phase_left, phase_right;
    double freq_left, freq_right;
    double total_phase;
} pt_fit;

/* Library version (major * 10000 + minor * 100 + patch). */
int pt_version(void);

/* Message of the calling thread's last failure ("" if none). */
const char* pt_last_error(void);

/* Create a context on HIP device `device`; it owns the device buffers,
 * cached launch graphs and tuning data of its fits.  PT_EDEVICE when the
 * device does not exist or is not a gfx950 part. */
int pt_ctx_create(int device, pt_ctx** out);

/* Destroy a context and free everything it owns (NULL is ignored). */
void pt_ctx_destroy(pt_ctx* ctx);

/* Fit one block (Sec. 2.2 problem statement; Sec. 1.2 / Table 4 DE).
 * The whole fit -- initial population, every generation's objective,
 * mutation, crossover, selection and the stop rule -- runs on the device;
 * the host reads back only the final record.  Returns after `out` is
 * filled.  The fit is deterministic for a given (seed, block.stream). */
int pt_fit_block(pt_ctx* ctx, const pt_block* block, const pt_de_settings* de,
                 void* hip_stream, pt_fit* out);

/* Fit nblk independent blocks of possibly different lengths, each with its
 * own population and stream, with the same DE settings, in shared device
 * launches (one objective grid over every block's samples x population per
 * generation).  out[b] equals what pt_fit_block gives for block b alone
 * (same kernels, same reduction order).  1 <= nblk <= 4096. */
int pt_fit_batch(pt_ctx* ctx, const pt_block* blocks, int nblk, const pt_de_settings* de,
                 void* hip_stream, pt_fit* out);

/* Objective of an arbitrary population, for parity checks (Eq. 2-2-4 or
 * Eq. 2-2-5).
 *   pop       device pointer, P x PT_NSLOT FP64, row-major
 *   out       device pointer, P FP64
 *   precision pt_precision; objective pt_objective_kind */
int pt_objective(pt_ctx* ctx, const pt_block* block, const double* pop, int P,
                 int precision, int objective, void* hip_stream, double* out);

/* Bytes of the fixed device array pt_objective_noalloc works in: one copy per
 * device the library runs on, held until the process ends. */
#define PT_NOALLOC_SCRATCH_BYTES (4u << 20)

/* pt_objective for callers that cannot allocate: it calls no hipMalloc,
 * hipFree or other allocating routine (tight serving loops, harnesses that
 * forbid device allocation).  Arguments, results and the arithmetic are those
 * of pt_objective (same kernels, same geometry, bit-identical outputs); the
 * caller still owns pop and out.
 *   - The descriptor, the packed rows and the P x ceil(n / (256 S)) tile
 *     partial sums (S = samples per lane of the chosen geometry) live in the
 *     library's fixed array of PT_NOALLOC_SCRATCH_BYTES bytes; a call that
 *     needs more (roughly P x n > 2e9 samples at 16 samples per lane) fails with
 *     PT_EINVAL and a message giving the size it needed.
 *   - block.samples must be a device pointer (on_device = 1), else PT_EINVAL.
 *   - Every call on one device uses that device's single array, which keeps
 *     the last call's contents (every word a call reads it writes first).
 *     Calls that overlap on one device -- from two host threads, or two
 *     streams -- race on it and must be serialised by the caller.
 *   - Returns after out is written (the stream is synchronised), as
 *     pt_objective does; it cannot be captured into a HIP graph. */
int pt_objective_noalloc(pt_ctx* ctx, const pt_block* block, const double* pop, int P,
                         int precision, int objective, void* hip_stream, double* out);

/* Final population and objectives of block `index` of the context's most
 * recent pt_fit_block / pt_fit_batch call.  pop_host: P x PT_NSLOT FP64; fpop_host:
 * P FP64 (either may be NULL); P must equal that call's population size. */
int pt_last_population(pt_ctx* ctx, int index, double* pop_host, double* fpop_host, int P);

/* Best-so-far objective after each generation 0..generations of block
 * `index` of the most recent fit; copies min(n, generations + 1) values to
 * hist_host and stores that count in *count. */
int pt_last_history(pt_ctx* ctx, int index, double* hist_host, int n, int* count);

/* ---- derived observables (host FP64; t is seconds from the fit's
 * reference sample) ---- */

/* Instantaneous phase and frequency at n time tags (Eq. 3-1-1).  Outputs
 * (each may be NULL): phase [rad], phase mod 2 pi [rad], frequency [Hz],
 * frequency rate [Hz/s]. */
int pt_phase(const pt_fit* fit, const double* t, int64_t n, double* phase,
             double* phase_mod2pi, double* freq_hz, double* fdot_hz_s);

/* Phase change phi(t_end) - phi(t_start) inside one block (Eq. 4-1-1
 * numerator) and the corresponding integration Doppler [rad/s]. */
int pt_total_phase(const pt_fit* fit, double t_start, double t_end, double* dphi_rad,
                   double* f_int_rad_s);

/* Phase connection over nblk contiguous blocks (Eq. 4-1-2): Phi_total =
 * sum_i [phi_i(t_right) - phi_i(t_left)], count interval T_c = sum of the
 * block lengths, F_int_dop = Phi_total / T_c [rad/s]. */
int pt_connect_phase(const pt_fit* fits, int nblk, double* phi_total_rad, double* f_int_rad_s);

/* Line-of-sight acceleration at time t from phi''(t) (Eq. 4-2-1):
 * a = phi'' c / (2 pi f_carrier) one-way (three_way == 0) or
 * a = phi'' c / (4 pi M2 f_carrier) three-way; f_carrier [Hz] is the sky
 * carrier, M2 the transponder ratio. */
int pt_los_accel(const pt_fit* fit, double t, double f_carrier_hz, double M2, int three_way,
                 double* a_m_s2);

/* ---- range determination and continuity (Sec. 3.1.1, Sec. 3.1.3) ---- */

/* Options of pt_seed_block.
 *   snippet  M, samples per snippet: a power of two in [64, pt_seed_max_snippet()];
 *            0 selects 4096 (or the maximum, if smaller)
 *   spacing  samples between the middle snippet's centre and each outer one;
 *            0 selects n / 4 */
typedef struct {
    int32_t snippet;
    int32_t reserved;  /* 0 */
    int64_t spacing;
} pt_seed_opts;

/* Estimates of pt_seed_block.  Snippet k (0 = left, 1 = middle, 2 = right)
 * holds samples [c_k - M/2, c_k + M/2) with c_k = floor(ref) + (k - 1) spacing;
 * t[k] is the mid-time of its samples, seconds from the reference sample.
 * A real signal shows |frequency|: f[k] lies in (0, fs/2), so for a negative
 * carrier offset the estimates describe the mirror-image phase (phi0, f0,
 * f1, f2) -> (-phi0, -f0, -f1, -f2), which gives the same samples.
 * Standard errors: single-tone Cramer-Rao bound with the measured noise,
 * sd_f = sqrt(6) sigma / (pi A T_s sqrt(M)), T_s = M / fs, propagated
 * through the difference formulas. */
typedef struct {
    double f[3];      /* peak frequency of each snippet [Hz] */
    double amp[3];    /* amplitude of each snippet at f[k] */
    double noise[3];  /* noise standard deviation of each snippet */
    double t[3];      /* [s] */
    int32_t bin[3];   /* FFT peak bin of each snippet */
    int32_t snippet;  /* M used */
    double f0;        /* f[1] moved to the reference time with f1 [Hz] */
    double f1;        /* (f[2] - f[0]) / (t[2] - t[0]) [Hz/s] */
    double f2;        /* (f[2] - 2 f[1] + f[0]) / dt^2, dt = spacing / fs [Hz/s^2] */
    double A, sigma;  /* amplitude and noise std of the middle snippet */
    double sd_f0, sd_f1, sd_f2, sd_A;
} pt_seed;

/* Largest snippet pt_seed_block accepts on the context's device (limited by
 * the LDS one workgroup may hold: 16 bytes per sample). */
int pt_seed_max_snippet(pt_ctx* ctx);

/* Initial-range estimates of Sec. 3.1.1 for one block: each of three
 * equally spaced snippets is transformed by an FFT on the device, its peak
 * bin refined by Candan's interpolator and its amplitude measured at the
 * refined frequency; the host then forms f0, f1 (central difference) and f2
 * (second difference).  The block's box is not used.  Errors: PT_EINVAL
 * for a bad block or options, or a snippet reaching outside the block.
 * Returns after `out` is filled (synchronises hip_stream). */
int pt_seed_block(pt_ctx* ctx, const pt_block* block, const pt_seed_opts* opts, void* hip_stream,
                  pt_seed* out);

/* Box rules of pt_seed_box.
 * PT_RANGE_PAPER, Sec. 3.1.1 as printed: phi0 in [0, 2 pi]; f0 +-10 % of
 *   |f0|; f1 +-10 % of |f1| (the paper gives the value only; it is widened
 *   to at least nsig sd_f1); f2 in +-150/pi Hz/s^2 (c3 in [-50, 50] rad/s^3);
 *   A +-10 %; Adot in +-0.2 A / T when `slope`, else fixed at 0.
 * PT_RANGE_SIGMA: phi0 in [0, 2 pi]; f0, f1, f2 each +-nsig standard errors
 *   around the estimate; A +-max(10 %, nsig sd_A); Adot as above.  This is the
 *   default of the server's seeding: a 10 % frequency range is thousands of
 *   chi-square peak widths (1 / T) for a kHz carrier, beyond what a 40-member
 *   population finds. */
enum { PT_RANGE_PAPER = 0, PT_RANGE_SIGMA = 1 };

/* Search box from seed estimates; T is the block length [s] (n / fs). */
int pt_seed_box(const pt_seed* seed, int rule, double nsig, double T, int slope, pt_box* out);

/* Phase continuity at the border of two adjacent blocks (Eq. 3-1-2): block
 * `a` ends where block `b` starts.  dphi = phi_a(a.t_right) - phi_b(b.t_left)
 * wrapped to [-pi, pi] [rad]; dfreq = F_a(a.t_right) - F_b(b.t_left) [Hz]. */
int pt_continuity(const pt_fit* a, const pt_fit* b, double* dphi_rad, double* dfreq_hz);

/* ---- serving: continuous batching of arriving blocks ----
 * A server keeps up to max_slots blocks resident on the device (samples,
 * population, partial sums and DE state of each).  pt_server_step runs
 * gens_per_step generations of every resident block in shared launches (one
 * objective grid per objective arithmetic over the resident blocks, then
 * each block's DE step), then retires the blocks whose stop rule fired;
 * blocks submitted meanwhile are admitted at the start of the next step as
 * slots and the HBM budget free up.
 *
 * A track's blocks are contiguous in time and fitted in submission order,
 * which makes the server a tracker (Sec. 3.1.1, 3.1.3):
 *   - first block: its own box, or (seed_first) a box from pt_seed_block on
 *     its samples with PT_RANGE_SIGMA and seed_nsig standard errors; slots the
 *     given box fixes stay fixed;
 *   - later blocks start warm from the track's last accepted fit, whose phase
 *     is re-expanded about the new block's reference time.  range_rule
 *     PT_RUN_WARM: the block's own box half-widths times warm_narrow around
 *     that prediction.  PT_RUN_EXTRAPOLATE (the running range of Sec. 3.1.1):
 *     f0 spans the previous fit's frequency from the new block's start to its
 *     end, f1 likewise its frequency rate, each widened to at least
 *     warm_narrow times the block's own half-width; A is the prediction +-10 %;
 *     phi0, f2 and Adot as PT_RUN_WARM;
 *   - with max_attempts > 1 or a continuity limit set, a fit fails when its
 *     best member sits on a bound of A, f0 or f1 (the range missed the
 *     signal; f2 and Adot of short blocks are noise-dominated and may sit on
 *     their bounds, which only sets PT_FLAG_AT_BOUND) or, when qc_phase_rad /
 *     qc_freq_hz are set and the track's previous block was accepted, when
 *     the border phase or frequency jump (pt_continuity) exceeds them.  A
 *     failed block is fitted again with every half-width times `enlarge`
 *     (the phase one capped at pi), up to max_attempts fits in all; after the
 *     last it is delivered with PT_FLAG_ABANDONED (and PT_FLAG_DISCONTINUOUS
 *     when continuity failed), and the track's next block is predicted from
 *     the last accepted fit.  Otherwise every fit is accepted as it is.
 * A block's arithmetic (mixed, FP64 phasor or FP64 per-sample) follows from
 * its own box, and every block uses the same DE settings and geometry, so a
 * block's result does not depend on which other blocks share its steps. */
typedef struct pt_server pt_server;

enum { PT_RUN_WARM = 0, PT_RUN_EXTRAPOLATE = 1 };
enum { PT_FLAG_ABANDONED = 16, PT_FLAG_DISCONTINUOUS = 32 };

typedef struct {
    int32_t max_slots;          /* resident blocks, 1..1024 */
    int32_t gens_per_step;      /* generations per scheduler step, >= 1 */
    int32_t max_pending;        /* queued (not yet admitted) blocks, >= 1 */
    int32_t spl, cpg;           /* objective geometry; 0, 0 = default for 400K samples */
    int32_t range_rule;         /* PT_RUN_WARM or PT_RUN_EXTRAPOLATE */
    double warm_narrow;         /* box scale of warm starts, 0 (no warm start) .. 1 */
    uint64_t hbm_budget_bytes;  /* device bytes resident blocks may hold; a block of n samples
                                   holds n * sizeof(sample) + (max_gens + 1) * 8 + 2 * (P * 136 +
                                   P * ntiles * 8 + 48), ntiles = ceil(n / (256 * spl)): samples,
                                   history and two slots of rows, objectives, partials and state */
    pt_de_settings de;          /* settings of every block (pop <= 256) */
    int32_t seed_first;         /* 1: seed each track's first box from its samples */
    int32_t seed_snippet;       /* pt_seed_opts.snippet (0 = default) */
    double seed_nsig;           /* standard errors per seeded half-width (> 0) */
    int32_t max_attempts;       /* fits per block, 1..16 (0 = 1: no retry) */
    int32_t reserved;           /* 0 */
    double enlarge;             /* half-width factor per retry (>= 1) */
    double qc_phase_rad;        /* continuity limit on the border phase jump; 0 = off */
    double qc_freq_hz;          /* continuity limit on the border frequency jump; 0 = off */
} pt_server_config;

typedef struct {
    uint64_t ticket;            /* from pt_server_submit */
    int32_t track;
    int32_t warm;               /* 0: given box, 1: warm start, 2: seeded from its samples */
    double t_submit, t_done;    /* seconds on the server clock */
    pt_box box;                 /* search box of the delivered fit */
    pt_fit fit;
    int32_t attempts;           /* fits run for this block */
    int32_t qc;                 /* continuity check: 0 not made, 1 passed, -1 failed */
    double border_dphi;         /* pt_continuity against the previous block, when qc != 0 */
    double border_dfreq;
} pt_server_result;

/* Create a server on ctx.  Its generations run as objective + DE step
 * launches, or, when the context's step fusion is PT_FUSION_LEAD at this
 * call (and pop <= 256), as one leading-step launch per generation for every
 * resident block; the choice holds for the server's lifetime.  Both give
 * bit-identical fits. */
int pt_server_create(pt_ctx* ctx, const pt_server_config* cfg, pt_server** out);

/* Destroy a server (its queued and running blocks are dropped). */
void pt_server_destroy(pt_server* srv);

/* Queue a block of `track` (samples copied by the call, host or device).
 * PT_EBUSY when max_pending blocks are already queued; PT_EINVAL when the
 * block alone exceeds the HBM budget, or, with seed_first, when it is too
 * short for the three seeding snippets. */
int pt_server_submit(pt_server* srv, int32_t track, const pt_block* block, uint64_t* ticket);

/* One scheduler step on hip_stream (admit, run gens_per_step generations,
 * retire); returns after the step's results are queued.  n_active: blocks
 * still running afterwards; n_pending: blocks still queued. */
int pt_server_step(pt_server* srv, void* hip_stream, int32_t* n_active, int32_t* n_pending);

/* Move up to max finished results to out (oldest first). */
int pt_server_poll(pt_server* srv, pt_server_result* out, int32_t max, int32_t* n_out);

/* Resident blocks, queued blocks and budgeted device bytes in use. */
int pt_server_stats(pt_server* srv, int32_t* active, int32_t* pending, uint64_t* used_bytes);

/* Seconds since the server was created (monotonic host clock). */
double pt_server_clock(pt_server* srv);

/* ---- launch strategy ---- */

/* How a fit's generations are launched.
 *   PT_LAUNCH_PERSISTENT: one cooperative grid runs every generation of
 *     every block; workgroups keep their sample chunks in registers, and the
 *     workgroup that completes a block's generation runs its DE step (no
 *     grid-wide barrier, no per-generation launches).  Needs P <= 256 and a
 *     grid that fits on the device at once.
 *   PT_LAUNCH_GRAPH: per generation one objective launch and one DE-step
 *     launch (or one launch with the step fused, see pt_ctx_set_step_fusion),
 *     replayed from captured HIP graphs of 50 generations (250 for fits
 *     without a window rule).
 *   PT_LAUNCH_AUTO (default): graph.  On MI355X the per-block barrier of
 *     the persistent grid costs about as much as graph-replayed launches,
 *     which run back to back, so the graph path is the faster default.
 * Both give bit-identical results for the same geometry. */
enum { PT_LAUNCH_AUTO = 0, PT_LAUNCH_GRAPH = 1, PT_LAUNCH_PERSISTENT = 2 };

int pt_ctx_set_launch_mode(pt_ctx* ctx, int mode);

/* Launch strategy the context's most recent fit used (PT_LAUNCH_GRAPH or
 * PT_LAUNCH_PERSISTENT). */
int pt_ctx_last_launch(pt_ctx* ctx, int* mode);

/* ---- FP64 objective arithmetic ----
 * PT_FP64_AUTO (default): inside each lane's chunk of S samples the phasor
 *   exp(2 pi i Phi) follows from an exact FP64 anchor by a three-term
 *   recurrence for the linear phase and a first-order correction for the
 *   quadratic one (five operations per sample), wherever that is accurate to
 *   2e-11 per sample for the whole box: the dropped cubic and quartic terms
 *   below 1e-12 turns, the quadratic correction's error below 1e-11, and
 *   the carrier at least S * 2.2e-4 / (2 pi) of fs away from 0 and fs / 2
 *   (the recurrence's conditioning); otherwise the per-sample path.  The
 *   choice is made per block: in a graph-launched batch the blocks that
 *   qualify and those that do not run as two objective launches per
 *   generation (a persistent launch uses the per-sample path for all when
 *   any block needs it).
 * PT_FP64_POLY: always the per-sample path (exact reduction of the phase in
 *   turns, degree-10 cosine polynomial). */
enum { PT_FP64_AUTO = 0, PT_FP64_POLY = 1 };

int pt_ctx_set_fp64_method(pt_ctx* ctx, int method);

/* ---- step fusion ----
 * How a fit's generations map onto launches (graph-replayed fits; the DE
 * step is that of Table 4, DE/rand/1/bin, in every form):
 * PT_FUSION_AUTO (default): PT_FUSION_LEAD when the launch's work units fit
 *   in two rounds of resident workgroups (the kernel's occupancy times the
 *   compute units: a latency-bound fit, such as one paper-scale block) and
 *   max_gens <= 20000 (the leading form keeps one captured graph per 50
 *   generations), else PT_FUSION_LAST
 *   (a throughput-bound batch, where the leading step's repeated work costs
 *   more than the last workgroup's wait).
 * PT_FUSION_LEAD (P <= 256): one launch per generation.  Every
 *   objective workgroup first repeats the previous generation's DE step for
 *   itself (objectives of all P trials from the tile partials, selection,
 *   best member, stop rule) and draws the trials of its own candidates; the
 *   workgroup of the block's first work unit stores the step.  Nothing waits
 *   and nothing is read in the launch that writes it (two buffer slots
 *   alternate by launch parity).  One extra launch runs the last step.
 * PT_FUSION_LAST (P <= 256): one launch per generation; the DE step runs
 *   once, in the objective workgroup that finishes the block's last work
 *   unit (arrival counters, no waiting).
 * PT_FUSION_OFF: objective and DE step as two launches.
 * All three give bit-identical fits.  Returns PT_EINVAL for another value. */
enum { PT_FUSION_OFF = 0, PT_FUSION_LEAD = 1, PT_FUSION_LAST = 2, PT_FUSION_AUTO = 3 };

int pt_ctx_set_step_fusion(pt_ctx* ctx, int mode);

/* Objective arithmetic of the context's most recent fit or objective
 * evaluation: per-sample FP64 cosine, mixed precision, or FP64 phasor (also
 * for a batch whose blocks used both FP64 arithmetics). */
enum { PT_ARITH_FP64_POLY = 0, PT_ARITH_MIXED = 1, PT_ARITH_FP64_PHASOR = 2 };

int pt_ctx_last_arithmetic(pt_ctx* ctx, int* arith);

/* Chunk geometry (samples per lane, candidates per workgroup) of the
 * context's most recent fit or objective evaluation; 0, 0 before the first.
 * PT_EINVAL on null arguments. */
int pt_ctx_last_geometry(pt_ctx* ctx, int* samples_per_lane, int* cand_per_group);

/* Objective-kernel launches of the context's most recent fit (all blocks of
 * a batch share them): one per generation including generation 0, plus one
 * for the last DE step in the leading-step form; 1 for a persistent launch.
 * A fit that stopped early by the window rule may have run fewer. */
int pt_ctx_last_fit_launches(pt_ctx* ctx, int64_t* launches);

/* ---- instrumentation ---- */

/* Turn per-kernel timing of the objective kernel on (1) or off (0).  While
 * on, fits launch kernels one by one (no graph replay), each generation as
 * the objective alone and then the DE step whatever the step-fusion
 * setting, and bracket every objective launch with HIP events on the fit's
 * stream; results are bit-identical to those of the other forms. */
int pt_ctx_set_timing(pt_ctx* ctx, int on);

/* Launch count and summed duration [ms] of objective-kernel launches timed
 * since timing was turned on. */
int pt_ctx_kernel_stats(pt_ctx* ctx, int64_t* launches, double* total_ms);

/* Time `reps` back-to-back launches of the objective kernel alone on the
 * population `pop` (device, P x PT_NSLOT) with HIP events on hip_stream; *avg_ms
 * receives the mean duration of one launch.  Same kernel, geometry and
 * grid as a fit of this block uses. */
int pt_time_objective(pt_ctx* ctx, const pt_block* block, const double* pop, int P, int precision, int reps,
                      void* hip_stream, double* avg_ms);

/* Chunk geometry of the objective kernel used for blocks of n samples and
 * population P in the given precision: samples per lane and candidates per
 * workgroup (the autotuner's choice once it has run).  It applies to single
 * blocks and to batches up to four work units per compute unit; a larger
 * batch (throughput-bound) uses the geometry with the most candidate·samples
 * per lane instead (32 x 8 for P = 40), unless pt_ctx_set_tile forces one. */
int pt_ctx_get_tile(pt_ctx* ctx, int64_t n, int P, int precision, int* samples_per_lane,
                    int* cand_per_group);

/* Force a chunk geometry for every later fit in this context (0, 0 = back
 * to the tuned/default choice).  Supported samples_per_lane: 4, 8, 16, 32;
 * cand_per_group: 1, 2, 4, 8. */
int pt_ctx_set_tile(pt_ctx* ctx, int samples_per_lane, int cand_per_group);

/* Time every supported geometry on a block of n samples and population P:
 * short fits of 100 generations in the context's current launch form and
 * step fusion, on synthetic data on the device in a box of the paper's
 * widths around one carrier at the largest drift rate and drift
 * acceleration of the paper-scale synthetic blocks (5 Hz/s, 0.05 Hz/s^2),
 * so that each geometry is timed with the FP64 arithmetic it would use at
 * the edge of such a box.  Remembers the fastest for that size class
 * (floor(log2 n)) and precision, for single blocks and small batches;
 * replaces the context's last-fit record (pt_last_population).
 * best_spl / best_cpg may be NULL. */
int pt_ctx_autotune(pt_ctx* ctx, int64_t n, int P, int precision, void* hip_stream,
                    int* best_spl, int* best_cpg);

#ifdef __cplusplus
}
#endif
#endif /* PHASETRACK_H */
