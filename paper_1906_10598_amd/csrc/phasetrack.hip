// phasetrack.hip -- host runtime and C ABI of libphasetrack.so (gfx950).
//
// The runtime owns device buffers per context, plans the objective grid of
// a launch (units of (block, sample tile, candidate group)), captures chunks
// of DE generations into HIP graphs and replays them, and turns the final
// device records into the per-block output of the paper's Appendix 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/phasetrack.h"
#include "instances.h"
#include "kernels.h"
#include "seed.h"

using namespace pt;

// Device memory of pt_objective_noalloc: the block descriptor, the packed
// population rows and the tile partial sums of one call.  Each device the
// library runs on holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress gives for the
// current device (pt_ctx::noalloc), never through this name.
static __device__ __align__(256) unsigned char scratch[PT_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(PT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kChunk = 50;       // generations per captured graph
constexpr int kChunkLong = 250;  // ... for fits without a window rule
constexpr int kMaxLeadGens = 20000;  // longest fit PT_FUSION_AUTO runs in the leading-step form
// the leading-step form takes a launch's buffer slot from its parity, so every
// graph must start at an even launch
static_assert(kChunk % 2 == 0 && kChunkLong % 2 == 0, "graph chunks must hold an even number of launches");

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return PT_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes, (size_t)256);
        if (hipMalloc(&p, want) != hipSuccess) {
            p = nullptr;
            return fail(PT_ENOMEM, "hipMalloc(%zu bytes) failed", want);
        }
        cap = want;
        return PT_OK;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct PinBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes) {
        if (bytes <= cap) return PT_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = std::max(bytes, (size_t)4096);
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return fail(PT_ENOMEM, "hipHostMalloc(%zu bytes) failed", want);
        }
        cap = want;
        return PT_OK;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct Geometry {
    int spl;  // samples per lane
    int cpg;  // candidates per workgroup
};

const int kSpl[] = {4, 8, 16, 32};
const int kCpg[] = {1, 2, 4, 8};

bool spl_ok(int s) { return s == 4 || s == 8 || s == 16 || s == 32; }
bool cpg_ok(int c) { return c == 1 || c == 2 || c == 4 || c == 8; }

int size_class(int64_t n) {
    int c = 0;
    while (n > 1) {
        n >>= 1;
        ++c;
    }
    return c;  // floor(log2 n)
}

// ----------------------------------------------------------------- launchers
// lead: 0 the objective alone (or with the last-workgroup step); 1, 2 the
// leading-step form (launched with fused >= 2), 2 taking the step's inputs as
// kernel arguments (one-block fits)
ObjKernel objective_kernel(int dtype, Geometry g, int mode, bool slope, int lead = 0) {
    const bool f64 = dtype == PT_F64;
    switch (g.spl) {
        case 4: return f64 ? objective_kernel_f64_s4(g.cpg, mode, slope, lead)
                           : objective_kernel_f32_s4(g.cpg, mode, slope, lead);
        case 8: return f64 ? objective_kernel_f64_s8(g.cpg, mode, slope, lead)
                           : objective_kernel_f32_s8(g.cpg, mode, slope, lead);
        case 16: return f64 ? objective_kernel_f64_s16(g.cpg, mode, slope, lead)
                            : objective_kernel_f32_s16(g.cpg, mode, slope, lead);
        default: return f64 ? objective_kernel_f64_s32(g.cpg, mode, slope, lead)
                            : objective_kernel_f32_s32(g.cpg, mode, slope, lead);
    }
}

PersistKernel persistent_kernel(int dtype, Geometry g, int mode, bool slope) {
    const bool f64 = dtype == PT_F64;
    switch (g.spl) {
        case 4: return f64 ? persistent_kernel_f64_s4(g.cpg, mode, slope) : persistent_kernel_f32_s4(g.cpg, mode, slope);
        case 8: return f64 ? persistent_kernel_f64_s8(g.cpg, mode, slope) : persistent_kernel_f32_s8(g.cpg, mode, slope);
        case 16:
            return f64 ? persistent_kernel_f64_s16(g.cpg, mode, slope) : persistent_kernel_f32_s16(g.cpg, mode, slope);
        default:
            return f64 ? persistent_kernel_f64_s32(g.cpg, mode, slope) : persistent_kernel_f32_s32(g.cpg, mode, slope);
    }
}

// Validity of the FP64 phasor path (see lane_rot) for every candidate with
// f0 in [f0lo, f0hi], |f1| <= f1max, |f2| <= f2max, |f3| <= f3max and chunk
// centres |m| <= span samples from the reference (turns per sample^k at a
// centre: c3 = a3 + 4 a4 m, c2 = a2 + 3 a3 m + 6 a4 m^2, c1 = f(t) / fs), with
// C = S / 2 and T = 256 S samples per tile:
//   (1) C^3 |c3| + C^4 |c4| <= 1e-12 turns (dropped terms);
//   (2) theta^2 / 2 <= 1e-11 with theta = 2 pi |c2| C^2 (first-order
//       quadratic correction);
//   (3) |sin 2 pi c1| >= S * 2.2e-4 over the block's frequency range
//       (conditioning of the three-term recurrence);
//   (4) 2 pi T (2 |c2| + 3 |c3| T + 4 |c4| T^2) <= 6e-3: the local frequency
//       moves by less than that angle across a tile (small-angle rotation).
bool phasor_ok(int spl, double fs, double span, double f0lo, double f0hi, double f1max, double f2max,
               double f3max) {
    const double a3 = f2max / (6.0 * fs * fs * fs);
    const double a4 = f3max / (24.0 * fs * fs * fs * fs);
    const double b3 = a3 + 4.0 * a4 * span;
    const double b2 = f1max / (2.0 * fs * fs) + 3.0 * a3 * span + 6.0 * a4 * span * span;
    const double C = spl / 2;
    if (!(C * C * C * (b3 + C * a4) <= 1e-12)) return false;
    const double th = 2.0 * M_PI * b2 * C * C;
    if (!(0.5 * th * th <= 1e-11)) return false;
    const double T = 256.0 * spl;
    if (!(2.0 * M_PI * T * (2.0 * b2 + 3.0 * b3 * T + 4.0 * a4 * T * T) <= 6e-3)) return false;
    const double tmax = span / fs;
    const double dev = f1max * tmax + f2max * tmax * tmax / 2.0 + f3max * tmax * tmax * tmax / 6.0;
    const double xlo = (f0lo - dev) / fs, xhi = (f0hi + dev) / fs;  // turns per sample
    if (!(std::isfinite(xlo) && std::isfinite(xhi)) || xhi - xlo > 1e6) return false;
    const double delta = std::asin(std::min(1.0, spl * 2.2e-4)) / (2.0 * M_PI);
    // no multiple of 1/2 within delta of [xlo, xhi]
    const double k0 = std::ceil(2.0 * (xlo - delta));
    return !(k0 / 2.0 <= xhi + delta);
}

double box_max(const pt_box& bx, int j) { return std::max(std::fabs(bx.lo[j]), std::fabs(bx.hi[j])); }
bool box_quartic(const pt_box& bx) { return bx.lo[6] != 0.0 || bx.hi[6] != 0.0; }

unsigned pow2_at_least(int v) {
    unsigned p = 256;
    while ((int)p < v) p <<= 1;
    return p;
}

// Launch plan of one fit / batch.
struct Plan {
    int nblk = 0;
    int P = 0;
    int dtype = PT_F32;
    bool mixed = false;
    bool slope = false;
    int mode = 0;          // kernel arithmetic: kModePoly / kModeMixed / kModePhasor
    Geometry geo{16, 4};
    int total_units = 0;
    int grid = 0;          // objective workgroups (multiple of 8)
    int grid_lead = 0;     // leading-step form: objective units plus one per block (multiple of 8)
    unsigned de_threads = 64;
    size_t de_lds = 0;
    int max_gens = 0;
    bool window = false;
    int fused = 0;         // DE step inside the objective launch: 0 no, 1 last workgroup, 2 leading step
    // Objective launches of one generation in the graph form: blocks whose
    // boxes allow the FP64 phasor arithmetic and those that do not run as
    // separate launches, each over its own copy of its blocks' descriptors
    // (units numbered from 0); otherwise one launch over the main table.
    struct Launch {
        int desc_off;      // first descriptor of the launch in the context's table
        int nblk;
        int mode;
        int total_units, grid, grid_lead;
        ObjKernel obj;       // objective alone, or with the last-workgroup step
        ObjKernel obj_lead;  // leading-step instance (null unless that form is planned)
    };
    std::vector<Launch> launches;
    // One-block leading-step fits: the step's inputs as kernel arguments, per
    // launch parity p (slot p ^ 1) -- tile partials, population rows, trial
    // rows, population objectives -- and lp = P | ntiles << 9.  Null: every
    // launch reads them from the descriptor.
    struct LeadArgs {
        const double* part = nullptr;
        const double* rows = nullptr;
        const double* trial = nullptr;
        const double* fpop = nullptr;
        int lp = 0;
    };
    LeadArgs lead_args[2];
};

// Launch of an objective-kernel instance (argument order of k_objective).
void launch_objective(ObjKernel k, unsigned grid, size_t lds, hipStream_t s, const BlockDesc* d, int nblk,
                      int units, int fused, const Plan::LeadArgs& la = Plan::LeadArgs()) {
    hipLaunchKernelGGL(k, dim3(grid), dim3(kThreads), lds, s, fused, nblk, units, la.lp, la.part, la.rows, la.trial,
                       la.fpop, d);
}

}  // namespace

// ------------------------------------------------------------------ context
struct pt_ctx {
    int device = 0;
    int ncu = 0;
    hipStream_t cap_stream = nullptr;
    // second stream and fork / join events: the objective launches of a batch
    // split by arithmetic run side by side (their blocks share nothing)
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // the window rule's stop checks: copies of the state behind alternate chunks
    hipEvent_t ev_state[2] = {nullptr, nullptr};
    DevBuf desc, pop, trial, fpop, partials, hist, state, rec, staging, eval_pop, tune_block, sync;
    PinBuf hdesc, hrec, hstate;
    // last fit (for pt_last_population / pt_last_history)
    int last_nblk = 0, last_P = 0, last_maxg = 0;
    std::vector<int> last_gens;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    int64_t launches = 0;
    double total_ms = 0.0;
    // launch mode and the persistent kernel's error flag
    int launch_mode = PT_LAUNCH_AUTO;
    int fp64_method = PT_FP64_AUTO;
    int last_launch = PT_LAUNCH_GRAPH;
    int last_arith = PT_ARITH_FP64_POLY;
    Geometry last_geo{0, 0};  // geometry of the most recent fit or objective evaluation
    int64_t last_fit_launches = 0;
    int step_fusion = PT_FUSION_AUTO;
    uint64_t spin_ticks = 0;
    DevBuf errflag;
    // initial-range estimation
    int seed_max_log = 0;  // largest log2(snippet) the device's LDS allows
    DevBuf seed_out, seed_stage;
    PinBuf hseed;
    // geometry
    Geometry forced{0, 0};
    std::map<std::tuple<int, int, int>, Geometry> tuned;  // (size class, P, mixed)
    // this device's copy of the allocation-free entry point's array
    unsigned char* noalloc = nullptr;
    // graph cache
    struct GraphKey {
        void* desc;
        int nblk, grid, total_units, spl, cpg, dtype, mixed, slope;
        unsigned de_threads;
        size_t de_lds;
        int iters, fused, base;
        std::vector<int> launches;  // (descriptor offset, blocks, arithmetic, units) per objective launch
        std::vector<const void*> args;  // pointers the launches take as kernel arguments
        bool operator<(const GraphKey& o) const {
            return std::tie(desc, nblk, grid, total_units, spl, cpg, dtype, mixed, slope, de_threads, de_lds, iters,
                            fused, base, launches, args) < std::tie(o.desc, o.nblk, o.grid, o.total_units, o.spl,
                                                                    o.cpg, o.dtype, o.mixed, o.slope, o.de_threads,
                                                                    o.de_lds, o.iters, o.fused, o.base, o.launches,
                                                                    o.args);
        }
    };
    // Cached graph executables, at most kMaxGraphs (the leading-step form keeps
    // one per chunk of a fit, so a context that fits many shapes would
    // otherwise grow without bound); `used` orders them for eviction.
    struct GraphEntry {
        hipGraphExec_t exec;
        uint64_t used;
    };
    static constexpr size_t kMaxGraphs = 256;
    std::map<GraphKey, GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // resident workgroups per compute unit of an objective kernel instance
    // with the leading step's LDS, by (kernel, dynamic LDS bytes)
    std::map<std::pair<const void*, size_t>, int> resident;

    void drop_graphs() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second.exec);
        graphs.clear();
    }
};

namespace {

Geometry default_geometry(int64_t n, int P) {
    // Prefer long lane chunks and many candidates per workgroup (amortises the
    // FP64 anchor and the reduction) while keeping >= ~1000 workgroups.
    Geometry best{4, 1};
    double best_score = -1;
    for (int s : kSpl) {
        for (int c : kCpg) {
            const int64_t tiles = (n + 256LL * s - 1) / (256LL * s);
            const int64_t groups = (P + c - 1) / c;
            const int64_t units = tiles * groups;
            const double waste = (double)(groups * c - P) / (groups * c);
            double score = (double)s * c * (1.0 - waste);
            if (units < 1024) score *= (double)units / 1024.0;
            if (score > best_score) {
                best_score = score;
                best = {s, c};
            }
        }
    }
    return best;
}

// The geometry with the most candidate·samples per lane (the fewest
// per-candidate set-up operations per sample), for throughput-bound launches.
Geometry throughput_geometry(int P) {
    Geometry best{4, 1};
    double best_score = -1;
    for (int s : kSpl) {
        for (int c : kCpg) {
            const int64_t groups = (P + c - 1) / c;
            const double score = (double)s * c * (double)P / (double)(groups * c);
            if (score > best_score) {
                best_score = score;
                best = {s, c};
            }
        }
    }
    return best;
}

Geometry choose_geometry(pt_ctx* ctx, int64_t n, int P, bool mixed) {
    if (ctx->forced.spl) return ctx->forced;
    auto it = ctx->tuned.find(std::make_tuple(size_class(n), P, (int)mixed));
    if (it != ctx->tuned.end()) return it->second;
    return default_geometry(n, P);
}

int check_block(const pt_block* b, int idx) {
    if (!b) return fail(PT_EINVAL, "block %d: null", idx);
    if (!b->samples) return fail(PT_EINVAL, "block %d: samples is null", idx);
    if (b->n < 8) return fail(PT_EINVAL, "block %d: n = %lld < 8", idx, (long long)b->n);
    if (b->n > (int64_t)1 << 31) return fail(PT_EINVAL, "block %d: n = %lld exceeds 2^31", idx, (long long)b->n);
    if (b->dtype != PT_F32 && b->dtype != PT_F64) return fail(PT_EINVAL, "block %d: dtype %d", idx, b->dtype);
    if (!(b->fs > 0) || !std::isfinite(b->fs)) return fail(PT_EINVAL, "block %d: fs must be > 0", idx);
    if (!std::isnan(b->ref) && !std::isfinite(b->ref)) return fail(PT_EINVAL, "block %d: ref not finite", idx);
    if (!std::isnan(b->ref) && std::fabs(b->ref) > 4.0 * (double)b->n)
        return fail(PT_EINVAL, "block %d: |ref| > 4 n", idx);
    int D = 0;
    for (int j = 0; j < PT_NSLOT; ++j) {
        if (!std::isfinite(b->box.lo[j]) || !std::isfinite(b->box.hi[j]))
            return fail(PT_EINVAL, "block %d: box slot %d not finite", idx, j);
        if (b->box.lo[j] > b->box.hi[j]) return fail(PT_EINVAL, "block %d: box slot %d has lo > hi", idx, j);
        if (b->box.lo[j] < b->box.hi[j]) ++D;
    }
    if (D == 0) return fail(PT_EINVAL, "block %d: every box slot is fixed", idx);
    return PT_OK;
}

int check_de(const pt_de_settings* de) {
    if (!de) return fail(PT_EINVAL, "DE settings are null");
    if (de->pop < 4 || de->pop > PT_MAX_POP) return fail(PT_EINVAL, "pop = %d outside [4, %d]", de->pop, PT_MAX_POP);
    if (de->max_gens < 0 || de->max_gens > 10000000) return fail(PT_EINVAL, "max_gens = %d", de->max_gens);
    if (!(de->F > 0 && de->F <= 2)) return fail(PT_EINVAL, "F must be in (0, 2]");
    if (!(de->CR >= 0 && de->CR <= 1)) return fail(PT_EINVAL, "CR must be in [0, 1]");
    if (de->rel_tol > 0 && de->window < 1) return fail(PT_EINVAL, "window must be >= 1 with rel_tol > 0");
    if (de->precision != PT_PREC_FP64 && de->precision != PT_PREC_MIXED)
        return fail(PT_EINVAL, "precision %d", de->precision);
    if (de->objective != PT_OBJ_CHI2 && de->objective != PT_OBJ_COR)
        return fail(PT_EINVAL, "objective %d", de->objective);
    if (std::isnan(de->vtr)) return fail(PT_EINVAL, "vtr is NaN");
    return PT_OK;
}

double block_ref(const pt_block* b) { return std::isnan(b->ref) ? 0.5 * (double)b->n : b->ref; }

hipEvent_t take_event(pt_ctx* ctx) {
    if (!ctx->ev_free.empty()) {
        hipEvent_t e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int collect_timing(pt_ctx* ctx) {
    for (auto& pr : ctx->ev_pending) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
        ctx->total_ms += ms;
        ctx->launches += 1;
        ctx->ev_free.push_back(pr.first);
        ctx->ev_free.push_back(pr.second);
    }
    ctx->ev_pending.clear();
    return PT_OK;
}

// Enqueue one generation: objective over all units, then the DE step.  L:
// the launch's index within the fit (the leading-step form's kernel argument).
int enqueue_generation(pt_ctx* ctx, const Plan& pl, hipStream_t s, bool timed, int L) {
    const BlockDesc* d = static_cast<const BlockDesc*>(ctx->desc.p);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        e0 = take_event(ctx);
        e1 = take_event(ctx);
        if (!e0 || !e1) return fail(PT_EDEVICE, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e0, s));
    }
    if (pl.fused && !timed) {
        // the DE step runs in each block's last objective workgroup (1), or
        // ahead of the objective in every workgroup (2 + launch index); a
        // second launch (blocks of the other arithmetic) runs beside the
        // first on the auxiliary stream, forked from and joined back to s
        const int f = pl.fused == 2 ? 2 + L : 1;
        const bool fork = pl.launches.size() > 1;
        if (fork) {
            HIPCHK(hipEventRecord(ctx->ev_fork, s));
            HIPCHK(hipStreamWaitEvent(ctx->aux_stream, ctx->ev_fork, 0));
        }
        for (size_t k = 0; k < pl.launches.size(); ++k) {
            const Plan::Launch& g = pl.launches[k];
            const int grid = pl.fused == 2 ? g.grid_lead : g.grid;
            launch_objective(pl.fused == 2 ? g.obj_lead : g.obj, grid, pl.de_lds, k ? ctx->aux_stream : s,
                             d + g.desc_off, g.nblk, g.total_units, f,
                             pl.fused == 2 ? pl.lead_args[L & 1] : Plan::LeadArgs());
            HIPCHK(hipGetLastError());
        }
        if (fork) {
            HIPCHK(hipEventRecord(ctx->ev_join, ctx->aux_stream));
            HIPCHK(hipStreamWaitEvent(s, ctx->ev_join, 0));
        }
        return PT_OK;
    }
    // (objective alone, then the DE step: the timed path, and the form
    // without fusion)
    for (const Plan::Launch& g : pl.launches) {
        launch_objective(g.obj, g.grid, 0, s, d + g.desc_off, g.nblk, g.total_units, 0);
        HIPCHK(hipGetLastError());
    }
    if (timed) {
        HIPCHK(hipEventRecord(e1, s));
        ctx->ev_pending.push_back({e0, e1});
    }
    hipLaunchKernelGGL(k_de_step, dim3(pl.nblk), dim3(pl.de_threads), pl.de_lds, s, d);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

// Graph of `iters` generations starting at launch `base` (the leading-step
// form passes the launch index, so its graphs are kept per base; the others
// share base 0).
int get_graph(pt_ctx* ctx, const Plan& pl, int iters, int base, hipGraphExec_t* out) {
    if (pl.fused != 2) base = 0;
    std::vector<int> sig;
    for (const Plan::Launch& g : pl.launches) {
        sig.push_back(g.desc_off);
        sig.push_back(g.nblk);
        sig.push_back(g.mode);
        sig.push_back(g.total_units);
    }
    std::vector<const void*> args;
    for (const Plan::LeadArgs& la : pl.lead_args) {
        args.push_back(la.part);
        args.push_back(la.rows);
        args.push_back(la.trial);
        args.push_back(la.fpop);
        args.push_back(reinterpret_cast<const void*>((uintptr_t)(unsigned)la.lp));
    }
    pt_ctx::GraphKey key{ctx->desc.p, pl.nblk, pl.grid, pl.total_units, pl.geo.spl, pl.geo.cpg, pl.dtype,
                         pl.mode, (int)pl.slope, pl.de_threads, pl.de_lds, iters, (int)pl.fused, base, sig, args};
    auto it = ctx->graphs.find(key);
    if (it != ctx->graphs.end()) {
        it->second.used = ++ctx->graph_clock;
        *out = it->second.exec;
        return PT_OK;
    }
    if (ctx->graphs.size() >= pt_ctx::kMaxGraphs) {
        // Evict the least recently used quarter.  A fit without the window rule
        // queues all its chunks at once, so an old executable may still be
        // queued: wait for the device first (a rare path, taken only when a
        // new graph is captured anyway).
        HIPCHK(hipDeviceSynchronize());
        std::vector<std::pair<uint64_t, const pt_ctx::GraphKey*>> order;
        for (const auto& kv : ctx->graphs) order.push_back({kv.second.used, &kv.first});
        std::sort(order.begin(), order.end(),
                  [](const auto& a, const auto& b) { return a.first < b.first; });
        std::vector<pt_ctx::GraphKey> victims;
        for (size_t k = 0; k < pt_ctx::kMaxGraphs / 4; ++k) victims.push_back(*order[k].second);
        for (const pt_ctx::GraphKey& v : victims) {
            auto vi = ctx->graphs.find(v);
            (void)hipGraphExecDestroy(vi->second.exec);
            ctx->graphs.erase(vi);
        }
    }
    hipStream_t cs = ctx->cap_stream;
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = PT_OK;
    for (int k = 0; k < iters && rc == PT_OK; ++k) rc = enqueue_generation(ctx, pl, cs, false, base + k);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != PT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(PT_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PT_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    ctx->graphs[key] = {ex, ++ctx->graph_clock};
    *out = ex;
    return PT_OK;
}

// Everything up to (and including) copying descriptors for nblk blocks.
// Whether a leading-step launch of `units` work units (bookkeeping units
// included) of kernel k fits in two rounds of resident workgroups; larger
// launches are throughput-bound and run the DE step elsewhere.
bool lead_fits(pt_ctx* ctx, ObjKernel k, size_t lds, int64_t units) {
    auto key = std::make_pair(reinterpret_cast<const void*>(k), lds);
    auto it = ctx->resident.find(key);
    int per_cu = 0;
    if (it != ctx->resident.end()) {
        per_cu = it->second;
    } else {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), kThreads, lds) !=
            hipSuccess)
            per_cu = 0;
        ctx->resident[key] = per_cu;
    }
    return units <= 2LL * per_cu * ctx->ncu;
}

// Descriptor fields of one block that do not depend on where its buffers
// live: samples (the caller's pointer), sizes, box, active slots and the DE
// settings.  Buffer pointers, unit_begin and sync are left null / zero.
BlockDesc base_desc(const pt_block& B, const pt_de_settings* de, int ntiles, int groups) {
    BlockDesc d;
    std::memset(&d, 0, sizeof d);
    d.samples = B.samples;
    d.n = B.n;
    d.fs = B.fs;
    d.ref = block_ref(&B);
    d.dtype = B.dtype;
    d.P = de->pop;
    int D = 0;
    for (int j = 0; j < kSlots; ++j) {
        d.lo[j] = B.box.lo[j];
        d.hi[j] = B.box.hi[j];
        if (B.box.lo[j] < B.box.hi[j]) {
            d.act[D++] = j;
            d.amask |= 1 << j;
        }
    }
    d.D = D;
    d.ntiles = ntiles;
    d.ngroups = groups;
    d.window = de->window;
    d.max_gens = de->max_gens;
    d.F = de->F;
    d.CR = de->CR;
    d.vtr = de->vtr;
    d.rel_tol = de->rel_tol;
    d.seed = de->seed;
    d.stream = B.stream;
    d.gen_begin = 0;
    d.objective = de->objective;
    d.quartic = box_quartic(B.box);
    return d;
}

int prepare(pt_ctx* ctx, const pt_block* blocks, int nblk, const pt_de_settings* de, hipStream_t s, Plan* pl,
            bool with_state) {
    const int P = de->pop;
    pl->nblk = nblk;
    pl->P = P;
    pl->dtype = blocks[0].dtype;
    pl->mixed = de->precision == PT_PREC_MIXED;
    pl->max_gens = de->max_gens;
    pl->window = de->rel_tol > 0;
    bool slope = false;
    int64_t nmax = 0;
    for (int b = 0; b < nblk; ++b) {
        if (blocks[b].dtype != pl->dtype) return fail(PT_EINVAL, "block %d: all blocks need one dtype", b);
        if (blocks[b].box.lo[5] != 0.0 || blocks[b].box.hi[5] != 0.0) slope = true;
        nmax = std::max(nmax, blocks[b].n);
    }
    pl->slope = slope;
    // geometry from the largest block (one kernel instance per launch).  A
    // batch with more than four work units per compute unit at that geometry
    // is throughput-bound: there the geometry with the most work per lane
    // wins, whatever a single-block tuning chose (64 uneven blocks, P = 40,
    // FP64: 32 x 8 0.226 s, 32 x 4 0.263 s, 16 x 8 0.269 s, 16 x 4 0.308 s;
    // mixed: 0.257, 0.276, 0.285, 0.316 s)
    pl->geo = choose_geometry(ctx, nmax, P, pl->mixed);
    if (nblk > 1 && !ctx->forced.spl) {
        int64_t units = 0;
        for (int b = 0; b < nblk; ++b)
            units += (blocks[b].n + (int64_t)kThreads * pl->geo.spl - 1) / ((int64_t)kThreads * pl->geo.spl) *
                     ((P + pl->geo.cpg - 1) / pl->geo.cpg);
        if (units > 4LL * ctx->ncu) pl->geo = throughput_geometry(P);
    }
    pl->mode = pl->mixed ? kModeMixed : kModePoly;
    std::vector<char> phasor(nblk, 0);
    int nphasor = 0;
    if (!pl->mixed && ctx->fp64_method != PT_FP64_POLY) {
        for (int b = 0; b < nblk; ++b) {
            const pt_box& bx = blocks[b].box;
            const double span = (double)blocks[b].n + std::fabs(block_ref(&blocks[b]));
            phasor[b] = phasor_ok(pl->geo.spl, blocks[b].fs, span, bx.lo[2], bx.hi[2], box_max(bx, 3),
                                  box_max(bx, 4), box_max(bx, 6));
            nphasor += phasor[b];
        }
        if (nphasor == nblk) pl->mode = kModePhasor;  // one kernel for every block
    }
    const int tile = kThreads * pl->geo.spl;
    const int groups = (P + pl->geo.cpg - 1) / pl->geo.cpg;

    // sizes
    std::vector<int> ntiles(nblk);
    size_t part_elems = 0, stage_bytes = 0;
    int64_t units = 0;
    for (int b = 0; b < nblk; ++b) {
        ntiles[b] = (int)((blocks[b].n + tile - 1) / tile);
        part_elems += (size_t)P * ntiles[b];
        units += (int64_t)ntiles[b] * groups;
        if (!blocks[b].on_device)
            stage_bytes += ((size_t)blocks[b].n * (blocks[b].dtype == PT_F64 ? 8 : 4) + 255) & ~(size_t)255;
    }
    if (units > (int64_t)1 << 30) return fail(PT_EINVAL, "batch too large (%lld work units)", (long long)units);
    pl->total_units = (int)units;
    pl->grid = (int)((units + 7) / 8 * 8);
    pl->grid_lead = (int)((units + nblk + 7) / 8 * 8);
    pl->de_threads = pow2_at_least(P);  // >= 256 and >= P: also fixes the partial-sum order
    pl->de_lds = (size_t)P * kSlots * 8 + (size_t)pl->de_threads * (8 + 8 + 4);
    // leading step (2) for launches that fit in two rounds of resident
    // workgroups, last-workgroup step (1) for larger ones (measured on the
    // paper-scale block at 16 x 4, 981 units in two rounds of 768: 32.6 ms
    // leading against 35.8 ms last-workgroup; a 64-block batch of 15 000
    // units: 533 ms against 486 ms)
    // (the leading form keeps one graph per 50-launch chunk, since the launch
    // index is a kernel argument: fits longer than kMaxLeadGens generations
    // use the last-workgroup form, whose graph is replayed)
    int fusion = ctx->step_fusion;
    if (fusion == PT_FUSION_AUTO)
        fusion = de->max_gens <= kMaxLeadGens &&
                         lead_fits(ctx, objective_kernel(pl->dtype, pl->geo, pl->mode, pl->slope, 1),
                                   pl->de_lds + (size_t)P * kSlots * 8, units + nblk)
                     ? PT_FUSION_LEAD
                     : PT_FUSION_LAST;
    pl->fused = (with_state && fusion != PT_FUSION_OFF && pl->de_threads == (unsigned)kThreads)
                    ? (fusion == PT_FUSION_LAST ? 1 : 2)
                    : 0;
    if (pl->fused == 2) pl->de_lds += (size_t)P * kSlots * 8;  // the leading step stages both row sets

    // two slots of the DE buffers (the leading-step form alternates between them)
    const size_t rows = (size_t)nblk * P * kStride * sizeof(double);
    int rc;
    if ((rc = ctx->desc.ensure(2 * sizeof(BlockDesc) * nblk)) || (rc = ctx->pop.ensure(2 * rows)) ||
        (rc = ctx->trial.ensure(2 * rows)) || (rc = ctx->fpop.ensure(2 * (size_t)nblk * P * sizeof(double))) ||
        (rc = ctx->partials.ensure(2 * part_elems * sizeof(double))) ||
        (rc = ctx->hist.ensure((size_t)nblk * (de->max_gens + 1) * sizeof(double))) ||
        (rc = ctx->state.ensure(2 * (size_t)nblk * sizeof(DeState))) ||
        (rc = ctx->sync.ensure((size_t)nblk * kSyncInts * sizeof(int))) ||
        (rc = ctx->rec.ensure((size_t)nblk * sizeof(FitRecord))) ||
        (rc = ctx->hdesc.ensure(2 * sizeof(BlockDesc) * nblk)) ||
        (rc = ctx->hrec.ensure((size_t)nblk * sizeof(FitRecord))) ||
        (rc = ctx->hstate.ensure(4 * (size_t)nblk * sizeof(DeState) + sizeof(int))))
        return rc;
    if (stage_bytes && (rc = ctx->staging.ensure(stage_bytes))) return rc;

    // descriptor table (pinned host -> device)
    BlockDesc* hd = static_cast<BlockDesc*>(ctx->hdesc.p);
    double* pop = static_cast<double*>(ctx->pop.p);
    double* trial = static_cast<double*>(ctx->trial.p);
    double* fpop = static_cast<double*>(ctx->fpop.p);
    double* part = static_cast<double*>(ctx->partials.p);
    double* hist = static_cast<double*>(ctx->hist.p);
    DeState* st = static_cast<DeState*>(ctx->state.p);
    char* stage = static_cast<char*>(ctx->staging.p);
    size_t part_off = 0, stage_off = 0;
    int unit_off = 0;
    for (int b = 0; b < nblk; ++b) {
        const pt_block& B = blocks[b];
        BlockDesc d = base_desc(B, de, ntiles[b], groups);
        const size_t bytes = (size_t)B.n * (B.dtype == PT_F64 ? 8 : 4);
        if (!B.on_device) {
            HIPCHK(hipMemcpyAsync(stage + stage_off, B.samples, bytes, hipMemcpyHostToDevice, s));
            d.samples = stage + stage_off;
            stage_off += (bytes + 255) & ~(size_t)255;
        }
        d.unit_begin = unit_off;
        unit_off += ntiles[b] * groups;
        d.pop = pop + (size_t)b * P * kStride;
        d.trial = trial + (size_t)b * P * kStride;
        d.fpop = fpop + (size_t)b * P;
        d.partials = part + part_off;
        part_off += (size_t)P * ntiles[b];
        d.hist = hist + (size_t)b * (de->max_gens + 1);
        d.st = with_state ? st + b : nullptr;
        if (pl->fused == 2) {
            d.pop2 = d.pop + (size_t)nblk * P * kStride;
            d.trial2 = d.trial + (size_t)nblk * P * kStride;
            d.fpop2 = d.fpop + (size_t)nblk * P;
            d.partials2 = d.partials + part_elems;
            d.st2 = d.st + nblk;
        }
        d.sync = with_state ? static_cast<int*>(ctx->sync.p) + (size_t)b * kSyncInts : nullptr;
        hd[b] = d;
    }
    // objective launches: one over the main table, or (FP64 batches whose
    // blocks differ in arithmetic) the phasor blocks and the others apart; a
    // one-block leading-step fit passes the step's inputs as kernel arguments
    const bool lead_fast = pl->fused == 2 && nblk == 1 && P < 512 && ntiles[0] < (1 << 22) && units < (1 << 23);
    pl->launches.clear();
    auto add_launch = [&](int desc_off, int n, int mode, int64_t u) {
        Plan::Launch L;
        L.desc_off = desc_off;
        L.nblk = n;
        L.mode = mode;
        L.total_units = (int)u;
        L.grid = (int)((u + 7) / 8 * 8);
        L.grid_lead = (int)((u + n + 7) / 8 * 8);
        L.obj = objective_kernel(pl->dtype, pl->geo, mode, pl->slope, 0);
        L.obj_lead = pl->fused == 2 ? objective_kernel(pl->dtype, pl->geo, mode, pl->slope, lead_fast ? 2 : 1)
                                    : nullptr;
        pl->launches.push_back(L);
    };
    int ndesc = nblk;
    if (nphasor == 0 || nphasor == nblk) {
        add_launch(0, nblk, pl->mode, units);
    } else {
        for (int want = 1; want >= 0; --want) {
            const int off = ndesc;
            int64_t u = 0;
            for (int b = 0; b < nblk; ++b) {
                if (phasor[b] != want) continue;
                BlockDesc d = hd[b];
                d.unit_begin = (int)u;
                u += (int64_t)d.ntiles * d.ngroups;
                hd[ndesc++] = d;
            }
            add_launch(off, ndesc - off, want ? kModePhasor : kModePoly, u);
        }
    }
    pl->lead_args[0] = pl->lead_args[1] = Plan::LeadArgs();
    if (lead_fast) {
        const BlockDesc& d0 = hd[0];  // gen_begin 0: launch L has parity L & 1
        for (int p = 0; p < 2; ++p)
            pl->lead_args[p] = Plan::LeadArgs{p ? d0.partials : d0.partials2, p ? d0.pop : d0.pop2,
                                              p ? d0.trial : d0.trial2, p ? d0.fpop : d0.fpop2,
                                              P | (int)(ntiles[0] << 9)};
    }
    HIPCHK(hipMemcpyAsync(ctx->desc.p, hd, sizeof(BlockDesc) * ndesc, hipMemcpyHostToDevice, s));
    return PT_OK;
}

void derive(pt_fit* f) {
    const double two_pi = 2.0 * M_PI;
    const double phi0 = f->coef[1], f0 = f->coef[2], f1 = f->coef[3], f2 = f->coef[4], f3 = f->coef[6];
    auto phase = [&](double t) {
        return phi0 + two_pi * (f0 * t + f1 * t * t / 2.0 + f2 * t * t * t / 6.0 + f3 * t * t * t * t / 24.0);
    };
    auto freq = [&](double t) { return f0 + f1 * t + f2 * t * t / 2.0 + f3 * t * t * t / 6.0; };
    auto wrap = [&](double p) {
        double r = std::fmod(p, two_pi);
        return r < 0 ? r + two_pi : r;
    };
    f->phase_centre = wrap(phi0);
    f->phase_left = wrap(phase(f->t_left));
    f->phase_right = wrap(phase(f->t_right));
    f->freq_left = freq(f->t_left);
    f->freq_right = freq(f->t_right);
    f->total_phase = phase(f->t_right) - phase(f->t_left);
}

int run_fit(pt_ctx* ctx, const pt_block* blocks, int nblk, const pt_de_settings* de, void* hip_stream,
            pt_fit* out) {
    int rc = check_de(de);
    if (rc) return rc;
    if (nblk < 1 || nblk > 4096) return fail(PT_EINVAL, "nblk = %d outside [1, 4096]", nblk);
    if (!out) return fail(PT_EINVAL, "out is null");
    for (int b = 0; b < nblk; ++b)
        if ((rc = check_block(&blocks[b], b))) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Plan pl;
    void* old_desc = ctx->desc.p;
    if ((rc = prepare(ctx, blocks, nblk, de, s, &pl, true))) return rc;
    if (ctx->desc.p != old_desc) ctx->drop_graphs();
    const BlockDesc* d = static_cast<const BlockDesc*>(ctx->desc.p);

    // persistent launch: one cooperative grid runs every generation
    bool persistent = false;
    int pgrid = 0, resident = 0;
    PersistKernel pk = nullptr;
    if (ctx->launch_mode == PT_LAUNCH_PERSISTENT && !ctx->timing && pl.P <= 256) {
        pk = persistent_kernel(pl.dtype, pl.geo, pl.mode, pl.slope);
        int per_cu = 0;
        HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(pk), kThreads,
                                                            0));
        const int cap = per_cu * ctx->ncu / 8 * 8;
        if (cap >= 8) {
            pgrid = std::min(cap, (pl.total_units + 7) / 8 * 8);
            resident = (pl.total_units + 7) / 8 <= pgrid / 8;
            persistent = true;
        }
    }
    if (ctx->launch_mode == PT_LAUNCH_PERSISTENT && !persistent)
        return fail(PT_EUNSUPPORTED, "persistent launch not possible (P = %d, timing %d)", pl.P, (int)ctx->timing);
    if ((rc = ctx->errflag.ensure(sizeof(int)))) return rc;
    int* err = static_cast<int*>(ctx->errflag.p);

    hipLaunchKernelGGL(k_de_init, dim3(nblk), dim3(pl.de_threads), 0, s, d, err);
    HIPCHK(hipGetLastError());

    // evaluation of gen 0 plus max_gens generations; the leading-step form adds
    // one launch for the DE step of the last generation
    const bool lead = pl.fused == 2 && !ctx->timing;
    const int iters = de->max_gens + 1 + (lead ? 1 : 0);
    if (persistent) {
        int nb = nblk, tu = pl.total_units, steps = de->max_gens + 1;
        uint64_t ticks = ctx->spin_ticks;
        void* args[] = {&d, &nb, &tu, &steps, &resident, &err, &ticks};
        hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(pk), dim3(pgrid), dim3(kThreads),
                                                  args, 0, s);
        if (e != hipSuccess) {
            if (ctx->launch_mode == PT_LAUNCH_PERSISTENT)
                return fail(PT_EDEVICE, "hipLaunchCooperativeKernel: %s", hipGetErrorString(e));
            (void)hipGetLastError();
            persistent = false;  // fall back to the graph path below
        }
    }
    ctx->last_launch = persistent ? PT_LAUNCH_PERSISTENT : PT_LAUNCH_GRAPH;
    // (a batch split by arithmetic reports the phasor path, whose per-sample
    // error is the larger)
    ctx->last_arith = persistent || pl.launches.size() == 1 ? pl.mode : kModePhasor;
    ctx->last_geo = pl.geo;
    ctx->last_fit_launches = persistent ? 1 : iters;
    if (persistent) {
        // nothing else to enqueue
    } else if (ctx->timing) {
        for (int k = 0; k < iters; ++k)
            if ((rc = enqueue_generation(ctx, pl, s, true, k))) return rc;
    } else {
        hipGraphExec_t ex = nullptr;
        // fits without a window rule need no stop checks between chunks:
        // longer chunks, fewer graph launches
        const int chunk = pl.window ? kChunk : kChunkLong;
        const int full = iters / chunk, rem = iters % chunk;
        DeState* hst = static_cast<DeState*>(ctx->hstate.p);
        const int ns = lead ? 2 * nblk : nblk;  // leading-step form: either slot may hold the stop
        auto stopped = [&](const DeState* h) {
            for (int b = 0; b < nblk; ++b)
                if (!(h[b].done != 0 || (lead && h[nblk + b].done != 0))) return false;
            return true;
        };
        bool all = false;
        for (int c = 0; c < full && !all; ++c) {
            if ((c == 0 || lead) && (rc = get_graph(ctx, pl, chunk, c * chunk, &ex))) return rc;
            HIPCHK(hipGraphLaunch(ex, s));
            if (pl.window && c + 1 < full) {
                // Stop launching once every block has met its stop rule.  The
                // state after chunk c is copied behind it; the host waits for
                // the copy after chunk c - 1's only once chunk c is queued, so
                // the device never idles for the check (a chunk queued after
                // the stop runs as early-exit launches).
                HIPCHK(hipMemcpyAsync(hst + (c & 1) * ns, ctx->state.p, sizeof(DeState) * ns,
                                      hipMemcpyDeviceToHost, s));
                HIPCHK(hipEventRecord(ctx->ev_state[c & 1], s));
                if (c >= 1) {
                    HIPCHK(hipEventSynchronize(ctx->ev_state[(c - 1) & 1]));
                    all = stopped(hst + ((c - 1) & 1) * ns);
                }
            }
        }
        for (int k = 0; k < rem && !all; ++k)
            if ((rc = enqueue_generation(ctx, pl, s, false, full * chunk + k))) return rc;
    }
    hipLaunchKernelGGL(k_finalize, dim3(nblk), dim3(64), 0, s, d, static_cast<FitRecord*>(ctx->rec.p));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(ctx->hrec.p, ctx->rec.p, sizeof(FitRecord) * nblk, hipMemcpyDeviceToHost, s));
    int* herr = reinterpret_cast<int*>(static_cast<DeState*>(ctx->hstate.p) + 4 * nblk);
    HIPCHK(hipMemcpyAsync(herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (ctx->timing && (rc = collect_timing(ctx))) return rc;
    if (*herr) return fail(PT_EDEVICE, "persistent fit: a block's generation did not complete in time");

    const FitRecord* r = static_cast<const FitRecord*>(ctx->hrec.p);
    ctx->last_nblk = nblk;
    ctx->last_P = de->pop;
    ctx->last_maxg = de->max_gens;
    ctx->last_gens.assign(nblk, 0);
    for (int b = 0; b < nblk; ++b) {
        pt_fit& f = out[b];
        std::memset(&f, 0, sizeof f);
        for (int j = 0; j < PT_NSLOT; ++j) f.coef[j] = r[b].x[j];
        f.objective = r[b].f;
        f.generations = r[b].gens;
        f.flags = r[b].flags;
        f.ref = block_ref(&blocks[b]);
        f.t_left = (0.0 - f.ref) / blocks[b].fs;
        f.t_right = ((double)blocks[b].n - f.ref) / blocks[b].fs;
        derive(&f);
        ctx->last_gens[b] = r[b].gens;
    }
    return PT_OK;
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int pt_version(void) { return 10000; }

const char* pt_last_error(void) { return g_err.c_str(); }

int pt_ctx_create(int device, pt_ctx** out) {
    if (!out) return fail(PT_EINVAL, "out is null");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(PT_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(PT_EDEVICE, "device %d not in [0, %d)", device, count);
    HIPCHK(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, device));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(PT_EDEVICE, "device %d is %s; this library is built for gfx950 only", device, prop.gcnArchName);
    std::unique_ptr<pt_ctx> c(new (std::nothrow) pt_ctx());
    if (!c) return fail(PT_ENOMEM, "out of host memory");
    c->device = device;
    c->ncu = prop.multiProcessorCount;
    // the allocation-free entry point's array: its address on this device
    void* na = nullptr;
    HIPCHK(hipGetSymbolAddress(&na, HIP_SYMBOL(scratch)));
    c->noalloc = static_cast<unsigned char*>(na);
    int clk_khz = 0;
    if (hipDeviceGetAttribute(&clk_khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || clk_khz <= 0)
        clk_khz = 100000;
    c->spin_ticks = (uint64_t)clk_khz * 1000ull * 5ull;  // 5 s
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess)
        lds_max = 65536;
    // 16 bytes of LDS per snippet sample plus the kernel's 1 KiB of reduction space
    for (int lg = kSeedMaxLog; lg >= 6; --lg)
        if ((16 << lg) + 1024 <= lds_max) {
            c->seed_max_log = lg;
            break;
        }
    HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    for (hipEvent_t& e : c->ev_state) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    *out = c.release();
    return PT_OK;
}

void pt_ctx_destroy(pt_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->drop_graphs();
    for (auto e : ctx->ev_free) (void)hipEventDestroy(e);
    for (auto& pr : ctx->ev_pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    DevBuf* bufs[] = {&ctx->desc,    &ctx->pop,      &ctx->trial,   &ctx->fpop,  &ctx->partials, &ctx->hist,
                      &ctx->state,   &ctx->rec,      &ctx->staging, &ctx->eval_pop, &ctx->tune_block, &ctx->errflag,
                      &ctx->sync,    &ctx->seed_out, &ctx->seed_stage};
    for (DevBuf* b : bufs) b->release();
    ctx->hdesc.release();
    ctx->hrec.release();
    ctx->hseed.release();
    ctx->hstate.release();
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->aux_stream) (void)hipStreamDestroy(ctx->aux_stream);
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    for (hipEvent_t e : ctx->ev_state)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

int pt_fit_block(pt_ctx* ctx, const pt_block* block, const pt_de_settings* de, void* hip_stream, pt_fit* out) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (!block) return fail(PT_EINVAL, "block is null");
    return run_fit(ctx, block, 1, de, hip_stream, out);
}

int pt_fit_batch(pt_ctx* ctx, const pt_block* blocks, int nblk, const pt_de_settings* de, void* hip_stream,
                 pt_fit* out) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (!blocks) return fail(PT_EINVAL, "blocks is null");
    return run_fit(ctx, blocks, nblk, de, hip_stream, out);
}

// Shared set-up of the bare objective entry points: descriptor of one block
// without DE state, the caller's P x 6 rows copied into the stride-8 trial
// rows, and the objective kernel of the chosen geometry.
static_assert(kSlots == PT_NSLOT, "device rows hold the C-ABI's slots");

// Rows of a caller's population (P x kSlots, packed) into the kStride layout
// of a trial buffer; the pad slot is zero.
__global__ void k_pack_rows(const double* __restrict__ src, double* __restrict__ dst, int P) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P * kStride; e += gridDim.x * blockDim.x) {
        const int r = e / kStride, c = e - r * kStride;
        dst[e] = c < kSlots ? src[(size_t)r * kSlots + c] : 0.0;
    }
}

// Extents of a population that decide the objective's arithmetic: the
// amplitude-slope and quartic terms are on when any row uses them, and the
// FP64 phasor path applies when every row satisfies its bound.  Rows are
// added in any number of pieces.
struct PopExtents {
    double lo[2] = {0.0, 0.0}, hi[2] = {0.0, 0.0};  // slots 5 and 6 (zero rows excluded)
    double f0lo = INFINITY, f0hi = -INFINITY, f1 = 0.0, f2 = 0.0, f3 = 0.0;
    void add(const double* rows, int n) {
        for (int p = 0; p < n; ++p) {
            const double* r = rows + (size_t)p * PT_NSLOT;
            for (int k = 0; k < 2; ++k) {
                const double v = r[5 + k];
                if (v != 0.0 || !std::isfinite(v)) {
                    lo[k] = std::min(lo[k], v);
                    hi[k] = std::max(hi[k], v);
                    if (!std::isfinite(v)) hi[k] = 1.0;  // keep the term on; the result is not finite anyway
                }
            }
            f0lo = std::min(f0lo, r[2]);
            f0hi = std::max(f0hi, r[2]);
            f1 = std::max(f1, std::fabs(r[3]));
            f2 = std::max(f2, std::fabs(r[4]));
            f3 = std::max(f3, std::fabs(r[6]));
        }
    }
    // the block as the objective kernels see it: slots 5 and 6 span the rows
    void apply(pt_block& blk) const {
        for (int k = 0; k < 2; ++k) {
            blk.box.lo[5 + k] = std::isfinite(lo[k]) ? lo[k] : -1.0;
            blk.box.hi[5 + k] = std::isfinite(hi[k]) ? hi[k] : 1.0;
        }
    }
    int mode(const Plan& pl, const pt_ctx* ctx, const pt_block* block) const {
        if (pl.mixed || ctx->fp64_method == PT_FP64_POLY) return pl.mode;
        const double span = (double)block->n + std::fabs(block_ref(block));
        return std::isfinite(f1) && std::isfinite(f2) && std::isfinite(f3) &&
                       phasor_ok(pl.geo.spl, block->fs, span, f0lo, f0hi, f1, f2, f3)
                   ? kModePhasor
                   : kModePoly;
    }
};

static int check_eval_args(const pt_block* block, const double* pop, int P, int precision, int objective) {
    int rc = check_block(block, 0);
    if (rc) return rc;
    if (!pop) return fail(PT_EINVAL, "pop is null");
    if (P < 1 || P > PT_MAX_POP) return fail(PT_EINVAL, "P = %d outside [1, %d]", P, PT_MAX_POP);
    if (precision != PT_PREC_FP64 && precision != PT_PREC_MIXED) return fail(PT_EINVAL, "precision %d", precision);
    if (objective != PT_OBJ_CHI2 && objective != PT_OBJ_COR) return fail(PT_EINVAL, "objective %d", objective);
    return PT_OK;
}

static pt_de_settings eval_settings(int P, int precision, int objective) {
    pt_de_settings de;
    std::memset(&de, 0, sizeof de);
    de.pop = P;
    de.max_gens = 0;
    de.F = 0.5;
    de.CR = 0.5;
    de.precision = precision;
    de.objective = objective;
    return de;
}

static int eval_setup(pt_ctx* ctx, const pt_block* block, const double* pop, int P, int precision, int objective,
                      hipStream_t s, Plan* pl, ObjKernel* obj) {
    int rc = check_eval_args(block, pop, P, precision, objective);
    if (rc) return rc;
    HIPCHK(hipSetDevice(ctx->device));
    std::vector<double> hp((size_t)P * PT_NSLOT);
    HIPCHK(hipMemcpyAsync(hp.data(), pop, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    PopExtents ext;
    ext.add(hp.data(), P);
    pt_block blk = *block;
    ext.apply(blk);
    pt_de_settings de = eval_settings(P, precision, objective);
    void* old_desc = ctx->desc.p;
    if ((rc = prepare(ctx, &blk, 1, &de, s, pl, false))) return rc;
    if (ctx->desc.p != old_desc) ctx->drop_graphs();
    const BlockDesc* hd = static_cast<const BlockDesc*>(ctx->hdesc.p);
    // (a kernel, not a strided 2-D copy: those have returned wrong data under
    // the profiler on this runtime)
    hipLaunchKernelGGL(k_pack_rows, dim3(1), dim3(256), 0, s, pop, hd[0].trial, P);
    HIPCHK(hipGetLastError());
    pl->mode = ext.mode(*pl, ctx, block);
    *obj = objective_kernel(pl->dtype, pl->geo, pl->mode, pl->slope);
    ctx->last_arith = pl->mode;
    ctx->last_geo = pl->geo;
    return PT_OK;
}

int pt_objective(pt_ctx* ctx, const pt_block* block, const double* pop, int P, int precision, int objective,
                 void* hip_stream, double* out) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (!out) return fail(PT_EINVAL, "out is null");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Plan pl;
    ObjKernel obj = nullptr;
    int rc = eval_setup(ctx, block, pop, P, precision, objective, s, &pl, &obj);
    if (rc) return rc;
    const BlockDesc* d = static_cast<const BlockDesc*>(ctx->desc.p);
    launch_objective(obj, pl.grid, 0, s, d, 1, pl.total_units, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_out, dim3(1), dim3(pl.de_threads), pl.de_threads * sizeof(double), s, d, out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    return PT_OK;
}

// One descriptor into device memory, passed by value (no host staging).
__global__ void k_put_desc(BlockDesc d, BlockDesc* dst) {
    if (threadIdx.x == 0) *dst = d;
}

int pt_objective_noalloc(pt_ctx* ctx, const pt_block* block, const double* pop, int P, int precision,
                         int objective, void* hip_stream, double* out) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (!out) return fail(PT_EINVAL, "out is null");
    int rc = check_eval_args(block, pop, P, precision, objective);
    if (rc) return rc;
    if (!block->on_device) return fail(PT_EINVAL, "pt_objective_noalloc: samples must be a device pointer");
    if (!ctx->noalloc) return fail(PT_EDEVICE, "pt_objective_noalloc: no device array on this context");
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);

    // population extents (the arithmetic choice of pt_objective), read in
    // pieces through a fixed host buffer
    constexpr int kRows = 64;
    double rows_h[kRows * PT_NSLOT];
    PopExtents ext;
    for (int r0 = 0; r0 < P; r0 += kRows) {
        const int cnt = std::min(kRows, P - r0);
        HIPCHK(hipMemcpyAsync(rows_h, pop + (size_t)r0 * PT_NSLOT, sizeof(double) * PT_NSLOT * cnt,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        ext.add(rows_h, cnt);
    }
    pt_block blk = *block;
    ext.apply(blk);
    const pt_de_settings de = eval_settings(P, precision, objective);

    // the plan pt_objective's set-up makes for one block without DE state
    Plan pl;
    pl.nblk = 1;
    pl.P = P;
    pl.dtype = blk.dtype;
    pl.mixed = precision == PT_PREC_MIXED;
    pl.slope = blk.box.lo[5] != 0.0 || blk.box.hi[5] != 0.0;
    pl.geo = choose_geometry(ctx, blk.n, P, pl.mixed);
    pl.mode = pl.mixed ? kModeMixed : kModePoly;
    pl.mode = ext.mode(pl, ctx, block);
    const int64_t tile = (int64_t)kThreads * pl.geo.spl;
    const int groups = (P + pl.geo.cpg - 1) / pl.geo.cpg;
    const int64_t ntiles = (blk.n + tile - 1) / tile;
    const int64_t units = ntiles * groups;
    pl.de_threads = pow2_at_least(P);

    // layout in the array: descriptor | rows (P x kStride) | partials (P x ntiles)
    constexpr size_t kDescBytes = 1024;
    static_assert(sizeof(BlockDesc) <= kDescBytes, "descriptor slot too small");
    const size_t row_bytes = ((size_t)P * kStride * sizeof(double) + 255) & ~(size_t)255;
    const size_t need = kDescBytes + row_bytes + (size_t)P * (size_t)ntiles * sizeof(double);
    if (need > (size_t)PT_NOALLOC_SCRATCH_BYTES)
        return fail(PT_EINVAL,
                    "pt_objective_noalloc: P = %d and n = %lld need %zu bytes of device memory, more than the "
                    "%zu-byte array (P x ceil(n / %lld) partial sums must fit)",
                    P, (long long)blk.n, need, (size_t)PT_NOALLOC_SCRATCH_BYTES, (long long)tile);
    BlockDesc* dd = reinterpret_cast<BlockDesc*>(ctx->noalloc);
    double* rows = reinterpret_cast<double*>(ctx->noalloc + kDescBytes);
    double* part = reinterpret_cast<double*>(ctx->noalloc + kDescBytes + row_bytes);
    BlockDesc d = base_desc(blk, &de, (int)ntiles, groups);
    d.trial = rows;
    d.pop = rows;
    d.partials = part;

    const ObjKernel obj = objective_kernel(pl.dtype, pl.geo, pl.mode, pl.slope);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, d, dd);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_pack_rows, dim3(1), dim3(256), 0, s, pop, rows, P);
    HIPCHK(hipGetLastError());
    launch_objective(obj, (unsigned)((units + 7) / 8 * 8), 0, s, (const BlockDesc*)dd, 1, (int)units, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_out, dim3(1), dim3(pl.de_threads), pl.de_threads * sizeof(double), s,
                       (const BlockDesc*)dd, out);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    ctx->last_arith = pl.mode;
    ctx->last_geo = pl.geo;
    return PT_OK;
}

int pt_time_objective(pt_ctx* ctx, const pt_block* block, const double* pop, int P, int precision, int reps,
                      void* hip_stream, double* avg_ms) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (!avg_ms) return fail(PT_EINVAL, "avg_ms is null");
    if (reps < 1 || reps > 100000) return fail(PT_EINVAL, "reps = %d outside [1, 100000]", reps);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    Plan pl;
    ObjKernel obj = nullptr;
    int rc = eval_setup(ctx, block, pop, P, precision, PT_OBJ_CHI2, s, &pl, &obj);
    if (rc) return rc;
    const BlockDesc* d = static_cast<const BlockDesc*>(ctx->desc.p);
    launch_objective(obj, pl.grid, 0, s, d, 1, pl.total_units, 0);  // warm
    HIPCHK(hipGetLastError());
    hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx);
    if (!e0 || !e1) return fail(PT_EDEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch_objective(obj, pl.grid, 0, s, d, 1, pl.total_units, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ctx->ev_free.push_back(e0);
    ctx->ev_free.push_back(e1);
    *avg_ms = (double)ms / reps;
    return PT_OK;
}

int pt_last_population(pt_ctx* ctx, int index, double* pop_host, double* fpop_host, int P) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (index < 0 || index >= ctx->last_nblk) return fail(PT_EINVAL, "index %d outside the last fit", index);
    if (P != ctx->last_P) return fail(PT_EINVAL, "P = %d, last fit used %d", P, ctx->last_P);
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    if (pop_host) {
        // whole rows, then the slots (a strided 2-D copy to host memory has
        // returned wrong data under the profiler on this runtime)
        const double* src = static_cast<const double*>(ctx->pop.p) + (size_t)index * P * kStride;
        std::vector<double> rows((size_t)P * kStride);
        HIPCHK(hipMemcpy(rows.data(), src, rows.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int p = 0; p < P; ++p)
            for (int j = 0; j < PT_NSLOT; ++j) pop_host[(size_t)p * PT_NSLOT + j] = rows[(size_t)p * kStride + j];
    }
    if (fpop_host) {
        const double* src = static_cast<const double*>(ctx->fpop.p) + (size_t)index * P;
        HIPCHK(hipMemcpy(fpop_host, src, sizeof(double) * P, hipMemcpyDeviceToHost));
    }
    return PT_OK;
}

int pt_last_history(pt_ctx* ctx, int index, double* hist_host, int n, int* count) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (index < 0 || index >= ctx->last_nblk) return fail(PT_EINVAL, "index %d outside the last fit", index);
    if (!hist_host || n < 0) return fail(PT_EINVAL, "hist_host is null or n < 0");
    const int avail = ctx->last_gens[index] + 1;
    const int k = std::min(n, avail);
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipDeviceSynchronize());
    const double* src = static_cast<const double*>(ctx->hist.p) + (size_t)index * (ctx->last_maxg + 1);
    if (k) HIPCHK(hipMemcpy(hist_host, src, sizeof(double) * k, hipMemcpyDeviceToHost));
    if (count) *count = k;
    return PT_OK;
}

// ------------------------------------------------------ derived observables
// phi(t) [rad] and F(t) [Hz] of a fit (Eq. 3-1-1, with the quartic term of slot 6)
static double fit_phase(const pt_fit* f, double t) {
    const double* c = f->coef;
    return c[1] + 2.0 * M_PI * (c[2] * t + c[3] * t * t / 2.0 + c[4] * t * t * t / 6.0 + c[6] * t * t * t * t / 24.0);
}
static double fit_freq(const pt_fit* f, double t) {
    const double* c = f->coef;
    return c[2] + c[3] * t + c[4] * t * t / 2.0 + c[6] * t * t * t / 6.0;
}

int pt_phase(const pt_fit* fit, const double* t, int64_t n, double* phase, double* phase_mod2pi, double* freq_hz,
             double* fdot_hz_s) {
    if (!fit) return fail(PT_EINVAL, "fit is null");
    if (n < 0 || (n > 0 && !t)) return fail(PT_EINVAL, "t is null or n < 0");
    const double two_pi = 2.0 * M_PI;
    for (int64_t k = 0; k < n; ++k) {
        const double tk = t[k];
        const double p = fit_phase(fit, tk);
        if (phase) phase[k] = p;
        if (phase_mod2pi) {
            double r = std::fmod(p, two_pi);
            phase_mod2pi[k] = r < 0 ? r + two_pi : r;
        }
        if (freq_hz) freq_hz[k] = fit_freq(fit, tk);
        if (fdot_hz_s) fdot_hz_s[k] = fit->coef[3] + fit->coef[4] * tk + fit->coef[6] * tk * tk / 2.0;
    }
    return PT_OK;
}

int pt_total_phase(const pt_fit* fit, double t_start, double t_end, double* dphi_rad, double* f_int_rad_s) {
    if (!fit) return fail(PT_EINVAL, "fit is null");
    if (!(t_end != t_start)) return fail(PT_EINVAL, "t_end must differ from t_start");
    const double d = fit_phase(fit, t_end) - fit_phase(fit, t_start);
    if (dphi_rad) *dphi_rad = d;
    if (f_int_rad_s) *f_int_rad_s = d / (t_end - t_start);
    return PT_OK;
}

int pt_connect_phase(const pt_fit* fits, int nblk, double* phi_total_rad, double* f_int_rad_s) {
    if (!fits || nblk < 1) return fail(PT_EINVAL, "fits is null or nblk < 1");
    double tot = 0.0, Tc = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const pt_fit* f = &fits[b];
        if (!(f->t_right > f->t_left)) return fail(PT_EINVAL, "fit %d: t_right <= t_left", b);
        tot += fit_phase(f, f->t_right) - fit_phase(f, f->t_left);
        Tc += f->t_right - f->t_left;
    }
    if (phi_total_rad) *phi_total_rad = tot;
    if (f_int_rad_s) *f_int_rad_s = tot / Tc;
    return PT_OK;
}

int pt_los_accel(const pt_fit* fit, double t, double f_carrier_hz, double M2, int three_way, double* a_m_s2) {
    if (!fit || !a_m_s2) return fail(PT_EINVAL, "fit / a_m_s2 is null");
    if (!(f_carrier_hz > 0)) return fail(PT_EINVAL, "f_carrier must be > 0");
    if (three_way && !(M2 > 0)) return fail(PT_EINVAL, "M2 must be > 0 for three-way");
    const double c = 299792458.0;
    const double phi2 = 2.0 * M_PI * (fit->coef[3] + fit->coef[4] * t + fit->coef[6] * t * t / 2.0);  // rad/s^2
    const double k = three_way ? 4.0 * M_PI * M2 * f_carrier_hz : 2.0 * M_PI * f_carrier_hz;
    *a_m_s2 = phi2 * c / k;
    return PT_OK;
}

int pt_continuity(const pt_fit* a, const pt_fit* b, double* dphi_rad, double* dfreq_hz) {
    if (!a || !b) return fail(PT_EINVAL, "fit is null");
    const double ta = a->t_right, tb = b->t_left;
    const double d = fit_phase(a, ta) - fit_phase(b, tb);
    if (dphi_rad) *dphi_rad = std::remainder(d, 2.0 * M_PI);
    if (dfreq_hz) {
        *dfreq_hz = fit_freq(a, ta) - fit_freq(b, tb);
    }
    return PT_OK;
}

// ------------------------------------------------- range determination (seed)
int pt_seed_max_snippet(pt_ctx* ctx) { return ctx && ctx->seed_max_log ? 1 << ctx->seed_max_log : 0; }

int pt_seed_block(pt_ctx* ctx, const pt_block* block, const pt_seed_opts* opts, void* hip_stream, pt_seed* out) {
    if (!ctx || !block || !out) return fail(PT_EINVAL, "ctx / block / out is null");
    if (!block->samples) return fail(PT_EINVAL, "samples is null");
    if (block->dtype != PT_F32 && block->dtype != PT_F64) return fail(PT_EINVAL, "dtype %d", block->dtype);
    if (!(block->fs > 0) || !std::isfinite(block->fs)) return fail(PT_EINVAL, "fs must be > 0");
    if (!std::isnan(block->ref) && !std::isfinite(block->ref)) return fail(PT_EINVAL, "ref not finite");
    if (ctx->seed_max_log == 0) return fail(PT_EUNSUPPORTED, "device LDS too small for the spectrum kernel");
    const int maxM = 1 << ctx->seed_max_log;
    int M = opts && opts->snippet ? opts->snippet : std::min(4096, maxM);
    if (M < 64 || M > maxM || (M & (M - 1))) return fail(PT_EINVAL, "snippet %d: a power of two in [64, %d]", M, maxM);
    const int64_t n = block->n;
    if (n < M) return fail(PT_EINVAL, "block of %lld samples is shorter than one snippet (%d)", (long long)n, M);
    const int64_t spacing = opts && opts->spacing ? opts->spacing : n / 4;
    if (spacing < 1) return fail(PT_EINVAL, "spacing %lld < 1", (long long)spacing);
    const double ref = block_ref(block);
    SeedStarts st;
    for (int k = 0; k < 3; ++k) {
        const int64_t c = (int64_t)std::floor(ref) + (int64_t)(k - 1) * spacing;
        st.v[k] = c - M / 2;
        if (st.v[k] < 0 || st.v[k] + M > n)
            return fail(PT_EINVAL, "snippet %d [%lld, %lld) outside the block of %lld samples", k,
                        (long long)st.v[k], (long long)(st.v[k] + M), (long long)n);
    }
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t esz = block->dtype == PT_F64 ? 8 : 4;
    const void* src = block->samples;
    SeedStarts dst = st;
    int rc;
    if (!block->on_device) {
        // host samples: only the three snippets travel
        if ((rc = ctx->seed_stage.ensure(3 * (size_t)M * esz))) return rc;
        for (int k = 0; k < 3; ++k) {
            HIPCHK(hipMemcpyAsync(static_cast<char*>(ctx->seed_stage.p) + (size_t)k * M * esz,
                                  static_cast<const char*>(block->samples) + (size_t)st.v[k] * esz, (size_t)M * esz,
                                  hipMemcpyHostToDevice, s));
            dst.v[k] = (int64_t)k * M;
        }
        src = ctx->seed_stage.p;
    }
    if ((rc = ctx->seed_out.ensure(3 * sizeof(SeedSnippet))) || (rc = ctx->hseed.ensure(3 * sizeof(SeedSnippet))))
        return rc;
    int lg = 0;
    while ((1 << lg) < M) ++lg;
    const size_t lds = (size_t)16 * M;
    SeedSnippet* dout = static_cast<SeedSnippet*>(ctx->seed_out.p);
    if (block->dtype == PT_F64) {
        auto k = k_seed_spectrum<double>;
        if (lds > 65536) HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k, dim3(3), dim3(kSeedThreads), lds, s, static_cast<const double*>(src), dst, lg,
                           block->fs, dout);
    } else {
        auto k = k_seed_spectrum<float>;
        if (lds > 65536) HIPCHK(hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(k, dim3(3), dim3(kSeedThreads), lds, s, static_cast<const float*>(src), dst, lg,
                           block->fs, dout);
    }
    HIPCHK(hipGetLastError());
    SeedSnippet* h = static_cast<SeedSnippet*>(ctx->hseed.p);
    HIPCHK(hipMemcpyAsync(h, dout, 3 * sizeof(SeedSnippet), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    pt_seed r;
    std::memset(&r, 0, sizeof r);
    for (int k = 0; k < 3; ++k) {
        r.f[k] = h[k].f;
        r.amp[k] = h[k].amp;
        r.noise[k] = h[k].noise;
        r.bin[k] = h[k].bin;
        r.t[k] = ((double)st.v[k] + 0.5 * (M - 1) - ref) / block->fs;
    }
    r.snippet = M;
    const double dt = (double)spacing / block->fs;
    r.f1 = (r.f[2] - r.f[0]) / (2.0 * dt);
    r.f0 = r.f[1] - r.f1 * r.t[1];
    r.f2 = (r.f[2] - 2.0 * r.f[1] + r.f[0]) / (dt * dt);
    r.A = r.amp[1];
    r.sigma = r.noise[1];
    const double Ts = (double)M / block->fs;
    const double sdf = r.A > 0 ? std::sqrt(6.0) * r.sigma / (M_PI * r.A * Ts * std::sqrt((double)M)) : INFINITY;
    r.sd_f0 = sdf;
    r.sd_f1 = std::sqrt(2.0) * sdf / (2.0 * dt);
    r.sd_f2 = std::sqrt(6.0) * sdf / (dt * dt);
    r.sd_A = r.sigma * std::sqrt(2.0 / M);
    *out = r;
    return PT_OK;
}

int pt_seed_box(const pt_seed* sd, int rule, double nsig, double T, int slope, pt_box* out) {
    if (!sd || !out) return fail(PT_EINVAL, "seed / out is null");
    if (rule != PT_RANGE_PAPER && rule != PT_RANGE_SIGMA) return fail(PT_EINVAL, "range rule %d", rule);
    if (!(nsig >= 0) || !std::isfinite(nsig)) return fail(PT_EINVAL, "nsig must be finite and >= 0");
    if (!(T > 0) || !std::isfinite(T)) return fail(PT_EINVAL, "T must be > 0");
    if (!(sd->A > 0) || !std::isfinite(sd->sd_f0)) return fail(PT_EINVAL, "seed has no signal estimate");
    double half[PT_NSLOT], mid[PT_NSLOT];
    mid[0] = sd->A;
    mid[1] = M_PI;
    half[1] = M_PI;
    mid[2] = sd->f0;
    mid[3] = sd->f1;
    mid[5] = 0.0;
    half[5] = slope ? 0.2 * sd->A / T : 0.0;
    mid[6] = 0.0;  // seeding gives no estimate of f3: the cubic model
    half[6] = 0.0;
    if (rule == PT_RANGE_PAPER) {
        half[0] = 0.1 * sd->A;
        half[2] = 0.1 * std::fabs(sd->f0);
        half[3] = std::max(0.1 * std::fabs(sd->f1), nsig * sd->sd_f1);
        mid[4] = 0.0;
        half[4] = 150.0 / M_PI;  // c3 = pi f2 / 3 in [-50, 50] rad/s^3
    } else {
        half[0] = std::max(0.1 * sd->A, nsig * sd->sd_A);
        half[2] = nsig * sd->sd_f0;
        half[3] = nsig * sd->sd_f1;
        mid[4] = sd->f2;
        half[4] = nsig * sd->sd_f2;
    }
    for (int j = 0; j < PT_NSLOT; ++j) {
        out->lo[j] = mid[j] - half[j];
        out->hi[j] = mid[j] + half[j];
    }
    return PT_OK;
}

// ------------------------------------------------------------ instrumentation
int pt_ctx_set_launch_mode(pt_ctx* ctx, int mode) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (mode != PT_LAUNCH_AUTO && mode != PT_LAUNCH_GRAPH && mode != PT_LAUNCH_PERSISTENT)
        return fail(PT_EINVAL, "launch mode %d", mode);
    ctx->launch_mode = mode;
    return PT_OK;
}

int pt_ctx_set_fp64_method(pt_ctx* ctx, int method) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (method != PT_FP64_AUTO && method != PT_FP64_POLY) return fail(PT_EINVAL, "fp64 method %d", method);
    ctx->fp64_method = method;
    return PT_OK;
}

int pt_ctx_last_launch(pt_ctx* ctx, int* mode) {
    if (!ctx || !mode) return fail(PT_EINVAL, "ctx / mode is null");
    *mode = ctx->last_launch;
    return PT_OK;
}

int pt_ctx_set_step_fusion(pt_ctx* ctx, int mode) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (mode != PT_FUSION_OFF && mode != PT_FUSION_LEAD && mode != PT_FUSION_LAST && mode != PT_FUSION_AUTO)
        return fail(PT_EINVAL, "step fusion %d", mode);
    ctx->step_fusion = mode;
    return PT_OK;
}

int pt_ctx_last_fit_launches(pt_ctx* ctx, int64_t* launches) {
    if (!ctx || !launches) return fail(PT_EINVAL, "ctx / launches is null");
    *launches = ctx->last_fit_launches;
    return PT_OK;
}

int pt_ctx_last_arithmetic(pt_ctx* ctx, int* arith) {
    if (!ctx || !arith) return fail(PT_EINVAL, "ctx / arith is null");
    *arith = ctx->last_arith;
    return PT_OK;
}

int pt_ctx_last_geometry(pt_ctx* ctx, int* spl, int* cpg) {
    if (!ctx || !spl || !cpg) return fail(PT_EINVAL, "ctx / spl / cpg is null");
    *spl = ctx->last_geo.spl;
    *cpg = ctx->last_geo.cpg;
    return PT_OK;
}

int pt_ctx_set_timing(pt_ctx* ctx, int on) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    ctx->timing = on != 0;
    ctx->launches = 0;
    ctx->total_ms = 0.0;
    return PT_OK;
}

int pt_ctx_kernel_stats(pt_ctx* ctx, int64_t* launches, double* total_ms) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (launches) *launches = ctx->launches;
    if (total_ms) *total_ms = ctx->total_ms;
    return PT_OK;
}

int pt_ctx_get_tile(pt_ctx* ctx, int64_t n, int P, int precision, int* spl, int* cpg) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (n < 1 || P < 1) return fail(PT_EINVAL, "n and P must be positive");
    Geometry g = choose_geometry(ctx, n, P, precision == PT_PREC_MIXED);
    if (spl) *spl = g.spl;
    if (cpg) *cpg = g.cpg;
    return PT_OK;
}

int pt_ctx_set_tile(pt_ctx* ctx, int spl, int cpg) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (spl == 0 && cpg == 0) {
        ctx->forced = {0, 0};
        return PT_OK;
    }
    if (!spl_ok(spl) || !cpg_ok(cpg)) return fail(PT_EINVAL, "unsupported geometry (%d, %d)", spl, cpg);
    ctx->forced = {spl, cpg};
    return PT_OK;
}

int pt_ctx_autotune(pt_ctx* ctx, int64_t n, int P, int precision, void* hip_stream, int* best_spl, int* best_cpg) {
    if (!ctx) return fail(PT_EINVAL, "ctx is null");
    if (n < 8 || n > ((int64_t)1 << 31) || P < 4 || P > PT_MAX_POP) return fail(PT_EINVAL, "n or P out of range");
    if (precision != PT_PREC_FP64 && precision != PT_PREC_MIXED) return fail(PT_EINVAL, "precision %d", precision);
    HIPCHK(hipSetDevice(ctx->device));
    // synthetic FP32 block (values only matter for timing)
    int rc;
    if ((rc = ctx->tune_block.ensure((size_t)n * 4))) return rc;
    std::vector<float> hs((size_t)std::min<int64_t>(n, 1 << 20));
    for (size_t k = 0; k < hs.size(); ++k) hs[k] = (float)std::cos(0.37 * (double)k);
    for (int64_t off = 0; off < n; off += (int64_t)hs.size()) {
        const size_t cnt = (size_t)std::min<int64_t>((int64_t)hs.size(), n - off);
        HIPCHK(hipMemcpy(static_cast<float*>(ctx->tune_block.p) + off, hs.data(), cnt * 4, hipMemcpyHostToDevice));
    }
    // a box around one carrier with the paper's widths and the largest drift
    // rate and drift acceleration of the paper-scale synthetic blocks
    // (5 Hz/s, 0.05 Hz/s^2), so that every
    // geometry is timed with the arithmetic the phasor bounds allow it at the
    // edge of a paper-scale box; a geometry whose bounds only hold for slow
    // drifts would otherwise win here and run the per-sample cosine in a fit
    pt_block b;
    std::memset(&b, 0, sizeof b);
    b.samples = ctx->tune_block.p;
    b.n = n;
    b.dtype = PT_F32;
    b.on_device = 1;
    b.fs = 50000.0;
    b.ref = NAN;
    const double lo[PT_NSLOT] = {0.8, 0.0, 1000.0, 4.8, -0.05, 0.0, 0.0};
    const double hi[PT_NSLOT] = {1.2, 6.28, 1001.0, 5.0, 0.05, 0.0, 0.0};
    for (int j = 0; j < PT_NSLOT; ++j) {
        b.box.lo[j] = lo[j];
        b.box.hi[j] = hi[j];
    }
    pt_de_settings de;
    std::memset(&de, 0, sizeof de);
    de.pop = P;
    de.max_gens = 100;
    de.F = 0.5;
    de.CR = 0.9;
    de.seed = 1;
    de.vtr = -INFINITY;
    de.precision = precision;
    de.objective = PT_OBJ_CHI2;
    const Geometry saved = ctx->forced;
    Geometry best{0, 0};
    double best_ms = 1e30;
    // per geometry: one untimed fit of 100 generations in the context's launch
    // form (builds its graphs), then two timed ones; the faster counts
    std::map<std::pair<int, int>, double> t;
    pt_fit fit;
    for (int spl : kSpl) {
        for (int cpg : kCpg) {
            ctx->forced = {spl, cpg};
            double ms = 1e30;
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                rc = run_fit(ctx, &b, 1, &de, hip_stream, &fit);
                const auto t1 = std::chrono::steady_clock::now();
                if (rep) ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
            }
            if (rc) break;
            t[std::make_pair(spl, cpg)] = ms;
        }
        if (rc) break;
    }
    for (int spl : kSpl) {
        for (int cpg : kCpg) {
            if (rc) break;
            const double ms = t[std::make_pair(spl, cpg)];
            if (ms < best_ms) {
                best_ms = ms;
                best = {spl, cpg};
            }
        }
        if (rc) break;
    }
    ctx->forced = saved;
    if (rc) return rc;
    ctx->tuned[std::make_tuple(size_class(n), P, precision == PT_PREC_MIXED ? 1 : 0)] = best;
    if (best_spl) *best_spl = best.spl;
    if (best_cpg) *best_cpg = best.cpg;
    return PT_OK;
}

}  // extern "C"

// ==================================================================== server
// Continuous batching of arriving blocks, run as a tracker (Sec. 3.1.1,
// 3.1.3).  Each admitted block owns a device slot (samples, population,
// partials, DE state).  A scheduler step runs `gens_per_step` generations of
// every active slot in shared launches (per objective arithmetic one grid
// over those slots' work units, then every slot's DE step); blocks admitted
// while others run join at the next step, and a block that meets its stop
// rule is checked (bound, continuity) and either retired, or re-initialised
// in a wider box and run again, in the step in which it stopped.  A track's
// next block waits for its previous block and starts from the last accepted
// fit (warm start).
struct pt_server {
    bool lead = false;  // leading-step launches (the context's step fusion was PT_FUSION_LEAD at creation)
    struct Slot {
        bool active = false, fresh = false;
        int track = -1;
        uint64_t ticket = 0;
        int gen = 0;
        int warm = 0;      // 0 given box, 1 warm start, 2 seeded
        int mode = 0;      // objective arithmetic of this block
        int attempts = 0;  // fits started for this block
        bool has_prev = false;  // `prev` is the accepted fit of the track's preceding block
        pt_fit prev{};
        double t_submit = 0.0;
        size_t bytes = 0;
        pt_block blk{};
        DevBuf samples, pop, trial, fpop, partials, hist, state;  // two slots each of pop ... state
        int lead = 0;  // leading-step form: launches this block has run since (re)initialisation
    };
    struct Pending {
        uint64_t ticket;
        int track;
        double t_submit;
        pt_block blk;
        std::vector<char> host;
    };
    struct Track {
        bool busy = false, has_fit = false;
        bool contiguous = false;  // the most recent block was accepted (it is `last`)
        pt_fit last{};            // last accepted fit
        double t_since = 0.0;     // seconds from last's reference sample to the end of the latest block
        double fs = 0.0;
    };
    pt_ctx* ctx = nullptr;
    pt_server_config cfg{};
    Geometry geo{16, 4};
    std::vector<Slot> slots;
    std::deque<Pending> pending;
    std::map<int, Track> tracks;
    std::deque<pt_server_result> done;
    size_t used_bytes = 0;
    uint64_t next_ticket = 1;
    DevBuf desc, rec;
    PinBuf hdesc, hrec, hstate;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// Phase of the previous fit re-expanded about the new block's reference
// time, dt seconds later: phi0 + 2 pi (f0 dt + f1 dt^2/2 + f2 dt^3/6 + f3 dt^4/24),
// f0 + f1 dt + f2 dt^2/2 + f3 dt^3/6, f1 + f2 dt + f3 dt^2/2, f2 + f3 dt, f3;
// amplitude A + Adot dt.
void predict(const double* c, double dt, double* out) {
    const double two_pi = 2.0 * M_PI;
    const double d2 = dt * dt, d3 = d2 * dt;
    double turns = c[2] * dt + c[3] * d2 / 2.0 + c[4] * d3 / 6.0 + c[6] * d3 * dt / 24.0;
    turns -= std::floor(turns);
    double ph = std::fmod(c[1] + two_pi * turns, two_pi);
    if (ph < 0) ph += two_pi;
    out[0] = c[0] + c[5] * dt;
    out[1] = ph;
    out[2] = c[2] + c[3] * dt + c[4] * d2 / 2.0 + c[6] * d3 / 6.0;
    out[3] = c[3] + c[4] * dt + c[6] * d2 / 2.0;
    out[4] = c[4] + c[6] * dt;
    out[5] = c[5];
    out[6] = c[6];
}

size_t slot_bytes(const pt_block& b, int P, int max_gens, int tile) {
    const size_t ntiles = (size_t)((b.n + tile - 1) / tile);
    return (size_t)b.n * (b.dtype == PT_F64 ? 8 : 4) + 2 * ((size_t)P * (2 * kStride + 1) * 8 + (size_t)P * ntiles * 8) +
           (size_t)(max_gens + 1) * 8 + 2 * sizeof(DeState);
}

// Objective arithmetic of one server block, from its own box only.
int slot_mode(const pt_server* sv, const pt_block& b) {
    if (sv->cfg.de.precision == PT_PREC_MIXED) return kModeMixed;
    if (sv->ctx->fp64_method == PT_FP64_POLY) return kModePoly;
    const double span = (double)b.n + std::fabs(b.ref);
    return phasor_ok(sv->geo.spl, b.fs, span, b.box.lo[2], b.box.hi[2], box_max(b.box, 3), box_max(b.box, 4),
                     box_max(b.box, 6))
               ? kModePhasor
               : kModePoly;
}

// Warm box of a track's next block around the prediction from its last fit.
void warm_box(const pt_server* sv, const pt_server::Track& tr, const pt_block& given, pt_block& b) {
    const double dt = tr.t_since + b.ref / b.fs;
    double pred[PT_NSLOT];
    predict(tr.last.coef, dt, pred);
    const double wn = sv->cfg.warm_narrow;
    for (int j = 0; j < PT_NSLOT; ++j) {
        const double half = 0.5 * (given.box.hi[j] - given.box.lo[j]);
        if (half > 0) {
            b.box.lo[j] = pred[j] - wn * half;
            b.box.hi[j] = pred[j] + wn * half;
        }
    }
    if (sv->cfg.range_rule != PT_RUN_EXTRAPOLATE) return;
    // Sec. 3.1.1 running range: frequency and rate over the new block's span
    const double* c = tr.last.coef;
    const double ta = tr.t_since, tb = tr.t_since + (double)b.n / b.fs;
    const double fa = fit_freq(&tr.last, ta), fb = fit_freq(&tr.last, tb);
    const double ra = c[3] + c[4] * ta + c[6] * ta * ta / 2.0, rb = c[3] + c[4] * tb + c[6] * tb * tb / 2.0;
    const double lo_v[2] = {std::min(fa, fb), std::min(ra, rb)}, hi_v[2] = {std::max(fa, fb), std::max(ra, rb)};
    for (int q = 0; q < 2; ++q) {
        const int j = 2 + q;
        const double half = 0.5 * (given.box.hi[j] - given.box.lo[j]);
        if (!(half > 0)) continue;
        const double mid = 0.5 * (lo_v[q] + hi_v[q]);
        b.box.lo[j] = std::min(lo_v[q], mid - wn * half);
        b.box.hi[j] = std::max(hi_v[q], mid + wn * half);
    }
    if (given.box.hi[0] > given.box.lo[0]) {
        b.box.lo[0] = pred[0] - 0.1 * std::fabs(pred[0]);
        b.box.hi[0] = pred[0] + 0.1 * std::fabs(pred[0]);
    }
}

// Snippet placement of the seeding step, or an error when it does not fit.
int seed_fits(const pt_block* b, int M) {
    const int64_t spacing = b->n / 4;
    const int64_t c = (int64_t)std::floor(block_ref(b));
    if (spacing < 1 || c - spacing - M / 2 < 0 || c + spacing + M / 2 > b->n)
        return fail(PT_EINVAL, "block of %lld samples is too short for seeding snippets of %d", (long long)b->n, M);
    return PT_OK;
}

int server_admit(pt_server* sv, hipStream_t s) {
    const int P = sv->cfg.de.pop;
    const int tile = kThreads * sv->geo.spl;
    for (auto it = sv->pending.begin(); it != sv->pending.end();) {
        pt_server::Track& tr = sv->tracks[it->track];
        if (tr.busy) {
            ++it;
            continue;
        }
        int free = -1;
        for (int k = 0; k < (int)sv->slots.size(); ++k)
            if (!sv->slots[k].active) {
                free = k;
                break;
            }
        const size_t need = slot_bytes(it->blk, P, sv->cfg.de.max_gens, tile);
        if (free < 0 || sv->used_bytes + need > sv->cfg.hbm_budget_bytes) break;  // no room now
        pt_server::Slot& sl = sv->slots[free];
        const size_t sbytes = (size_t)it->blk.n * (it->blk.dtype == PT_F64 ? 8 : 4);
        const size_t ntiles = (size_t)((it->blk.n + tile - 1) / tile);
        int rc;
        // two slots of the DE buffers (the leading-step form alternates between them)
        if ((rc = sl.samples.ensure(sbytes)) || (rc = sl.pop.ensure(2 * (size_t)P * kStride * 8)) ||
            (rc = sl.trial.ensure(2 * (size_t)P * kStride * 8)) || (rc = sl.fpop.ensure(2 * (size_t)P * 8)) ||
            (rc = sl.partials.ensure(2 * (size_t)P * ntiles * 8)) ||
            (rc = sl.hist.ensure((size_t)(sv->cfg.de.max_gens + 1) * 8)) ||
            (rc = sl.state.ensure(2 * sizeof(DeState))))
            return rc;
        HIPCHK(hipMemcpyAsync(sl.samples.p, it->host.data(), sbytes, hipMemcpyHostToDevice, s));
        sl.blk = it->blk;
        sl.blk.samples = sl.samples.p;
        sl.blk.on_device = 1;
        sl.blk.ref = block_ref(&it->blk);
        sl.warm = 0;
        sl.has_prev = false;
        if (tr.has_fit && sv->cfg.warm_narrow > 0.0 && tr.fs == it->blk.fs) {
            warm_box(sv, tr, it->blk, sl.blk);
            sl.warm = 1;
            sl.has_prev = tr.contiguous;
            sl.prev = tr.last;
        } else if (!tr.has_fit && sv->cfg.seed_first) {
            pt_seed_opts so{sv->cfg.seed_snippet, 0, 0};
            pt_seed sd;
            if ((rc = pt_seed_block(sv->ctx, &sl.blk, &so, s, &sd))) return rc;
            pt_box bx;
            const int slope = it->blk.box.lo[5] != it->blk.box.hi[5];
            if ((rc = pt_seed_box(&sd, PT_RANGE_SIGMA, sv->cfg.seed_nsig, (double)sl.blk.n / sl.blk.fs, slope, &bx)))
                return rc;
            for (int j = 0; j < PT_NSLOT; ++j)
                if (it->blk.box.lo[j] < it->blk.box.hi[j]) {  // slots the caller fixes stay fixed
                    sl.blk.box.lo[j] = bx.lo[j];
                    sl.blk.box.hi[j] = bx.hi[j];
                }
            sl.warm = 2;
        }
        sl.mode = slot_mode(sv, sl.blk);
        sl.attempts = 1;
        sl.active = true;
        sl.fresh = true;
        sl.track = it->track;
        sl.ticket = it->ticket;
        sl.t_submit = it->t_submit;
        sl.gen = 0;
        sl.bytes = need;
        sv->used_bytes += need;
        tr.busy = true;
        tr.fs = it->blk.fs;
        // the host copy can go once the stream has consumed it
        HIPCHK(hipStreamSynchronize(s));
        it = sv->pending.erase(it);
    }
    return PT_OK;
}

// Standard error of f2 [Hz/s^2] a block of the fitted amplitude and noise
// determines (Cramer-Rao bound of the phase coefficients phi0, f0, f1, f2 of
// a cosine in white noise): Fisher information (A^2 / 2 sigma^2) sum_n g g^T,
// g = (1, 2 pi t, pi t^2, pi t^3 / 3), with the time sums sum t^k taken as
// fs times the integral over the block's span; sigma^2 = chi^2 / n.
double sd_f2(const pt_fit& f, const pt_block& b) {
    const double n = (double)b.n, s2 = f.objective / n, A = std::fabs(f.coef[0]);
    if (!(A > 0) || !(s2 > 0)) return INFINITY;
    double m[7];  // sum over the block of t^k
    for (int k = 0; k <= 6; ++k)
        m[k] = b.fs * (std::pow(f.t_right, k + 1) - std::pow(f.t_left, k + 1)) / (k + 1);
    const double c[4] = {1.0, 2.0 * M_PI, M_PI, M_PI / 3.0};  // g_i = c_i t^i
    double J[4][5];
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) J[i][j] = c[i] * c[j] * m[i + j] * A * A / (2.0 * s2);
        J[i][4] = i == 3 ? 1.0 : 0.0;  // solve J x = e_3: x_3 = (J^-1)_33
    }
    for (int col = 0; col < 4; ++col) {  // Gauss-Jordan with partial pivoting
        int piv = col;
        for (int r = col + 1; r < 4; ++r)
            if (std::fabs(J[r][col]) > std::fabs(J[piv][col])) piv = r;
        if (!(std::fabs(J[piv][col]) > 0)) return INFINITY;
        for (int k = 0; k < 5; ++k) std::swap(J[col][k], J[piv][k]);
        for (int r = 0; r < 4; ++r) {
            if (r == col) continue;
            const double q = J[r][col] / J[col][col];
            for (int k = col; k < 5; ++k) J[r][k] -= q * J[col][k];
        }
    }
    const double v = J[3][4] / J[3][3];
    return v > 0 ? std::sqrt(v) : INFINITY;
}

// Widen a failed block's box for its next attempt (same centres).
void enlarge_box(pt_box& b, double k) {
    for (int j = 0; j < PT_NSLOT; ++j) {
        double half = 0.5 * (b.hi[j] - b.lo[j]);
        if (!(half > 0)) continue;
        const double mid = 0.5 * (b.lo[j] + b.hi[j]);
        half *= k;
        if (j == 1) half = std::min(half, M_PI);
        b.lo[j] = mid - half;
        b.hi[j] = mid + half;
    }
}

}  // namespace

extern "C" {

int pt_server_create(pt_ctx* ctx, const pt_server_config* cfg, pt_server** out) {
    if (!ctx || !cfg || !out) return fail(PT_EINVAL, "ctx / cfg / out is null");
    *out = nullptr;
    int rc = check_de(&cfg->de);
    if (rc) return rc;
    if (cfg->de.pop > 256) return fail(PT_EINVAL, "server population %d > 256", cfg->de.pop);
    if (cfg->max_slots < 1 || cfg->max_slots > 1024) return fail(PT_EINVAL, "max_slots %d", cfg->max_slots);
    if (cfg->gens_per_step < 1 || cfg->gens_per_step > 100000)
        return fail(PT_EINVAL, "gens_per_step %d", cfg->gens_per_step);
    if (cfg->max_pending < 1) return fail(PT_EINVAL, "max_pending %d", cfg->max_pending);
    if (!(cfg->warm_narrow >= 0.0 && cfg->warm_narrow <= 1.0)) return fail(PT_EINVAL, "warm_narrow outside [0, 1]");
    if (cfg->range_rule != PT_RUN_WARM && cfg->range_rule != PT_RUN_EXTRAPOLATE)
        return fail(PT_EINVAL, "range_rule %d", cfg->range_rule);
    if ((cfg->spl || cfg->cpg) && !(spl_ok(cfg->spl) && cpg_ok(cfg->cpg)))
        return fail(PT_EINVAL, "unsupported geometry (%d, %d)", cfg->spl, cfg->cpg);
    if (cfg->seed_first != 0 && cfg->seed_first != 1) return fail(PT_EINVAL, "seed_first %d", cfg->seed_first);
    if (cfg->seed_first) {
        const int maxM = pt_seed_max_snippet(ctx);
        const int M = cfg->seed_snippet;
        if (M && (M < 64 || M > maxM || (M & (M - 1))))
            return fail(PT_EINVAL, "seed_snippet %d: a power of two in [64, %d]", M, maxM);
        if (!(cfg->seed_nsig > 0) || !std::isfinite(cfg->seed_nsig)) return fail(PT_EINVAL, "seed_nsig must be > 0");
    }
    if (cfg->max_attempts < 0 || cfg->max_attempts > 16) return fail(PT_EINVAL, "max_attempts %d", cfg->max_attempts);
    if (cfg->max_attempts > 1 && !(cfg->enlarge >= 1.0 && std::isfinite(cfg->enlarge)))
        return fail(PT_EINVAL, "enlarge must be >= 1");
    if (!(cfg->qc_phase_rad >= 0) || !(cfg->qc_freq_hz >= 0)) return fail(PT_EINVAL, "qc limits must be >= 0");
    std::unique_ptr<pt_server> sv(new (std::nothrow) pt_server());
    if (!sv) return fail(PT_ENOMEM, "out of host memory");
    sv->ctx = ctx;
    sv->cfg = *cfg;
    if (sv->cfg.max_attempts == 0) sv->cfg.max_attempts = 1;
    sv->geo = cfg->spl ? Geometry{cfg->spl, cfg->cpg} : default_geometry(400000, cfg->de.pop);
    sv->lead = ctx->step_fusion == PT_FUSION_LEAD;
    sv->slots.resize(cfg->max_slots);
    *out = sv.release();
    return PT_OK;
}

void pt_server_destroy(pt_server* sv) {
    if (!sv) return;
    (void)hipSetDevice(sv->ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& sl : sv->slots) {
        DevBuf* b[] = {&sl.samples, &sl.pop, &sl.trial, &sl.fpop, &sl.partials, &sl.hist, &sl.state};
        for (DevBuf* x : b) x->release();
    }
    sv->desc.release();
    sv->rec.release();
    sv->hdesc.release();
    sv->hrec.release();
    sv->hstate.release();
    delete sv;
}

double pt_server_clock(pt_server* sv) { return sv ? sv->clock() : 0.0; }

int pt_server_submit(pt_server* sv, int32_t track, const pt_block* block, uint64_t* ticket) {
    if (!sv) return fail(PT_EINVAL, "server is null");
    int rc = check_block(block, 0);
    if (rc) return rc;
    if (sv->pending.size() >= (size_t)sv->cfg.max_pending) return fail(PT_EBUSY, "pending queue full");
    const int tile = kThreads * sv->geo.spl;
    if (slot_bytes(*block, sv->cfg.de.pop, sv->cfg.de.max_gens, tile) > sv->cfg.hbm_budget_bytes)
        return fail(PT_EINVAL, "block needs more than the whole HBM budget");
    if (sv->cfg.seed_first) {
        const int M = sv->cfg.seed_snippet ? sv->cfg.seed_snippet : std::min(4096, pt_seed_max_snippet(sv->ctx));
        if ((rc = seed_fits(block, M))) return rc;
    }
    pt_server::Pending pd;
    pd.ticket = sv->next_ticket++;
    pd.track = track;
    pd.t_submit = sv->clock();
    pd.blk = *block;
    const size_t bytes = (size_t)block->n * (block->dtype == PT_F64 ? 8 : 4);
    pd.host.resize(bytes);
    if (block->on_device) {
        HIPCHK(hipSetDevice(sv->ctx->device));
        HIPCHK(hipMemcpy(pd.host.data(), block->samples, bytes, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(pd.host.data(), block->samples, bytes);
    }
    pd.blk.samples = nullptr;
    sv->pending.push_back(std::move(pd));
    if (ticket) *ticket = sv->pending.back().ticket;
    return PT_OK;
}

int pt_server_step(pt_server* sv, void* hip_stream, int32_t* n_active, int32_t* n_pending) {
    if (!sv) return fail(PT_EINVAL, "server is null");
    pt_ctx* ctx = sv->ctx;
    HIPCHK(hipSetDevice(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int rc = server_admit(sv, s);
    if (rc) return rc;
    // active slots, grouped by objective kernel (arithmetic, dtype, slope)
    auto kernel_key = [&](int k) {
        const pt_server::Slot& sl = sv->slots[k];
        const bool slope = sl.blk.box.lo[5] != 0.0 || sl.blk.box.hi[5] != 0.0;
        return std::make_tuple(sl.mode, sl.blk.dtype, (int)slope);
    };
    std::vector<int> act;
    for (int k = 0; k < (int)sv->slots.size(); ++k)
        if (sv->slots[k].active) act.push_back(k);
    std::stable_sort(act.begin(), act.end(), [&](int a, int b) { return kernel_key(a) < kernel_key(b); });
    const int nb = (int)act.size();
    if (n_pending) *n_pending = (int)sv->pending.size();
    if (nb == 0) {
        if (n_active) *n_active = 0;
        return PT_OK;
    }
    const int P = sv->cfg.de.pop;
    const pt_de_settings& de = sv->cfg.de;
    const int tile = kThreads * sv->geo.spl;
    const int groups = (P + sv->geo.cpg - 1) / sv->geo.cpg;
    if ((rc = sv->desc.ensure(sizeof(BlockDesc) * nb)) || (rc = sv->hdesc.ensure(sizeof(BlockDesc) * nb)) ||
        (rc = sv->rec.ensure(sizeof(FitRecord) * nb)) || (rc = sv->hrec.ensure(sizeof(FitRecord) * nb)) ||
        (rc = sv->hstate.ensure(2 * sizeof(DeState) * nb)))
        return rc;
    // With step fusion PT_FUSION_LEAD (and P <= 256): one launch per
    // generation with the leading DE step; each block's launch index is its
    // descriptor's gen_begin plus the launch index within this step.
    // Otherwise objective and DE step as two launches (the default: with
    // many resident blocks the steps are throughput-bound, and the serving
    // run measured p99 25 ms this way against 36 ms with the leading step,
    // p50 3.2 against 3.0 ms).  The form is fixed for the server's lifetime
    // in practice: a block's buffers are laid out for one form, so the
    // setting must not change while blocks are resident.
    const unsigned de_threads = pow2_at_least(P);
    const bool lead = de_threads == (unsigned)kThreads && sv->lead;
    BlockDesc* hd = static_cast<BlockDesc*>(sv->hdesc.p);
    struct Launch {
        int first, count, units;
        ObjKernel k;
    };
    std::vector<Launch> launches;
    bool any_fresh = false;
    for (int q = 0; q < nb; ++q) {
        pt_server::Slot& sl = sv->slots[act[q]];
        const pt_block& B = sl.blk;
        if (launches.empty() || kernel_key(act[q]) != kernel_key(act[launches.back().first])) {
            const auto key = kernel_key(act[q]);
            launches.push_back({q, 0, 0, objective_kernel(std::get<1>(key), sv->geo, std::get<0>(key),
                                                          std::get<2>(key) != 0, lead)});
        }
        Launch& L = launches.back();
        BlockDesc d;
        std::memset(&d, 0, sizeof d);
        d.samples = B.samples;
        d.n = B.n;
        d.fs = B.fs;
        d.ref = B.ref;
        d.dtype = B.dtype;
        d.P = P;
        int D = 0;
        for (int j = 0; j < kSlots; ++j) {
            d.lo[j] = B.box.lo[j];
            d.hi[j] = B.box.hi[j];
            if (B.box.lo[j] < B.box.hi[j]) {
                d.act[D++] = j;
                d.amask |= 1 << j;
            }
        }
        d.D = D;
        d.ntiles = (int)((B.n + tile - 1) / tile);
        d.ngroups = groups;
        d.unit_begin = L.units;  // units count from the start of this block's launch group
        L.units += d.ntiles * groups;
        ++L.count;
        d.window = de.window;
        d.max_gens = de.max_gens;
        d.F = de.F;
        d.CR = de.CR;
        d.vtr = de.vtr;
        d.rel_tol = de.rel_tol;
        d.seed = de.seed;
        d.stream = B.stream;
        d.pop = static_cast<double*>(sl.pop.p);
        d.trial = static_cast<double*>(sl.trial.p);
        d.fpop = static_cast<double*>(sl.fpop.p);
        d.partials = static_cast<double*>(sl.partials.p);
        d.hist = static_cast<double*>(sl.hist.p);
        d.st = static_cast<DeState*>(sl.state.p);
        d.sync = nullptr;
        d.gen_begin = sl.gen;
        if (lead) {
            d.pop2 = d.pop + (size_t)P * kStride;
            d.trial2 = d.trial + (size_t)P * kStride;
            d.fpop2 = d.fpop + P;
            d.partials2 = d.partials + (size_t)P * d.ntiles;
            d.st2 = d.st + 1;
            d.gen_begin = sl.fresh ? 0 : sl.lead;
        }
        d.objective = de.objective;
        d.fresh = sl.fresh ? 1 : 0;  // k_de_init_fresh initialises only these
        any_fresh = any_fresh || sl.fresh;
        hd[q] = d;
    }
    HIPCHK(hipMemcpyAsync(sv->desc.p, hd, sizeof(BlockDesc) * nb, hipMemcpyHostToDevice, s));
    const BlockDesc* dd = static_cast<const BlockDesc*>(sv->desc.p);
    const size_t de_lds = (size_t)P * kSlots * 8 + (size_t)de_threads * (8 + 8 + 4);
    if (any_fresh) {
        hipLaunchKernelGGL(k_de_init_fresh, dim3(nb), dim3(de_threads), 0, s, dd);
        HIPCHK(hipGetLastError());
    }
    const int K = sv->cfg.gens_per_step;
    for (int k = 0; k < K; ++k) {
        if (lead) {
            for (const Launch& L : launches) {
                const int grid = (L.units + L.count + 7) / 8 * 8;  // plus one bookkeeping unit per block
                launch_objective(L.k, grid, de_lds + (size_t)P * kSlots * 8, s, dd + L.first, L.count, L.units,
                                 2 + k);
            }
            continue;
        }
        for (const Launch& L : launches) {
            const int grid = (L.units + 7) / 8 * 8;
            launch_objective(L.k, grid, 0, s, dd + L.first, L.count, L.units, 0);
        }
        hipLaunchKernelGGL(k_de_step, dim3(nb), dim3(de_threads), de_lds, s, dd);
    }
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_finalize, dim3(nb), dim3(64), 0, s, dd, static_cast<FitRecord*>(sv->rec.p));
    HIPCHK(hipGetLastError());
    DeState* hst = static_cast<DeState*>(sv->hstate.p);
    for (int q = 0; q < nb; ++q)
        HIPCHK(hipMemcpyAsync(hst + 2 * q, sv->slots[act[q]].state.p, (lead ? 2 : 1) * sizeof(DeState),
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(sv->hrec.p, sv->rec.p, sizeof(FitRecord) * nb, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double now = sv->clock();
    const FitRecord* r = static_cast<const FitRecord*>(sv->hrec.p);
    const pt_server_config& cf = sv->cfg;
    const bool qc_on = cf.qc_phase_rad > 0 || cf.qc_freq_hz > 0;
    int still = 0;
    for (int q = 0; q < nb; ++q) {
        pt_server::Slot& sl = sv->slots[act[q]];
        // the block's current state: in the leading-step form the slot holding
        // the stop, else the one the next launch would read
        const int L0 = sl.fresh ? 0 : sl.lead;
        const DeState& cur = !lead ? hst[2 * q]
                             : hst[2 * q].done ? hst[2 * q]
                             : hst[2 * q + 1].done ? hst[2 * q + 1]
                                                   : hst[2 * q + ((L0 + K) & 1)];
        sl.fresh = false;
        sl.gen = cur.gen;
        sl.lead = L0 + K;
        if (!cur.done) {
            ++still;
            continue;
        }
        pt_fit f;
        std::memset(&f, 0, sizeof f);
        for (int j = 0; j < PT_NSLOT; ++j) f.coef[j] = r[q].x[j];
        f.objective = r[q].f;
        f.generations = r[q].gens;
        f.flags = r[q].flags;
        f.ref = sl.blk.ref;
        f.t_left = (0.0 - f.ref) / sl.blk.fs;
        f.t_right = ((double)sl.blk.n - f.ref) / sl.blk.fs;
        derive(&f);
        int qc = 0;
        double dphi = 0.0, dfreq = 0.0;
        if (qc_on && sl.has_prev) {
            pt_continuity(&sl.prev, &f, &dphi, &dfreq);
            const bool bad = (cf.qc_phase_rad > 0 && !(std::fabs(dphi) <= cf.qc_phase_rad)) ||
                             (cf.qc_freq_hz > 0 && !(std::fabs(dfreq) <= cf.qc_freq_hz));
            qc = bad ? -1 : 1;
        }
        // a missed range: the best member on a bound of A, f0 or f1, or of f2
        // when the block determines f2 to better than a quarter of its box's
        // half-width (on short blocks f2 and Adot are noise-dominated and may
        // sit on their bounds; on long ones an f2 pressed against a bound
        // pulls f0, which correlates with it)
        bool miss = false;
        auto on_bound = [&](int j) {
            const double w = sl.blk.box.hi[j] - sl.blk.box.lo[j];
            return w > 0 && (f.coef[j] - sl.blk.box.lo[j] <= 1e-6 * w || sl.blk.box.hi[j] - f.coef[j] <= 1e-6 * w);
        };
        for (int j : {0, 2, 3})
            if (on_bound(j)) miss = true;
        if (on_bound(4) && 0.5 * (sl.blk.box.hi[4] - sl.blk.box.lo[4]) > 4.0 * sd_f2(f, sl.blk)) miss = true;
        const bool policy = cf.max_attempts > 1 || qc_on;  // otherwise every fit is accepted as it is
        const bool failed = policy && (miss || qc < 0);
        if (failed && sl.attempts < cf.max_attempts) {
            // Sec. 3.1.1: enlarge the range and search again
            enlarge_box(sl.blk.box, cf.enlarge);
            sl.mode = slot_mode(sv, sl.blk);
            ++sl.attempts;
            sl.fresh = true;
            sl.gen = 0;
            ++still;
            continue;
        }
        pt_server_result res;
        std::memset(&res, 0, sizeof res);
        res.ticket = sl.ticket;
        res.track = sl.track;
        res.warm = sl.warm;
        res.t_submit = sl.t_submit;
        res.t_done = now;
        res.box = sl.blk.box;
        if (failed) f.flags |= PT_FLAG_ABANDONED | (qc < 0 ? PT_FLAG_DISCONTINUOUS : 0);
        res.fit = f;
        res.attempts = sl.attempts;
        res.qc = qc;
        res.border_dphi = dphi;
        res.border_dfreq = dfreq;
        sv->done.push_back(res);
        pt_server::Track& tr = sv->tracks[sl.track];
        tr.busy = false;
        if (!failed) {
            tr.has_fit = true;
            tr.contiguous = true;
            tr.last = f;
            tr.t_since = f.t_right;
        } else {
            tr.contiguous = false;
            tr.t_since += (double)sl.blk.n / sl.blk.fs;
        }
        sv->used_bytes -= sl.bytes;
        sl.active = false;
    }
    if (n_active) *n_active = still;
    return PT_OK;
}

int pt_server_poll(pt_server* sv, pt_server_result* out, int32_t max, int32_t* n_out) {
    if (!sv || (!out && max > 0) || max < 0) return fail(PT_EINVAL, "server / out is null or max < 0");
    int k = 0;
    while (k < max && !sv->done.empty()) {
        out[k++] = sv->done.front();
        sv->done.pop_front();
    }
    if (n_out) *n_out = k;
    return PT_OK;
}

int pt_server_stats(pt_server* sv, int32_t* active, int32_t* pending, uint64_t* used_bytes) {
    if (!sv) return fail(PT_EINVAL, "server is null");
    int a = 0;
    for (auto& sl : sv->slots) a += sl.active;
    if (active) *active = a;
    if (pending) *pending = (int)sv->pending.size();
    if (used_bytes) *used_bytes = sv->used_bytes;
    return PT_OK;
}

}  // extern "C"
