"""Benchmark: full DE fits of a 400 000-sample block on one MI355X.

One step = one complete fit of the paper-scale block (400 000 FP32 samples
at 50 kHz, cubic phase, SNR 0 dB; DE/rand/1/bin with P = 40, F = 0.5,
CR = 0.9 and 2000 generations, i.e. 40 x 2001 objective evaluations over
all samples), starting from samples already resident in HBM and ending with
the fitted record (coefficients + derived observables) on the host.

Printed (one JSON line): candidate*sample evaluations per second of the
plain FP64 path, fit latency p50 / p99 of the plain and mixed-precision
paths, the mixed path's speedup and error against the FP64 oracle, the
objective kernel's roofline figures (HIP-event timing of its launches inside
a fit) and the CPU oracle's rate on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published, counts packed FP32)
# Unpacked FP32 issues at the FP64 instruction rate on this part (measured:
# 75 TFLOP/s for either with dependent-free FMA streams); this build does not
# form packed FP32 instructions, so the FP32 path's reachable peak is 78.6.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
VALU_ISSUE_SLOTS_PER_S = 1024 * 2.4e9 / 4.0  # wave64 VALU instructions: 1024 SIMDs, one per 4 cycles
# Algorithmic work per candidate*sample: the survey's figure for one direct
# evaluation of Eq. (2-2-2)/(2-2-4) -- the cubic phase (3 FMA), one cosine
# (12-16 FMA after the turn reduction), the residual FMA and the
# square-accumulate FMA -- about 40 FP64 FLOP.  Every arithmetic computes
# that objective and is credited the same work (the phasor path executes 12
# to 15 FP64 operations per candidate*sample, an FMA counted as two, so its
# algorithmic rate is an equivalent rate and can exceed the hardware peak);
# `executed` gives the counter-measured FP64 operations of the same launches.
ALG_FLOP = 40
ARITH_NAME = {0: "fp64-per-sample", 1: "mixed", 2: "fp64-phasor"}

from paper_1906_10598_amd.rocprof_summary import executed_flop, kernel_hash, read_profile  # noqa: E402

PROFILES = os.path.join(ROOT, "profiles")


def profile_of(name, workload, geometry, form):
    return read_profile(os.path.join(PROFILES, name), workload, geometry, form)


def executed_roofline(prof, launch_ms, peak=PEAK_FP64_TFLOPS):
    """Counter-measured FP64 / FP32 operations and VALU issue of a kernel (per
    dispatch, from its committed rocprofv3 summary) at the launch time measured
    here; None when no summary matches the current kernel sources."""
    if not prof or "fma_f64" not in prof or not launch_ms:
        return None
    f64, f32 = executed_flop(prof)
    t = launch_ms * 1e-3
    out = {"fp64_tflops": f64 / t / 1e12, "fp64_frac": f64 / t / 1e12 / peak,
           "fp32_tflops": f32 / t / 1e12, "fp64_flop_per_launch": f64, "fp32_flop_per_launch": f32,
           "source": "rocprofv3 SQ_INSTS_VALU_{FMA,ADD,MUL,TRANS}_{F64,F32} x 64 lanes (FMA x 2) per dispatch, "
                     "committed summary of the same kernel, divided by the launch time measured here"}
    if "valu" in prof:
        out["valu_issue"] = prof["valu"] / (VALU_ISSUE_SLOTS_PER_S * t)
    if prof.get("bytes_per_launch"):
        # achieved HBM rate: the counter traffic of the same summary over the launch time
        out["hbm_gb_s"] = prof["bytes_per_launch"] / t / 1e9
        out["hbm_frac"] = out["hbm_gb_s"] / PEAK_HBM_GBS
    return out


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def run_fits(ctx, blk, de_fn, n, label, events=None):
    """n fits; wall seconds, per-fit latencies [ms], fits.  events: a list that
    receives the GPU time [ms] between HIP events recorded on the fits' stream
    (torch's current stream) around the whole region."""
    import torch

    lat = []
    fits = []
    torch.cuda.synchronize()
    if events is not None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
    t0 = time.perf_counter()
    for k in range(n):
        t1 = time.perf_counter()
        fits.append(ctx.fit_block(blk, de_fn(k)))
        lat.append((time.perf_counter() - t1) * 1e3)
    if events is not None:
        e1.record()
    torch.cuda.synchronize()
    if events is not None:
        events.append(e0.elapsed_time(e1))
    return time.perf_counter() - t0, lat, fits


def run_serving(ctx, ptk, synth, np, torch, nblocks, crlb_f0_block, refit=True):
    """16 tracks, Poisson arrivals at 20 blocks/s, N in {1e5, 2e5, 4e5, 1e6}.

    Blocks are submitted when their arrival time has passed on the server
    clock; latency = completion - arrival.  Window stop rule (1e-9 over 50
    generations, cap 3000), warm starts with a 30 % narrower box.  With
    `refit`, every accepted block is fitted again afterwards in the box the
    server used, for a fixed 2000 generations (same seed and stream), to show
    what the window rule's early stop costs in f0."""
    items = synth.config4_stream(seed=0, ntracks=16, nblocks=nblocks, rate=20.0)
    de = ptk.make_settings(pop=40, max_gens=3000, F=0.5, CR=0.9, seed=0x19061059 ^ 0xDE, rel_tol=1e-9, window=50)
    cfg = ptk.make_server_config(de, max_slots=64, gens_per_step=32, hbm_budget_bytes=64 << 30, max_attempts=3,
                                 enlarge=2.0, qc_phase_rad=0.5, qc_freq_hz=0.1)
    srv = ptk.pt_server_create(ctx.handle, cfg)
    stream = ptk.current_stream()
    host = [torch.from_numpy(it["block"].samples) for it in items]
    blks = [ptk.make_block(h, it["block"].fs, it["block"].lo, it["block"].hi, ref=it["block"].ref,
                           stream=it["block"].stream) for h, it in zip(host, items)]
    t0 = ptk.pt_server_clock(srv)
    nxt, res, tick = 0, {}, {}
    active = pending = 0
    steps = 0
    while len(res) < len(items):
        now = ptk.pt_server_clock(srv) - t0
        while nxt < len(items) and items[nxt]["arrival"] <= now:
            t = ptk.pt_server_submit(srv, items[nxt]["track"], blks[nxt])
            if t is None:
                break
            tick[t] = nxt
            nxt += 1
        if active or pending or nxt > len(res):
            active, pending = ptk.pt_server_step(srv, stream)
            steps += 1
        elif nxt < len(items):
            time.sleep(max(0.0, min(0.002, items[nxt]["arrival"] - now)))
        for r in ptk.pt_server_poll(srv):
            res[tick[r.ticket]] = r
    elapsed = ptk.pt_server_clock(srv) - t0
    ptk.pt_server_destroy(srv)
    lat, errs, gens, warm, retried, abandoned, qc_fail = [], [], [], 0, 0, 0, 0
    served_vs_fixed, fixed_errs, work = [], [], 0.0
    for k, it in enumerate(items):
        r = res[k]
        lat.append((r.t_done - t0 - it["arrival"]) * 1e3)
        b = it["block"]
        work += 40.0 * (r.fit.generations + 1) * b.n
        gens.append(r.fit.generations)
        warm += r.warm == 1
        retried += r.attempts > 1
        abandoned += bool(r.fit.flags & ptk.PT_FLAG_ABANDONED)
        qc_fail += r.qc < 0
        if r.fit.flags & ptk.PT_FLAG_ABANDONED:
            continue
        sig = crlb_f0_block(b)
        errs.append(abs(r.fit.coef[2] - b.truth[2]) / sig)
        if refit:
            lo, hi = np.array(r.box.lo), np.array(r.box.hi)
            fx = ctx.fit_block(ptk.make_block(host[k].cuda(), b.fs, lo, hi, ref=b.ref, stream=b.stream),
                               ptk.make_settings(pop=40, max_gens=2000, F=0.5, CR=0.9, seed=de.seed))
            served_vs_fixed.append(abs(r.fit.coef[2] - fx.coef[2]) / sig)
            fixed_errs.append(abs(fx.coef[2] - b.truth[2]) / sig)
    out = {"workload": f"{len(items)} blocks from 16 tracks, Poisson arrivals at 20 blocks/s, N in "
                       "{1e5, 2e5, 4e5, 1e6} at 50 kHz, window stop 1e-9/50 (cap 3000), warm starts 0.7x box, "
                       "up to 3 fits per block (range x2 per retry), continuity limits 0.5 rad / 0.1 Hz",
           "retried_blocks": retried, "abandoned_blocks": abandoned, "continuity_failures": qc_fail,
           "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)},
           "blocks_per_s": len(items) / elapsed, "offered_blocks_per_s": 20.0,
           "f0_err_over_crlb": {"median": pct(errs, 50), "p99": pct(errs, 99), "max": max(errs),
                                "of_accepted_blocks": len(errs),
                                "crlb": "Cramer-Rao bound over the parameters the box frees (A, phi0, f0, f1, f2)"},
           "generations": {"mean": float(sum(gens) / len(gens)), "p50": pct(gens, 50), "max": max(gens)},
           "warm_fraction": warm / len(items), "scheduler_steps": steps,
           "candidate_samples_per_s": work / elapsed}
    if refit:
        out["early_stop"] = {
            "served_minus_fixed_2000_gen_f0_over_crlb": {"median": pct(served_vs_fixed, 50),
                                                         "p99": pct(served_vs_fixed, 99),
                                                         "max": max(served_vs_fixed)},
            "fixed_2000_gen_f0_err_over_crlb": {"median": pct(fixed_errs, 50), "p99": pct(fixed_errs, 99),
                                                "max": max(fixed_errs)},
            "what": "each accepted block fitted again in the box the server used, 2000 generations, same seed "
                    "and stream; |f0 served - f0 fixed| in CRLB units measures what the window rule's stop costs"}
    return out


def objective_comparison(ctx, ptk, synth, np, torch, nseeds):
    """Chi-square (Eq. 2-2-4) against the correlation objective (Eq. 2-2-5
    with the constant-amplitude model of Eq. 2-2-6) on paper-scale blocks.

    Both fits run 2000 generations from the same seed; the correlation fit
    fixes A at the block's RMS amplitude sqrt(2 mean s^2) (its optimum does
    not depend on that scale).  Convergence generation: first g with
    best[g] - best[G] <= 1e-3 (best[0] - best[G]) on the best-so-far history."""
    from synth.crlb import crlb_f0_block

    out = {"chi2": {"gens": [], "ms_per_gen": [], "f0_err_over_crlb": []},
           "cor": {"gens": [], "ms_per_gen": [], "f0_err_over_crlb": []}}
    for seed in range(nseeds):
        b = synth.config1(seed)
        dev = torch.from_numpy(b.samples).cuda()
        a_rms = math.sqrt(2.0 * float(np.mean(b.samples.astype(np.float64) ** 2)))
        lo_c, hi_c = b.lo.copy(), b.hi.copy()
        lo_c[0] = hi_c[0] = a_rms
        sig = crlb_f0_block(b)
        for name, kind, lo, hi in (("chi2", ptk.PT_OBJ_CHI2, b.lo, b.hi), ("cor", ptk.PT_OBJ_COR, lo_c, hi_c)):
            blk = ptk.make_block(dev, b.fs, lo, hi, ref=b.ref, stream=b.stream)
            de = ptk.make_settings(pop=b.de.pop, max_gens=b.de.max_gens, F=b.de.F, CR=b.de.CR, seed=b.de.seed,
                                   objective=kind)
            ctx.fit_block(blk, de)  # warm (graph capture)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f = ctx.fit_block(blk, de)
            dt = time.perf_counter() - t0
            h = ptk.pt_last_history(ctx.handle, 0, f.generations + 1)
            drop = h[0] - h[-1]
            g = int(np.argmax(h - h[-1] <= 1e-3 * drop)) if drop > 0 else 0
            out[name]["gens"].append(g)
            out[name]["ms_per_gen"].append(dt * 1e3 / (f.generations + 1))
            out[name]["f0_err_over_crlb"].append(abs(f.coef[2] - b.truth[2]) / sig)
    res = {"workload": f"{nseeds} paper-scale blocks (400000 samples, 50 kHz, 0 dB), P=40, 2000 generations; "
                       "correlation fit with A fixed at the RMS amplitude",
           "convergence": "first generation within 1e-3 of the total decrease of the best-so-far objective"}
    for name, v in out.items():
        res[name] = {"median_gens_to_converge": pct(v["gens"], 50), "max_gens_to_converge": max(v["gens"]),
                     "ms_per_generation": pct(v["ms_per_gen"], 50),
                     "f0_err_over_crlb": {"median": pct(v["f0_err_over_crlb"], 50),
                                          "max": max(v["f0_err_over_crlb"])}}
    res["cor_gens_over_chi2_gens"] = (res["cor"]["median_gens_to_converge"] /
                                      max(res["chi2"]["median_gens_to_converge"], 1))
    res["cor_cost_per_gen_over_chi2"] = res["cor"]["ms_per_generation"] / res["chi2"]["ms_per_generation"]
    return res


def quartic_fit(ctx, ptk, synth, np, torch):
    """Perigee-like 20 s block (1e6 samples) with the fourth Taylor order
    (Sec. 3.2.1): the quartic fit (f3 active) against the cubic one."""
    b = synth.config_quartic(3)
    dev = torch.from_numpy(b.samples).cuda()
    de = ptk.make_settings(pop=b.de.pop, max_gens=b.de.max_gens, F=b.de.F, CR=b.de.CR, seed=b.de.seed)
    blk = ptk.make_block(dev, b.fs, b.lo, b.hi, ref=b.ref, stream=b.stream)
    ctx.fit_block(blk, de)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q = ctx.fit_block(blk, de)
    dt = time.perf_counter() - t0
    arith = ARITH_NAME[ptk.pt_ctx_last_arithmetic(ctx.handle)]
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[6] = hi[6] = 0.0
    lo[4], hi[4] = b.truth[4] - 0.05, b.truth[4] + 0.05
    c = ctx.fit_block(ptk.make_block(dev, b.fs, lo, hi, ref=b.ref, stream=b.stream), de)
    noise = b.n * b.sigma ** 2
    return {"workload": "1e6 samples at 50 kHz (20 s), quartic phase, 0 dB; P=40, 2000 generations",
            "fit_ms": dt * 1e3, "candidate_samples_per_s": b.de.pop * (b.de.max_gens + 1) * b.n / dt,
            "arithmetic": arith, "f3_truth": float(b.truth[6]), "f3_fit": q.coef[6],
            "chi2_over_noise": {"quartic": q.objective / noise, "cubic": c.objective / noise}}


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, and the x86 family /
    model / stepping numbers (a virtual machine may print only a vendor
    string as the name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # first processor only
                k, _, v = line.partition(":")
                info[k.strip()] = v.strip()
    except OSError:
        return None
    name = info.get("model name")
    if name is None:
        return None
    ids = [f"{k} {info[k]}" for k in ("cpu family", "model", "stepping") if k in info]
    return f"{name} ({', '.join(ids)})" if ids else name


def cpu_baseline(b, gens, nthreads):
    """The oracle's fit of the same block over its first `gens` generations:
    candidate*samples per second and seconds."""
    import numpy as np

    import oracle

    s64 = b.samples.astype(np.float64)
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.de_fit(s64, b.fs, b.ref, b.lo, b.hi, b.de.pop, gens, F=b.de.F, CR=b.de.CR, seed=b.de.seed,
                      stream=b.stream, nthreads=nthreads)
    dt = time.perf_counter() - t0
    pairs = b.de.pop * (r["generations"] + 1) * b.n
    return pairs / dt, dt


def batch_fits(ctx, ptk, synth, np, torch, P, seed, crlb_f0_block, tiles):
    """64 uneven blocks, own populations, shared launches (FP64 and mixed)."""
    batch = {}
    blocks = synth.config3(0)
    bdev = [torch.from_numpy(x.samples).cuda() for x in blocks]
    pbs = [ptk.make_block(d, x.fs, x.lo, x.hi, ref=x.ref, stream=x.stream) for x, d in zip(blocks, bdev)]
    gens_b = blocks[0].de.max_gens
    pairs_b = sum(P * (gens_b + 1) * x.n for x in blocks)
    for name, prec in (("fp64", ptk.PT_PREC_FP64), ("mixed", ptk.PT_PREC_MIXED)):
        deb = ptk.make_settings(pop=P, max_gens=gens_b, F=0.5, CR=0.9, seed=seed, precision=prec)
        ctx.fit_batch(pbs, deb)  # warm (graph capture for this shape)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fits_b = ctx.fit_batch(pbs, deb)
        dt = time.perf_counter() - t0
        errs = [abs(f.coef[2] - x.truth[2]) / crlb_f0_block(x) for f, x in zip(fits_b, blocks)]
        geo = list(ptk.pt_ctx_last_geometry(ctx.handle))
        ach = ALG_FLOP * pairs_b / dt / 1e12
        batch[name] = {"value": pairs_b / dt, "unit": "candidate*sample/s", "seconds": dt,
                       "block_fits_per_s": len(blocks) / dt,
                       "f0_err_over_crlb": {"median": pct(errs, 50), "p99": pct(errs, 99), "max": max(errs)},
                       "geometry": geo,
                       "roofline": {"bound": "alu", "unit": "TFLOP/s", "peak": PEAK_FP64_TFLOPS,
                                    "achieved": ach, "frac": ach / PEAK_FP64_TFLOPS,
                                    "flop_per_candidate_sample": ALG_FLOP,
                                    "note": "whole-batch algorithmic rate (40 FLOP per candidate*sample over the "
                                            "wall time of the batch, DE steps and launch gaps included); above 1 "
                                            "because the FP64 phasor arithmetic executes ~12 FP64 operations per "
                                            "candidate*sample for the same result (`executed` gives the counter "
                                            "rate); the mixed path's per-sample FP32 cosine executes ~27 FP32 and ~2 FP64"}}
    batch["workload"] = ("64 blocks, N log-uniform in [5e4, 4e5] at 50 kHz (total %d samples), own "
                         "populations P=40, 1500 generations, one launch per generation" % sum(x.n for x in blocks))
    g = batch["fp64"]["geometry"]
    prof = profile_of("batch_last_64blocks_%dx%d.md" % tuple(g), "batch-64", g, "batch-last")
    if prof.get("avg_us"):
        ex = executed_roofline(prof, prof["avg_us"] * 1e-3)
        if ex:
            ex["kernel"] = ("k_objective (FP64 phasor, last-workgroup DE step) as the 64-block batch launches it, "
                            "per dispatch, profile time")
            ex["avg_launch_ms"] = prof["avg_us"] * 1e-3
        batch["fp64"]["roofline"]["executed"] = ex
        batch["fp64"]["roofline"]["traffic"] = prof.get("bytes_per_launch")
    return batch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--latency-fits", type=int, default=100, help="fits per path for p50/p99")
    ap.add_argument("--cpu-gens", type=int, default=800, help="oracle generations in the CPU sample")
    ap.add_argument("--cpu-gens-1t", type=int, default=40,
                    help="oracle generations in the single-thread CPU sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tile", default="", help="force the objective geometry, e.g. 16,4")
    ap.add_argument("--kernel-only", default="", choices=["", "fp64", "mixed"],
                    help="profiling mode: one fit, then --reps back-to-back objective launches; "
                         "also one 256 MiB device copy as the traffic-counter calibration")
    ap.add_argument("--reps", type=int, default=200)
    ap.add_argument("--launch", default="auto", choices=["auto", "graph", "persistent"],
                    help="launch strategy of the fits (pt_ctx_set_launch_mode)")
    ap.add_argument("--fusion", default="auto", choices=["auto", "lead", "last", "off"],
                    help="where a graph-launched fit runs its DE step (pt_ctx_set_step_fusion)")
    ap.add_argument("--fit-only", action="store_true",
                    help="profiling mode: --warmup + --steps fits of the paper-scale block (FP64, default "
                         "launch form), then one JSON line with the fit times")
    ap.add_argument("--batch-only", action="store_true",
                    help="profiling mode: the 64-block batch (FP64) once warm and once timed")
    ap.add_argument("--serve-only", action="store_true",
                    help="profiling mode: the serving run alone (no refits)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-block batched fits")
    ap.add_argument("--no-serve", action="store_true", help="skip the real-time serving run")
    ap.add_argument("--serve-blocks", type=int, default=160)
    ap.add_argument("--no-objcmp", action="store_true", help="skip the chi-square vs correlation comparison")
    ap.add_argument("--objcmp-seeds", type=int, default=8)
    ap.add_argument("--no-quartic", action="store_true", help="skip the quartic (perigee) fit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the fit of one block does not shard; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1906_10598_amd import phasetrack as ptk
    from synth.crlb import crlb_f0_block

    b = synth.config1(0)
    P, G, N = b.de.pop, b.de.max_gens, b.n
    pairs_per_fit = P * (G + 1) * N
    dev = torch.from_numpy(b.samples).cuda()
    ctx = ptk.Context(0)
    blk = ptk.make_block(dev, b.fs, b.lo, b.hi, ref=b.ref, stream=b.stream)
    stream = ptk.current_stream()

    def calibration_copy():
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)  # traffic-counter calibration: reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        return 2 * src.numel() * 4

    # launch form of the fits (the autotuner times fits in this form)
    ptk.pt_ctx_set_launch_mode(ctx.handle, {"auto": ptk.PT_LAUNCH_AUTO, "graph": ptk.PT_LAUNCH_GRAPH,
                                            "persistent": ptk.PT_LAUNCH_PERSISTENT}[args.launch])
    ptk.pt_ctx_set_step_fusion(ctx.handle, {"auto": ptk.PT_FUSION_AUTO, "lead": ptk.PT_FUSION_LEAD,
                                            "last": ptk.PT_FUSION_LAST, "off": ptk.PT_FUSION_OFF}[args.fusion])
    tiles = {}
    if args.tile:
        spl, cpg = (int(v) for v in args.tile.split(","))
        ptk.pt_ctx_set_tile(ctx.handle, spl, cpg)
    tune = not args.no_tune and not args.tile and not args.kernel_only and not args.serve_only
    for name, prec in (("fp64", ptk.PT_PREC_FP64), ("mixed", ptk.PT_PREC_MIXED)):
        if tune:
            ptk.pt_ctx_autotune(ctx.handle, N, P, prec, stream)
        tiles[name] = ptk.pt_ctx_get_tile(ctx.handle, N, P, prec)
    print(f"# geometry (samples/lane, candidates/workgroup): {tiles}", file=sys.stderr, flush=True)

    if args.kernel_only:
        prec = ptk.PT_PREC_FP64 if args.kernel_only == "fp64" else ptk.PT_PREC_MIXED
        # two-launch generations here, so every k_objective launch of this run is
        # the bare objective the roofline times
        ptk.pt_ctx_set_step_fusion(ctx.handle, ptk.PT_FUSION_OFF)
        ctx.fit_block(blk, ptk.make_settings(pop=P, max_gens=G, F=b.de.F, CR=b.de.CR, seed=b.de.seed,
                                             precision=prec))
        ptk.pt_ctx_set_step_fusion(ctx.handle, ptk.PT_FUSION_AUTO)
        pop, _ = ptk.pt_last_population(ctx.handle, 0, P)
        popd = torch.from_numpy(pop).cuda()
        torch.cuda.synchronize()
        avg_ms = ptk.pt_time_objective(ctx.handle, blk, popd.data_ptr(), P, prec, args.reps, stream)
        arith_k = ARITH_NAME[ptk.pt_ctx_last_arithmetic(ctx.handle)]
        cal = calibration_copy()
        print(json.dumps({"kernel_only": args.kernel_only, "avg_launch_ms": avg_ms, "reps": args.reps,
                          "arithmetic": arith_k, "geometry": tiles[args.kernel_only], "kernel_hash": kernel_hash(),
                          "calibration_copy_bytes": cal}), flush=True)
        ctx.close()
        return

    def de(prec):
        return lambda k: ptk.make_settings(pop=P, max_gens=G, F=b.de.F, CR=b.de.CR, seed=b.de.seed + k,
                                           precision=prec)

    if args.fit_only:
        run_fits(ctx, blk, de(ptk.PT_PREC_FP64), args.warmup, "warmup")
        el, lat, _ = run_fits(ctx, blk, de(ptk.PT_PREC_FP64), args.steps, "fp64")
        calibration_copy()
        print(json.dumps({"fit_only": True, "launch": args.launch, "fusion": args.fusion, "fits": args.steps,
                          "ms_per_fit": el / args.steps * 1e3,
                          "p50_ms": pct(lat, 50), "geometry": tiles["fp64"],
                          "arithmetic": ARITH_NAME[ptk.pt_ctx_last_arithmetic(ctx.handle)],
                          "kernel_hash": kernel_hash()}), flush=True)
        ctx.close()
        return

    if args.batch_only:
        out = batch_fits(ctx, ptk, synth, np, torch, P, b.de.seed, crlb_f0_block, tiles)
        calibration_copy()
        print(json.dumps({"batch_only": True, "fp64_seconds": out["fp64"]["seconds"],
                          "geometry": out["fp64"]["geometry"], "kernel_hash": kernel_hash()}), flush=True)
        ctx.close()
        return

    if args.serve_only:
        out = run_serving(ctx, ptk, synth, np, torch, args.serve_blocks, crlb_f0_block, refit=False)
        calibration_copy()
        print(json.dumps({"serve_only": True, "latency_ms": out["latency_ms"], "kernel_hash": kernel_hash()}),
              flush=True)
        ctx.close()
        return

    # ---- plain FP64: warmup + timed steps
    run_fits(ctx, blk, de(ptk.PT_PREC_FP64), args.warmup, "warmup")
    ev = []
    elapsed, lat_steps, fits64 = run_fits(ctx, blk, de(ptk.PT_PREC_FP64), args.steps, "fp64", events=ev)
    launches_per_fit = ptk.pt_ctx_fit_launches(ctx.handle)
    value = pairs_per_fit * args.steps / elapsed
    arith64 = ARITH_NAME[ptk.pt_ctx_last_arithmetic(ctx.handle)]
    print(f"# fp64: {args.steps} fits in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # ---- latency percentiles (distinct seeds), both paths
    extra = max(0, args.latency_fits - args.steps)
    _, lat_more, _ = run_fits(ctx, blk, lambda k: de(ptk.PT_PREC_FP64)(args.steps + k), extra, "fp64-lat")
    lat64 = lat_steps + lat_more
    # first fits of a fresh context at the same geometry: the first one captures
    # and instantiates the fit's launch graphs, the second replays them
    with ptk.Context(0) as cold:
        ptk.pt_ctx_set_tile(cold.handle, *tiles["fp64"])
        _, lat_cold, _ = run_fits(cold, blk, de(ptk.PT_PREC_FP64), 2, "fp64-cold")
    run_fits(ctx, blk, de(ptk.PT_PREC_MIXED), max(1, args.warmup), "mixed-warm")
    el_mx, lat_mx, fits_mx = run_fits(ctx, blk, de(ptk.PT_PREC_MIXED), max(args.latency_fits, 1), "mixed")
    value_mx = pairs_per_fit * len(lat_mx) / el_mx
    print(f"# mixed: {len(lat_mx)} fits in {el_mx:.3f} s", file=sys.stderr, flush=True)

    # ---- accuracy of both paths against the FP64 oracle (same seed as fit 0)
    import oracle

    s64 = b.samples.astype(np.float64)
    sig = crlb_f0_block(b)
    f64, fmx = fits64[0], fits_mx[0]
    chi_or = oracle.chi2(s64, b.fs, b.ref, list(fmx.coef))
    chi_or64 = oracle.chi2(s64, b.fs, b.ref, list(f64.coef))
    mixed_err = {
        "objective_rel_err": abs(fmx.objective - chi_or) / chi_or,
        "fp64_objective_rel_err": abs(f64.objective - chi_or64) / chi_or64,
        "f0_diff_hz": fmx.coef[2] - f64.coef[2],
        "f1_diff_hz_s": fmx.coef[3] - f64.coef[3],
        "f2_diff_hz_s2": fmx.coef[4] - f64.coef[4],
        "f0_err_vs_truth_over_crlb": {"fp64": (f64.coef[2] - b.truth[2]) / sig,
                                      "mixed": (fmx.coef[2] - b.truth[2]) / sig},
        "crlb_f0_hz": sig,
    }

    # ---- objective kernel alone: HIP events around back-to-back launches
    # (same geometry and grid as the fits, on the fit's final population)
    roof = {}
    for name, prec, method in (("fp64", ptk.PT_PREC_FP64, ptk.PT_FP64_AUTO),
                               ("fp64_per_sample", ptk.PT_PREC_FP64, ptk.PT_FP64_POLY),
                               ("mixed", ptk.PT_PREC_MIXED, ptk.PT_FP64_AUTO)):
        ptk.pt_ctx_set_fp64_method(ctx.handle, method)
        ctx.fit_block(blk, de(prec)(0))
        pop, _ = ptk.pt_last_population(ctx.handle, 0, P)
        popd = torch.from_numpy(pop).cuda()
        avg_ms = ptk.pt_time_objective(ctx.handle, blk, popd.data_ptr(), P, prec, 400, stream)
        arith = ptk.pt_ctx_last_arithmetic(ctx.handle)
        ptk.pt_ctx_set_fp64_method(ctx.handle, ptk.PT_FP64_AUTO)
        ach = ALG_FLOP * P * N / (avg_ms * 1e-3) / 1e12
        roof[name] = {"avg_launch_ms": avg_ms, "achieved": ach, "frac": ach / PEAK_FP64_TFLOPS,
                      "arithmetic": ARITH_NAME[arith]}
    obj_prof = profile_of("k_objective_fp64_paper400k_%dx%d.md" % tuple(tiles["fp64"]), "paper-400000-fp32",
                          tiles["fp64"], "objective")
    mx_prof = profile_of("k_objective_mixed_paper400k_%dx%d.md" % tuple(tiles["mixed"]), "paper-400000-fp32",
                         tiles["mixed"], "objective")
    fit_prof = profile_of("fit_lead_paper400k_%dx%d.md" % tuple(tiles["fp64"]), "paper-400000-fp32",
                          tiles["fp64"], "fit-lead")

    # the kernel as the timed fits launch it: HIP events around the timed region
    # on the fits' stream, divided by the launches it held (every launch but each
    # fit's last one evaluates the population: ALG_FLOP * P * N)
    fit_launch_ms = ev[0] / (args.steps * launches_per_fit)
    fit_ach = ALG_FLOP * pairs_per_fit * args.steps / (ev[0] * 1e-3) / 1e12

    batch = None
    if not args.no_batch:
        batch = batch_fits(ctx, ptk, synth, np, torch, P, b.de.seed, crlb_f0_block, tiles)
        print(f"# batch: {batch['fp64']['seconds']:.3f} s fp64, {batch['mixed']['seconds']:.3f} s mixed",
              file=sys.stderr, flush=True)

    serving = None
    if not args.no_serve:
        serving = run_serving(ctx, ptk, synth, np, torch, args.serve_blocks, crlb_f0_block)
        ach = ALG_FLOP * serving["candidate_samples_per_s"] / 1e12
        serving["roofline"] = {"bound": "arrivals", "unit": "TFLOP/s", "peak": PEAK_FP64_TFLOPS, "achieved": ach,
                               "frac": ach / PEAK_FP64_TFLOPS, "flop_per_candidate_sample": ALG_FLOP,
                               "note": "algorithmic work of the served fits over the run's wall time: the offered "
                                       "load (20 blocks/s) sets it, not the kernels; `step_kernel` is the objective "
                                       "launch the server makes, per dispatch"}
        sprof = profile_of("server_step_16tracks_16x4.md", "serving-16", (16, 4), "server")
        if sprof.get("avg_us"):
            ex = executed_roofline(sprof, sprof["avg_us"] * 1e-3)
            if ex:
                ex["avg_launch_ms"] = sprof["avg_us"] * 1e-3
                ex["kernel"] = "k_objective (16 x 4, objective alone) as the server launches it, profile time"
            serving["roofline"]["step_kernel"] = ex
        print(f"# serving: p50 {serving['latency_ms']['p50']:.1f} ms p99 {serving['latency_ms']['p99']:.1f} ms",
              file=sys.stderr, flush=True)

    objcmp = None
    if not args.no_objcmp:
        objcmp = objective_comparison(ctx, ptk, synth, np, torch, args.objcmp_seeds)
        print(f"# objectives: chi2 {objcmp['chi2']['median_gens_to_converge']} gens, "
              f"cor {objcmp['cor']['median_gens_to_converge']} gens", file=sys.stderr, flush=True)

    quartic = None
    if not args.no_quartic:
        quartic = quartic_fit(ctx, ptk, synth, np, torch)
        print(f"# quartic: {quartic['fit_ms']:.1f} ms per fit", file=sys.stderr, flush=True)

    # ---- CPU oracle baseline (bounded samples of the same fit, and the tiny fit)
    cpu = None
    if not args.no_cpu:
        import oracle as _oracle

        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
        rate, dt = cpu_baseline(b, args.cpu_gens, nthreads)
        rate1, dt1 = cpu_baseline(b, args.cpu_gens_1t, 1)
        b0 = synth.config0(0)
        t0 = time.perf_counter()
        _oracle.de_fit(b0.samples, b0.fs, b0.ref, b0.lo, b0.hi, b0.de.pop, b0.de.max_gens, F=b0.de.F,
                       CR=b0.de.CR, seed=b0.de.seed, stream=b0.stream, nthreads=nthreads)
        c0_s = time.perf_counter() - t0
        cpu = {"value": rate, "unit": "candidate*sample/s", "cores": nthreads, "kind": "oracle",
               "cpu_model": cpu_model(),
               "sample": f"first {args.cpu_gens} generations of the same 400000-sample fit "
                         f"(P=40, {40 * (args.cpu_gens + 1) * N:.3e} candidate*samples, {dt:.1f} s)",
               "single_thread": {"value": rate1, "sample": f"first {args.cpu_gens_1t} generations, 1 thread "
                                                           f"({dt1:.1f} s)"},
               "paper_scale_fit_s_extrapolated": pairs_per_fit / rate,
               "tiny_fit": {"workload": "4096 FP64 samples, P=32, 200 generations (whole fit)", "seconds": c0_s,
                            "threads": nthreads}}

    r64 = roof["fp64"]
    ex_fit = executed_roofline(fit_prof, fit_launch_ms)
    ex_obj = executed_roofline(obj_prof, r64["avg_launch_ms"])
    ex_mx = executed_roofline(mx_prof, roof["mixed"]["avg_launch_ms"], PEAK_FP32_UNPACKED_TFLOPS)
    line = {
        "metric": "candidate*sample evals/s + 400K-block fit p50/p99 latency, mixed vs plain FP64",
        "value": value,
        "unit": "candidate*sample/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper-scale block fit: N=400000 int16-quantised FP32 samples at 50 kHz, "
                               "cubic phase, SNR 0 dB; DE/rand/1/bin P=40, F=0.5, CR=0.9, 2000 generations",
                   "n_samples": N, "population": P, "generations": G, "precision": "fp64",
                   "arithmetic": arith64,
                   "geometry": {"samples_per_lane": tiles["fp64"][0], "cand_per_group": tiles["fp64"][1]}},
        "latency_ms": {
            "fp64": {"p50": pct(lat64, 50), "p99": pct(lat64, 99), "fits": len(lat64),
                     "first_fit_new_context": lat_cold[0], "second_fit_new_context": lat_cold[1]},
            "mixed": {"p50": pct(lat_mx, 50), "p99": pct(lat_mx, 99), "fits": len(lat_mx)},
        },
        "block_fits_per_s": {"fp64": args.steps / elapsed, "mixed": len(lat_mx) / el_mx},
        "mixed": {"value": value_mx, "speedup_vs_fp64": value_mx / value, **mixed_err,
                  "geometry": {"samples_per_lane": tiles["mixed"][0], "cand_per_group": tiles["mixed"][1]},
                  "roofline": {"bound": "alu", "achieved": roof["mixed"]["achieved"],
                               "peak": PEAK_FP32_UNPACKED_TFLOPS, "unit": "TFLOP/s",
                               "frac": roof["mixed"]["achieved"] / PEAK_FP32_UNPACKED_TFLOPS,
                               "peak_note": "unpacked FP32 (this build forms no packed FP32); published packed "
                                            "peak 157.3",
                               "avg_launch_ms": roof["mixed"]["avg_launch_ms"],
                               "traffic": mx_prof.get("bytes_per_launch"), "executed": ex_mx}},
        "roofline": {"bound": "alu", "achieved": fit_ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": fit_ach / PEAK_FP64_TFLOPS, "traffic": fit_prof.get("bytes_per_launch"),
                     "kernel": "k_objective (FP64, %s) as launched in the timed fits: one launch per "
                               "generation with the leading DE step" % arith64,
                     "avg_launch_ms": fit_launch_ms, "launches_per_fit": launches_per_fit,
                     "event_ms_timed_region": ev[0],
                     "flop_per_candidate_sample": ALG_FLOP, "kernel_hash": kernel_hash(),
                     "executed": ex_fit,
                     "objective_only": {"kernel": "k_objective (FP64, %s), objective alone" % r64["arithmetic"],
                                        "avg_launch_ms": r64["avg_launch_ms"], "achieved": r64["achieved"],
                                        "frac": r64["frac"], "traffic": obj_prof.get("bytes_per_launch"),
                                        "executed": ex_obj},
                     "fp64_per_sample_path": {k: roof["fp64_per_sample"][k] for k in
                                              ("avg_launch_ms", "achieved", "frac")}},
        "batch": batch,
        "serving": serving,
        "objective_comparison": objcmp,
        "quartic": quartic,
        "cpu_baseline": cpu,
        "paper_context": {"gtx580_fit_s": 6.5, "evaluations": 80000, "block": "~400K samples"},
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
