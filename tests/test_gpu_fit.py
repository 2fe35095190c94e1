"""GPU parity of the whole DE fit (pt_fit_block / pt_fit_batch) against the oracle.

Both sides draw the same Philox stream and apply the same DE/rand/1/bin
steps, so populations agree exactly until a selection compares two
objectives closer than their ~1e-13 disagreement.  The tests compare the
populations after the run, the best-so-far history (1e-10 relative) and
the recovered f0 (1e-6 Hz), and report how many members are bit-identical.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_chi2_close, block_of, crlb_f0, ctx, mixed_rel_at_optimum, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _oracle_fit(b: synth.Block, gens, **kw):
    de = b.de
    return oracle.de_fit(np.asarray(b.samples, dtype=np.float64), b.fs, b.ref, b.lo, b.hi, de.pop, gens,
                         F=de.F, CR=de.CR, seed=de.seed, stream=b.stream, vtr=kw.get("vtr", de.vtr),
                         rel_tol=kw.get("rel_tol", de.rel_tol), window=kw.get("window", de.window))


def _compare(b, gpu_fit, ref, P, label):
    pop, fpop = ptk.pt_last_population(ctx().handle, 0, P)
    hist = ptk.pt_last_history(ctx().handle, 0, ref["generations"] + 1)
    same = int(np.sum(np.all(pop == ref["pop"], axis=1)))
    print(f"[{label}] gens {gpu_fit.generations}/{ref['generations']} identical members {same}/{P} "
          f"best {gpu_fit.objective!r} vs {ref['objective']!r} "
          f"df0 {gpu_fit.coef[2] - ref['x'][2]:.3e}", flush=True)
    assert gpu_fit.generations == ref["generations"]
    assert gpu_fit.flags == ref["flags"]
    assert_chi2_close([gpu_fit.objective], [ref["objective"]], b.n)
    assert_chi2_close(hist, ref["hist"], b.n)
    assert abs(gpu_fit.coef[2] - ref["x"][2]) < 1e-6
    assert np.all(pop >= b.lo) and np.all(pop <= b.hi)
    return same


def test_tiny_block_fit_matches_oracle():
    for seed in range(3):
        b = synth.config0(seed)
        dev = to_dev(b.samples)
        # early generations: populations bit-identical
        f = ctx().fit_block(block_of(b, dev), settings_of(b, gens=30))
        ref = _oracle_fit(b, 30)
        assert _compare(b, f, ref, b.de.pop, f"tiny seed {seed} 30 gens") == b.de.pop
        # whole fit: history, best and f0 within tolerance
        f = ctx().fit_block(block_of(b, dev), settings_of(b))
        ref = _oracle_fit(b, b.de.max_gens)
        _compare(b, f, ref, b.de.pop, f"tiny seed {seed}")


def _populations(b, dev, gens):
    ctx().fit_block(block_of(b, dev), settings_of(b, gens=gens))
    gpu, _ = ptk.pt_last_population(ctx().handle, 0, b.de.pop)
    return gpu, _oracle_fit(b, gens)["pop"]


def test_trajectories_split_only_at_selection_near_ties():
    # Find the first generation at which GPU and oracle populations differ
    # and show that the differing selection compared a trial and a target
    # whose objectives agree to ~1e-12: a tie below the two sides' rounding
    # disagreement, not an arithmetic difference.
    b = synth.config0(0)
    dev = to_dev(b.samples)
    gmax = b.de.max_gens
    gpu, orc = _populations(b, dev, gmax)
    if np.array_equal(gpu, orc):
        return
    lo, hi = 0, gmax  # identical at lo (init is exact), different at hi
    while hi - lo > 1:
        mid = (lo + hi) // 2
        g_, o_ = _populations(b, dev, mid)
        if np.array_equal(g_, o_):
            lo = mid
        else:
            hi = mid
    prev, _ = _populations(b, dev, lo)
    g_hi, o_hi = _populations(b, dev, hi)
    s64 = np.asarray(b.samples, dtype=np.float64)
    act = oracle.active_slots(b.lo, b.hi)
    fprev = oracle.chi2_pop(s64, b.fs, b.ref, prev)
    rows = np.nonzero(np.any(g_hi != o_hi, axis=1))[0]
    print(f"[near-tie] first split at generation {hi}, members {rows.tolist()}", flush=True)
    for i in rows:
        r1, r2, r3, jr, U = oracle.de_draws(b.de.seed, b.stream, hi, int(i), b.de.pop, len(act))
        trial = oracle.de_trial(prev, int(i), r1, r2, r3, jr, U, act, b.de.F, b.de.CR, b.lo, b.hi)
        ft = oracle.chi2(s64, b.fs, b.ref, trial)
        gap = abs(ft - fprev[i]) / fprev[i]
        print(f"  member {i}: trial {ft!r} target {fprev[i]!r} rel gap {gap:.2e}", flush=True)
        assert gap < 1e-12


def test_paper_block_short_fit_matches_oracle():
    b = synth.config1(0)
    dev = to_dev(b.samples)
    f = ctx().fit_block(block_of(b, dev), settings_of(b, gens=25))
    ref = _oracle_fit(b, 25)
    same = _compare(b, f, ref, b.de.pop, "paper 25 gens")
    assert same == b.de.pop  # no near-ties this early


def test_paper_block_full_fit_sampled():
    # Full paper-scale run (400 000 samples, P = 40, 2000 generations) in the
    # benchmark's configuration; the oracle checks the reported objective of
    # the best member and of sampled members one by one.
    b = synth.config1(0)
    dev = to_dev(b.samples)
    f = ctx().fit_block(block_of(b, dev), settings_of(b))
    pop, fpop = ptk.pt_last_population(ctx().handle, 0, b.de.pop)
    s64 = b.samples.astype(np.float64)
    assert f.generations == 2000 and f.flags == ptk.PT_FLAG_MAXGEN
    best = np.array(f.coef)
    assert_chi2_close([f.objective], [oracle.chi2(s64, b.fs, b.ref, best)], b.n)
    idx = [0, 13, 27, 39]
    assert_chi2_close(fpop[idx], oracle.chi2_pop(s64, b.fs, b.ref, pop[idx]), b.n)
    assert np.all(pop >= b.lo) and np.all(pop <= b.hi)
    chi_truth = oracle.chi2(s64, b.fs, b.ref, b.truth)
    assert f.objective <= chi_truth
    sig = crlb_f0(b)
    print(f"[paper full] f0 err {f.coef[2] - b.truth[2]:.3e} Hz = {(f.coef[2] - b.truth[2]) / sig:+.2f} CRLB "
          f"({sig:.2e} Hz over A, phi0, f0, f1, f2), chi2 {f.objective:.6f} vs truth {chi_truth:.6f}", flush=True)
    assert abs(f.coef[2] - b.truth[2]) < 5 * sig


@pytest.mark.parametrize("seed", [0, 1])
def test_paper_block_whole_fit_matches_oracle_fit(seed):
    # The whole paper-scale fit (400 000 samples, P = 40, 2000 generations,
    # Sec. 1.3 / Table 4) against the oracle's whole fit of the same block and
    # the exact least-squares minimiser, both stored by
    # tests/golden/make_paper_fit.py (oracle only).  The two DE trajectories
    # part at the first selection near-tie, but both converge to the minimiser:
    # recovered f0 within 1e-6 Hz, best chi^2 within 1e-10 relative.
    g = json.load(open(os.path.join(GOLD, f"paper_fit_seed{seed}.json")))
    b = synth.config1(seed)
    assert g["n"] == b.n and g["de"]["seed"] == b.de.seed and g["de"]["max_gens"] == b.de.max_gens
    f = ctx().fit_block(block_of(b, to_dev(b.samples)), settings_of(b))
    ox, oobj = np.array(g["oracle_fit"]["x"]), g["oracle_fit"]["objective"]
    mx, mobj = np.array(g["minimiser"]["x"]), g["minimiser"]["objective"]
    sig = crlb_f0(b)
    print(f"[paper whole fit seed {seed}] gpu f0 - oracle f0 {f.coef[2] - ox[2]:+.3e} Hz, gpu f0 - minimiser "
          f"{f.coef[2] - mx[2]:+.3e} Hz, chi2 rel diff {(f.objective - oobj) / oobj:+.3e}; "
          f"f0 err vs truth {(f.coef[2] - b.truth[2]) / sig:+.2f} CRLB", flush=True)
    assert f.generations == g["oracle_fit"]["generations"] == 2000
    assert f.flags == g["oracle_fit"]["flags"]
    assert abs(f.coef[2] - ox[2]) < 1e-6
    assert abs(f.coef[2] - mx[2]) < 1e-6
    assert abs(f.objective - oobj) <= 1e-10 * oobj
    assert abs(f.objective - mobj) <= 1e-10 * mobj
    # f1 and f2 sit at the same optimum too (within 1e-4 of their box widths)
    for j, name in ((3, "f1"), (4, "f2")):
        assert abs(f.coef[j] - ox[j]) < 1e-4 * (b.hi[j] - b.lo[j]), name


def test_window_rule_and_vtr_match_oracle():
    b = synth.config0(4)
    dev = to_dev(b.samples)
    f = ctx().fit_block(block_of(b, dev), settings_of(b, gens=1500, rel_tol=1e-9, window=20))
    ref = _oracle_fit(b, 1500, rel_tol=1e-9, window=20)
    assert f.flags & ptk.PT_FLAG_CONVERGED
    _compare(b, f, ref, b.de.pop, "window rule")
    f = ctx().fit_block(block_of(b, dev), settings_of(b, vtr=1e9))
    assert f.generations == 0 and f.flags == ptk.PT_FLAG_VTR


def test_truth_outside_box_flags_at_bound():
    b = synth.config0(5)
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[2], hi[2] = b.truth[2] + 0.05, b.truth[2] + 2.0
    dev = to_dev(b.samples)
    f = ctx().fit_block(block_of(b, dev, lo=lo, hi=hi), settings_of(b, gens=150))
    assert f.flags & ptk.PT_FLAG_AT_BOUND


def test_fit_deterministic_and_stream_dependent():
    b = synth.config0(6)
    dev = to_dev(b.samples)
    f1 = ctx().fit_block(block_of(b, dev), settings_of(b, gens=40))
    f2 = ctx().fit_block(block_of(b, dev), settings_of(b, gens=40))
    f3 = ctx().fit_block(block_of(b, dev, stream=9), settings_of(b, gens=40))
    assert list(f1.coef) == list(f2.coef) and f1.objective == f2.objective
    assert list(f1.coef) != list(f3.coef)


def test_host_samples_match_device_samples():
    b = synth.config0(7)
    import torch

    host = torch.from_numpy(b.samples)
    f1 = ctx().fit_block(block_of(b, host), settings_of(b, gens=30))
    f2 = ctx().fit_block(block_of(b, to_dev(b.samples)), settings_of(b, gens=30))
    assert list(f1.coef) == list(f2.coef)


def test_batch_equals_alone():
    blocks = synth.config3(0, nblocks=6, gens=30)
    devs = [to_dev(b.samples) for b in blocks]
    pbs = [block_of(b, d) for b, d in zip(blocks, devs)]
    de = settings_of(blocks[0])
    c = ctx()
    ptk.pt_ctx_set_tile(c.handle, 16, 4)
    try:
        batch = c.fit_batch(pbs, de)
        alone = [c.fit_block(pb, de) for pb in pbs]
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
    for b, x, y in zip(blocks, batch, alone):
        assert list(x.coef) == list(y.coef) and x.objective == y.objective, b.name
    # and each block matches the oracle's own fit
    for b, x in zip(blocks[:2], batch[:2]):
        ref = _oracle_fit(b, 30)
        assert_chi2_close([x.objective], [ref["objective"]], b.n)


def test_derived_outputs_of_a_fit():
    b = synth.config0(8)
    f = ctx().fit_block(block_of(b, to_dev(b.samples)), settings_of(b, gens=60))
    c = oracle.derived.coefs_from_fit(f.coef[1], f.coef[2], f.coef[3], f.coef[4])
    T2 = b.n / b.fs / 2
    assert f.t_left == pytest.approx(-T2) and f.t_right == pytest.approx(T2)
    assert f.total_phase == pytest.approx(oracle.derived.block_total_phase(c, 2 * T2), rel=1e-13)
    assert abs(math.remainder(f.phase_left - float(oracle.derived.phase_mod2pi(c, -T2)), 2 * math.pi)) < 1e-9
    assert f.freq_right == pytest.approx(float(oracle.derived.freq_hz(c, T2)), rel=1e-14)


def test_amplitude_slope_fit_matches_oracle():
    # six-parameter fit with the amplitude slope c5 of Eq. (2-2-2) active
    rng = np.random.default_rng(17)
    n, fs = 20_000, 2_000.0
    t = (np.arange(n) - n / 2) / fs
    x = np.array([0.8, 1.9, 311.25, 0.75, 0.0, 0.06, 0.0])
    s = (x[0] + x[5] * t) * np.cos(x[1] + 2 * np.pi * (x[2] * t + x[3] * t * t / 2)) + rng.normal(0, 0.2, n)
    half = np.array([0.1, np.pi, 0.5, 0.5, 0.0, 0.1, 0.0])
    b = synth.Block(s, fs, n / 2, x, x - half, x + half,
                    synth.DESettings(pop=40, max_gens=400, seed=99), 0.2, stream=3, name="slope")
    dev = to_dev(s)
    f = ctx().fit_block(block_of(b, dev), settings_of(b, gens=25))
    assert _compare(b, f, _oracle_fit(b, 25), 40, "slope 25 gens") == 40
    f = ctx().fit_block(block_of(b, dev), settings_of(b))
    ref = _oracle_fit(b, b.de.max_gens)
    _compare(b, f, ref, 40, "slope")
    assert abs(f.coef[5] - x[5]) < 0.01


def test_batch_splits_blocks_by_arithmetic():
    # block 48 of the uneven batch has its carrier near 0 Hz, outside the
    # phasor bounds; the others qualify.  The batch runs them as separate
    # objective launches per generation, so every block gets the fit it gets
    # alone, bit for bit, in every one-launch form.
    blocks = synth.config3(0, nblocks=49, gens=20)
    sel = [blocks[0], blocks[1], blocks[48]]
    devs = [to_dev(b.samples) for b in sel]
    pbs = [block_of(b, d) for b, d in zip(sel, devs)]
    de = settings_of(sel[0])
    c = ctx()
    ptk.pt_ctx_set_tile(c.handle, 16, 8)  # one geometry (hence one summation order) for all fits
    try:
        alone = []
        for pb in pbs:
            f = c.fit_block(pb, de)
            alone.append((f, ptk.pt_ctx_last_arithmetic(c.handle)))
        assert [a for _, a in alone] == [ptk.PT_ARITH_FP64_PHASOR, ptk.PT_ARITH_FP64_PHASOR,
                                         ptk.PT_ARITH_FP64_POLY]
        for mode in (ptk.PT_FUSION_LEAD, ptk.PT_FUSION_LAST, ptk.PT_FUSION_OFF):
            ptk.pt_ctx_set_step_fusion(c.handle, mode)
            try:
                batch = c.fit_batch(pbs, de)
            finally:
                ptk.pt_ctx_set_step_fusion(c.handle, ptk.PT_FUSION_AUTO)
            for b, x, (y, _) in zip(sel, batch, alone):
                assert list(x.coef) == list(y.coef) and x.objective == y.objective, (b.name, mode)
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
    # the poly block against the oracle
    ref = _oracle_fit(sel[2], 20)
    assert_chi2_close([batch[2].objective], [ref["objective"]], sel[2].n)


@pytest.mark.parametrize("precision", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_full_64_block_batch_as_benchmarked(precision):
    # The batched workload at full size -- 64 blocks, N log-uniform in
    # [5e4, 4e5] at 50 kHz, SNR in [-5, 10] dB, own populations of 40, 1500
    # generations -- launched as the benchmark launches it: automatic launch
    # form and automatic geometry, which for a batch of more than four work
    # units per compute unit is the one with the most work per lane (32 x 8
    # for P = 40, in both precisions).  Sampled outputs against the oracle one
    # by one:
    # the reported objective is the oracle's chi^2 at the reported
    # coefficients (FP64 1e-10; mixed, at its optimum, mixed_rel_at_optimum,
    # which grows with the block's SNR and shrinks with its length), and
    # the block fitted alone gives the same fit bit for bit.  Every block:
    # all generations run and f0 within 6 Cramer-Rao bounds of the truth.
    blocks = synth.config3(0)
    assert len(blocks) == 64
    devs = [to_dev(b.samples) for b in blocks]
    pbs = [block_of(b, d) for b, d in zip(blocks, devs)]
    seed = synth.config1(0).de.seed  # the benchmark's seed
    de = ptk.make_settings(pop=40, max_gens=blocks[0].de.max_gens, F=0.5, CR=0.9, seed=seed, precision=precision)
    c = ctx()
    fits = c.fit_batch(pbs, de)
    geo = ptk.pt_ctx_last_geometry(c.handle)
    assert geo == (32, 8)
    ptk.pt_ctx_set_tile(c.handle, *geo)  # the fits alone in the batch's geometry
    try:
        sizes = [b.n for b in blocks]
        sample = sorted({0, int(np.argmax(sizes)), int(np.argmin(sizes)), 48})
        alone = {k: c.fit_block(pbs[k], de) for k in sample}
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
    errs = []
    for b, f in zip(blocks, fits):
        assert f.generations == de.max_gens, b.name
        errs.append(abs(f.coef[2] - b.truth[2]) / crlb_f0(b))
    for k in sample:
        b, f = blocks[k], fits[k]
        want = oracle.chi2(np.asarray(b.samples, dtype=np.float64), b.fs, b.ref, list(f.coef))
        rel = 1e-10 if precision == ptk.PT_PREC_FP64 else mixed_rel_at_optimum(b.n, want, f.coef[0], geo[0])
        assert abs(f.objective - want) <= rel * want, (b.name, f.objective, want, rel)
        a = alone[k]
        assert list(a.coef) == list(f.coef) and a.objective == f.objective, b.name
    print(f"[64-block batch prec={precision} geometry={geo}] sampled {sample}: objective == oracle chi^2 and "
          f"== fit alone; f0 error median {np.median(errs):.2f}, max {max(errs):.2f} CRLB", flush=True)
    assert max(errs) < 6.0
