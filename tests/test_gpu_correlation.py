"""GPU parity of the correlation objective (Eq. 2-2-5 with the constant-
amplitude model of Eq. 2-2-6) against the FP64 oracle.

F = 1 / (arctan C + pi/2) with C = sum_n s_n A cos phi_n.  Both sides form
C with different summation orders and phase arithmetic; the tolerance on F
follows from the one on C: |dF| <= F^2 |dC| / (1 + (|C| - |dC|)^2), with
|dC| <= sum|s| * max|A| * (eps_phi + eps_terms), eps_phi the FP64 phase
rounding of the candidate and eps_terms the cosine and summation error of
the path (FP64: 2e-14 plus the arithmetic's per-sample phase error, 2 pi 1e-12
for the phasor recurrence; mixed: 5e-6, from its FP32 phase offset, FP32
cosine and FP32 lane sums).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (MODEL_PHASE_ERR, block_of, ctx, model_phase_err, phase_rounding_bound, random_population,
                      settings_of, to_dev)
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# cosine and summation error of each path [relative to sum |s| A]; the FP64
# path adds its arithmetic's per-sample phase error (model_phase_err)
EPS_TERMS = {ptk.PT_PREC_FP64: 2e-14, ptk.PT_PREC_MIXED: 5e-6}


def _fixed_amplitude(b: synth.Block):
    """Box of Eq. (2-2-6): amplitude fixed at the block's mean amplitude."""
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[0] = hi[0] = b.truth[0]
    lo[5] = hi[5] = 0.0
    return lo, hi


def _assert_cor_close(got, want, s, pop, fs, ref, precision, model_err=0.0):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    eps_phi, amp = phase_rounding_bound(s, pop, fs, ref)
    n = s.size
    tmax = max(abs(ref), abs(n - 1 - ref)) / fs
    amax = amp + np.abs(np.atleast_2d(pop)[:, 5]) * tmax
    dC = float(np.sum(np.abs(s))) * amax * (eps_phi + EPS_TERMS[precision] + model_err)
    C = np.tan(1.0 / want - math.pi / 2)
    tol = want ** 2 * dC / (1.0 + np.maximum(np.abs(C) - dC, 0.0) ** 2) + 8 * 2.0 ** -53 * want
    err = np.abs(got - want)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{bad.size} outside tolerance; first {int(bad[0])}: gpu {got[bad[0]]!r} "
                           f"oracle {want[bad[0]]!r} tol {tol[bad[0]]!r}")
    return float(np.max(err / tol))


def _check(b, pop, precision=ptk.PT_PREC_FP64, samples=None):
    s = b.samples if samples is None else samples
    blk = block_of(b, to_dev(s))
    got = ctx().objective(blk, to_dev(pop), precision, objective=ptk.PT_OBJ_COR).cpu().numpy()
    merr = model_phase_err() if precision == ptk.PT_PREC_FP64 else 0.0
    s64 = np.asarray(s, dtype=np.float64)
    want = oracle.obj_pop(oracle.OBJ_COR, s64, b.fs, b.ref, pop)
    worst = _assert_cor_close(got, want, s64, pop, b.fs, b.ref, precision, merr)
    print(f"[cor {b.name} n={s.size} prec={precision}] worst err/tol {worst:.3f}", flush=True)
    return got, want


@pytest.mark.parametrize("precision", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_tiny_block(precision):
    b = synth.config0(0)
    lo, hi = _fixed_amplitude(b)
    pop = random_population(np.random.default_rng(20), lo, hi, 32, far=3)
    pop[3] = b.truth
    _check(b, pop, precision)


@pytest.mark.parametrize("precision", [ptk.PT_PREC_FP64, ptk.PT_PREC_MIXED])
def test_paper_block_full_size(precision):
    b = synth.config1(0)
    lo, hi = _fixed_amplitude(b)
    pop = random_population(np.random.default_rng(21), lo, hi, 40, far=2)
    pop[9] = b.truth
    got, want = _check(b, pop, precision)
    # the truth has the largest correlation, hence the smallest F, on both sides
    assert int(np.argmin(got)) == 9 and int(np.argmin(want)) == 9


@pytest.mark.parametrize("n", [8, 63, 4096 + 5, 65536 + 17])
def test_ragged_sizes(n):
    b = synth.config1(1, n=n)
    lo, hi = _fixed_amplitude(b)
    pop = random_population(np.random.default_rng(n + 1), lo, hi, 13, far=2)
    _check(b, pop)
    _check(b, pop, samples=b.samples.astype(np.float64))


def test_phasor_and_polynomial_paths_agree():
    # a population close to the truth lets the FP64 path use the phasor
    # recurrence; forcing the polynomial cosine must give the same objective
    b = synth.config1(2)
    rng = np.random.default_rng(22)
    pop = np.tile(b.truth, (24, 1))
    pop[:, 1] += rng.uniform(-1, 1, 24)
    pop[:, 2] += rng.uniform(-0.05, 0.05, 24)
    pop[:, 3] += rng.uniform(-1e-3, 1e-3, 24)
    pop[:, 4] += rng.uniform(-1e-5, 1e-5, 24)
    auto, want = _check(b, pop)
    c = ctx()
    ptk.pt_ctx_set_fp64_method(c.handle, ptk.PT_FP64_POLY)
    try:
        poly, _ = _check(b, pop)
    finally:
        ptk.pt_ctx_set_fp64_method(c.handle, ptk.PT_FP64_AUTO)
    _assert_cor_close(auto, poly, b.samples.astype(np.float64), pop, b.fs, b.ref, ptk.PT_PREC_FP64,
                      MODEL_PHASE_ERR[ptk.PT_ARITH_FP64_PHASOR])


def test_correlation_tends_to_one_over_pi_at_the_truth():
    b = synth.config1(3)
    blk = block_of(b, to_dev(b.samples))
    got = ctx().objective(blk, to_dev(b.truth[None, :].copy()), objective=ptk.PT_OBJ_COR).cpu().numpy()[0]
    # C ~ A^2 N / 2 at the truth, so F - 1/pi ~ 1 / (pi^2 C)
    C = b.truth[0] ** 2 * b.n / 2
    assert 0 < got - 1 / math.pi < 4 / (math.pi ** 2 * C)


def _oracle_fit(b, lo, hi, gens):
    de = b.de
    return oracle.de_fit(np.asarray(b.samples, dtype=np.float64), b.fs, b.ref, lo, hi, de.pop, gens,
                         F=de.F, CR=de.CR, seed=de.seed, stream=b.stream, vtr=de.vtr,
                         rel_tol=de.rel_tol, window=de.window, objective=oracle.OBJ_COR)


def test_fit_with_correlation_objective_matches_oracle():
    for seed in range(2):
        b = synth.config0(seed)
        lo, hi = _fixed_amplitude(b)
        dev = to_dev(b.samples)
        blk = block_of(b, dev, lo=lo, hi=hi)
        for gens in (30, b.de.max_gens):
            f = ctx().fit_block(blk, settings_of(b, gens=gens, objective=ptk.PT_OBJ_COR))
            ref = _oracle_fit(b, lo, hi, gens)
            pop, _ = ptk.pt_last_population(ctx().handle, 0, b.de.pop)
            hist = ptk.pt_last_history(ctx().handle, 0, ref["generations"] + 1)
            same = int(np.sum(np.all(pop == ref["pop"], axis=1)))
            print(f"[cor fit seed {seed} {gens} gens] identical {same}/{b.de.pop} "
                  f"F {f.objective!r} vs {ref['objective']!r} df0 {f.coef[2] - ref['x'][2]:.3e}", flush=True)
            assert f.generations == ref["generations"] and f.flags == ref["flags"]
            if gens == 30:
                assert same == b.de.pop
            s64 = b.samples.astype(np.float64)
            _assert_cor_close([f.objective], [ref["objective"]], s64, ref["x"][None, :], b.fs, b.ref,
                              ptk.PT_PREC_FP64, MODEL_PHASE_ERR[ptk.PT_ARITH_FP64_PHASOR])
            assert np.max(np.abs(hist - ref["hist"])) < 1e-12
            assert abs(f.coef[2] - ref["x"][2]) < 1e-6
        # the correlation fit recovers the carrier: within 10 CRLB of the truth
        sig = math.sqrt(6.0) * b.sigma / (math.pi * b.truth[0] * (b.n / b.fs) * math.sqrt(b.n))
        assert abs(f.coef[2] - b.truth[2]) < 10 * sig


def test_invalid_objective_kind():
    b = synth.config0(0)
    blk = block_of(b, to_dev(b.samples))
    with pytest.raises(ptk.PtError):
        ctx().objective(blk, to_dev(np.tile(b.truth, (4, 1))), objective=7)
    with pytest.raises(ptk.PtError):
        ctx().fit_block(blk, settings_of(b, gens=5, objective=7))


def _correlation_of(F):
    """C from F = 1 / (arctan C + pi/2): C = -1 / tan(1 / F), to ~4e-11 relative
    for the C ~ 1e5 of a paper-scale block (1 / F = pi - ~1 / C)."""
    return -1.0 / math.tan(1.0 / F)


def test_paper_block_whole_correlation_fit_matches_oracle_fit():
    # The whole paper-scale fit under the correlation objective (Eq. 2-2-5,
    # amplitude fixed at the truth as Eq. 2-2-6 asks; 400 000 samples, P = 40,
    # 2000 generations) against the oracle's whole fit of the same block,
    # stored by tests/golden/make_paper_fit.py --kind cor (oracle only).  The
    # trajectories part at the first selection near-tie; both reach the same
    # optimum: f0 within 1e-6 Hz, the correlation C within 1e-9 relative.
    # (F sits at 1/pi + 1/(pi^2 C) with C ~ 1.2e4 here, so an f0 offset d moves
    # F by ~(2 pi T d)^2 / (24 pi^2 C): a few ulp of F at d = 4e-7 Hz, the
    # objective's own resolution; the two fits are measured 4.3e-7 Hz apart.)
    g = json.load(open(os.path.join(GOLD, "paper_fit_cor_seed0.json")))
    b = synth.config1(0)
    lo, hi = _fixed_amplitude(b)
    assert g["n"] == b.n and g["de"]["seed"] == b.de.seed and g["kind"] == "cor"
    assert np.array_equal(np.array(g["box"]["lo"]), lo) and np.array_equal(np.array(g["box"]["hi"]), hi)
    f = ctx().fit_block(block_of(b, to_dev(b.samples), lo=lo, hi=hi), settings_of(b, objective=ptk.PT_OBJ_COR))
    ox, oF = np.array(g["oracle_fit"]["x"]), g["oracle_fit"]["objective"]
    cg, co = _correlation_of(f.objective), _correlation_of(oF)
    print(f"[paper whole correlation fit] gpu f0 - oracle f0 {f.coef[2] - ox[2]:+.3e} Hz, C rel diff "
          f"{(cg - co) / co:+.3e}", flush=True)
    assert f.generations == g["oracle_fit"]["generations"] == 2000
    assert f.flags == g["oracle_fit"]["flags"]
    assert abs(f.coef[2] - ox[2]) < 1e-6
    assert abs(cg - co) <= 1e-9 * co
