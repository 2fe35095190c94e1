"""The fourth Taylor order (Sec. 3.2.1, perigee arcs) on the GPU.

Slot 6 is f3 [Hz/s^3]: phase term 2 pi f3 t^4 / 24.  Covered:
  * objective parity with the FP64 oracle for populations that use f3, in
    each arithmetic (FP64 phasor where valid, FP64 per-sample forward
    differences of the quartic, mixed precision), on the 20 s block and on
    ragged sizes;
  * fit parity: populations bit-identical to the oracle's for the first
    generations of a quartic fit;
  * on a 20 s perigee-like block the quartic fit reaches the noise floor and
    recovers f3, while the cubic fit (f3 fixed at 0) leaves a large residual.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_chi2_close, block_of, crlb_f0, ctx, model_phase_err, random_population, settings_of,
                      to_dev)
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

MIXED_REL = 3e-7  # see the derivation beside the same bound in test_gpu_objective.py


def _check(b, pop, precision=ptk.PT_PREC_FP64, method=ptk.PT_FP64_AUTO, rel=1e-10):
    c = ctx()
    ptk.pt_ctx_set_fp64_method(c.handle, method)
    try:
        got = c.objective(block_of(b, to_dev(b.samples)), to_dev(pop), precision).cpu().numpy()
        arith = ptk.pt_ctx_last_arithmetic(c.handle)
        floor = model_phase_err(c)
    finally:
        ptk.pt_ctx_set_fp64_method(c.handle, ptk.PT_FP64_AUTO)
    want = oracle.chi2_pop(b.samples.astype(np.float64), b.fs, b.ref, pop)
    print(f"[quartic {b.name} prec {precision} method {method}] arithmetic {arith} max rel err "
          f"{float(np.max(np.abs(got - want) / want)):.2e}", flush=True)
    assert_chi2_close(got, want, b.n, amp=float(np.max(np.abs(pop[:, 0]))), rel=rel, floor=floor)
    return arith


def test_objective_every_arithmetic():
    b = synth.config_quartic(0)
    pop = random_population(np.random.default_rng(31), b.lo, b.hi, 40, far=2)
    pop[4] = b.truth
    assert np.any(pop[:, 6] != 0)
    c = ctx()
    ptk.pt_ctx_set_tile(c.handle, 16, 4)  # 16-sample chunks: the phasor bound holds for this population
    try:
        assert _check(b, pop) == ptk.PT_ARITH_FP64_PHASOR
        assert _check(b, pop, method=ptk.PT_FP64_POLY) == ptk.PT_ARITH_FP64_POLY
        assert _check(b, pop, precision=ptk.PT_PREC_MIXED, rel=MIXED_REL) == ptk.PT_ARITH_MIXED
    finally:
        ptk.pt_ctx_set_tile(c.handle, 0, 0)
    _check(b, pop)  # default geometry, whichever arithmetic it allows


@pytest.mark.parametrize("n", [9, 4099, 65536 + 77])
def test_objective_ragged(n):
    b = synth.config_quartic(1, n=n)
    pop = random_population(np.random.default_rng(n), b.lo, b.hi, 11, far=1)
    pop[:, 6] *= 1e4  # a quartic term that matters on a short block
    _check(b, pop, method=ptk.PT_FP64_POLY)
    _check(b, pop)
    _check(b, pop, precision=ptk.PT_PREC_MIXED, rel=MIXED_REL)


def test_fit_matches_oracle_first_generations():
    b = synth.config_quartic(2, n=400_000)
    dev = to_dev(b.samples)
    f = ctx().fit_block(block_of(b, dev), settings_of(b, gens=25))
    ref = oracle.de_fit(b.samples.astype(np.float64), b.fs, b.ref, b.lo, b.hi, b.de.pop, 25, F=b.de.F,
                        CR=b.de.CR, seed=b.de.seed, stream=b.stream)
    pop, _ = ptk.pt_last_population(ctx().handle, 0, b.de.pop)
    same = int(np.sum(np.all(pop == ref["pop"], axis=1)))
    print(f"[quartic fit 25 gens] identical {same}/{b.de.pop} best {f.objective!r} vs {ref['objective']!r}",
          flush=True)
    assert same == b.de.pop
    assert f.generations == ref["generations"]
    assert_chi2_close([f.objective], [ref["objective"]], b.n)


def test_quartic_fit_beats_cubic_on_a_perigee_arc():
    b = synth.config_quartic(3)
    dev = to_dev(b.samples)
    q = ctx().fit_block(block_of(b, dev), settings_of(b))
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[6] = hi[6] = 0.0
    lo[4], hi[4] = b.truth[4] - 0.05, b.truth[4] + 0.05  # let the cubic absorb what it can
    c = ctx().fit_block(block_of(b, dev, lo=lo, hi=hi), settings_of(b))
    noise = b.n * b.sigma ** 2
    sig = crlb_f0(b)
    print(f"[perigee] f3 truth {b.truth[6]:.3e} fit {q.coef[6]:.3e}; chi2/noise quartic {q.objective / noise:.5f} "
          f"cubic {c.objective / noise:.5f}; f0 err quartic {(q.coef[2] - b.truth[2]) / sig:+.2f} CRLB",
          flush=True)
    # chi2 at the truth is the noise power within a few standard deviations (sqrt(2/N) relative)
    assert q.objective / noise < 1 + 10 * np.sqrt(2.0 / b.n)
    assert c.objective / noise > q.objective / noise + 0.01
    assert abs(q.coef[6] - b.truth[6]) < 0.05 * abs(b.truth[6])
    assert abs(q.coef[2] - b.truth[2]) < 6 * sig
    # the derived observables carry the quartic term
    t = np.array([b.n / b.fs / 2])
    _, _, fr, _ = ptk.pt_phase(q, t)
    c5 = oracle.derived.coefs_from_fit(q.coef[1], q.coef[2], q.coef[3], q.coef[4], q.coef[6])
    assert abs(fr[0] - float(oracle.derived.freq_hz(c5, t)[0])) < 1e-9


def test_quartic_whole_fit_matches_oracle_fit():
    # The whole fit of the 20 s quartic-phase block (1e6 samples, f3 free,
    # P = 40, 2000 generations) against the oracle's whole fit and the exact
    # least-squares minimiser, stored by tests/golden/make_paper_fit.py
    # --kind quartic (oracle only): f0 within 1e-6 Hz, chi^2 within 1e-10
    # relative of both, f1, f2 and f3 at the same optimum.
    g = json.load(open(os.path.join(GOLD, "quartic_fit_seed0.json")))
    b = synth.config_quartic(0)
    assert g["n"] == b.n and g["de"]["seed"] == b.de.seed and g["kind"] == "quartic"
    f = ctx().fit_block(block_of(b, to_dev(b.samples)), settings_of(b))
    ox, oobj = np.array(g["oracle_fit"]["x"]), g["oracle_fit"]["objective"]
    mx, mobj = np.array(g["minimiser"]["x"]), g["minimiser"]["objective"]
    print(f"[quartic whole fit] gpu f0 - oracle {f.coef[2] - ox[2]:+.3e} Hz, - minimiser {f.coef[2] - mx[2]:+.3e} Hz, "
          f"chi2 rel diff {(f.objective - oobj) / oobj:+.3e}, f3 {f.coef[6]:.6e} vs {ox[6]:.6e}", flush=True)
    assert f.generations == g["oracle_fit"]["generations"] == 2000
    assert f.flags == g["oracle_fit"]["flags"]
    assert abs(f.coef[2] - ox[2]) < 1e-6 and abs(f.coef[2] - mx[2]) < 1e-6
    assert abs(f.objective - oobj) <= 1e-10 * oobj and abs(f.objective - mobj) <= 1e-10 * mobj
    for j, name in ((3, "f1"), (4, "f2"), (6, "f3")):
        assert abs(f.coef[j] - ox[j]) < 1e-4 * (b.hi[j] - b.lo[j]), name
