"""Pins of the oracle's DE/rand/1/bin fit (Sec. 1.2, Table 4).

  * hand-worked trial vectors for the special cases of the scheme (CR = 0:
    only the forced coordinate comes from the mutant; CR = 1: the whole
    mutant; F = 0: the base vector; the bound rule; fixed slots);
  * invariants of the loop: best-so-far never rises, members stay in the
    box, stored objectives are the objectives of the stored members,
    determinism per seed, the stop rules and flags;
  * brute force on tiny blocks: for a fixed frequency law the amplitude and
    phase enter linearly (a cos + b sin), so the exact minimiser over
    (A, phi0) is a 2 x 2 least-squares solve; a dense grid over the
    frequency parameters followed by a local polish gives the global
    minimiser, which the DE fit must reach.
"""
import math

import numpy as np
import pytest
from scipy import optimize

import oracle
import synth


def _pop():
    pop = np.zeros((5, 6))
    pop[0, :5] = 9.0
    pop[1, :5] = [3, 2, 3, 4, 5]
    pop[2, :5] = [0, 2, 2, 2, 2]
    pop[3, :5] = [2, 1, 2, 3, 4]
    pop[4, :5] = 7.0
    return pop


LO = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
HI = np.array([10.0, 10.0, 10.0, 10.0, 10.0, 0.0])
ACT = [0, 1, 2, 3, 4]
MUTANT = np.array([2.0, 2.5, 3.0, 3.5, 4.0])  # x1 + 0.5 (x2 - x3)


def test_trial_cr_zero_takes_only_forced_coordinate():
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 2, [0.5] * 5, ACT, 0.5, 0.0, LO, HI)
    assert list(t[:5]) == [9, 9, 3, 9, 9]


def test_trial_cr_one_is_mutant():
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 0, [0.999] * 5, ACT, 0.5, 1.0, LO, HI)
    assert np.array_equal(t[:5], MUTANT)


def test_trial_mixed_crossover():
    U = [0.1, 0.6, 0.7, 0.2, 0.9]
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 4, U, ACT, 0.5, 0.5, LO, HI)
    assert list(t[:5]) == [2.0, 9.0, 9.0, 3.5, 4.0]


def test_trial_zero_scale_is_base_vector():
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 0, [0.0] * 5, ACT, 0.0, 1.0, LO, HI)
    assert list(t[:5]) == [3, 2, 3, 4, 5]


def test_trial_bound_rule():
    lo = LO.copy(); lo[0] = 2.5
    hi = HI.copy(); hi[1] = 2.2
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 0, [0.0] * 5, ACT, 0.5, 1.0, lo, hi)
    # slot 0: mutant 2 < 2.5 -> (2.5 + 3) / 2; slot 1: 2.5 > 2.2 -> (2.2 + 2) / 2
    assert t[0] == 2.75 and t[1] == pytest.approx(2.1, abs=0)
    assert list(t[2:5]) == [3.0, 3.5, 4.0]


def test_trial_fixed_slot_untouched():
    act = [0, 1, 2, 3]  # slot 4 fixed
    t = oracle.de_trial(_pop(), 0, 1, 2, 3, 3, [0.0] * 4, act, 0.5, 1.0, LO, HI)
    assert list(t[:4]) == [2.0, 2.5, 3.0, 3.5] and t[4] == 9.0


def test_init_inside_box_and_fixed_slots():
    b = synth.config0(0)
    pop = oracle.de_init(5, 0, 200, b.lo, b.hi)
    assert np.all(pop >= b.lo) and np.all(pop <= b.hi)
    assert np.all(pop[:, 4] == b.lo[4]) and np.all(pop[:, 5] == b.lo[5])
    # each active coordinate fills its interval roughly uniformly
    for j in range(4):
        u = (pop[:, j] - b.lo[j]) / (b.hi[j] - b.lo[j])
        assert 0.4 < u.mean() < 0.6 and u.min() < 0.05 and u.max() > 0.95


def test_fit_invariants_and_determinism():
    b = synth.config0(1)
    r = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 60, seed=b.de.seed)
    assert r["generations"] == 60 and r["flags"] == oracle.FLAG_MAXGEN
    assert np.all(np.diff(r["hist"]) <= 0)
    assert np.all(r["pop"] >= b.lo) and np.all(r["pop"] <= b.hi)
    again = oracle.chi2_pop(b.samples, b.fs, b.ref, r["pop"])
    assert np.array_equal(again, r["fpop"])
    assert r["objective"] == r["fpop"].min() == r["hist"][-1]
    r2 = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 60, seed=b.de.seed)
    assert np.array_equal(r["pop"], r2["pop"])
    r3 = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 60, seed=b.de.seed + 1)
    assert not np.array_equal(r["pop"], r3["pop"])
    r4 = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 60, seed=b.de.seed, stream=1)
    assert not np.array_equal(r["pop"], r4["pop"])


def test_window_stop_rule():
    b = synth.config0(2)
    W, tol = 20, 1e-9
    r = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 3000, seed=b.de.seed,
                      rel_tol=tol, window=W)
    g, h = r["generations"], r["hist"]
    assert r["flags"] & oracle.FLAG_CONVERGED and g < 3000
    assert h[g - W] - h[g] <= tol * h[g]
    for k in range(W, g):
        assert h[k - W] - h[k] > tol * h[k]


def test_vtr_and_at_bound_flags():
    b = synth.config0(3)
    r = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 50, seed=1, vtr=1e12)
    assert r["generations"] == 0 and r["flags"] == oracle.FLAG_VTR
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[2], hi[2] = b.truth[2] + 0.05, b.truth[2] + 2.0   # truth below the box
    r = oracle.de_fit(b.samples, b.fs, b.ref, lo, hi, 32, 150, seed=1)
    assert r["flags"] & oracle.FLAG_AT_BOUND
    r = oracle.de_fit(b.samples, b.fs, b.ref, b.lo, b.hi, 32, 150, seed=1)
    assert not r["flags"] & oracle.FLAG_AT_BOUND


# ---------------------------------------------------------------- brute force
def _profile(s, t, freq_turns):
    """min over (A, phi0) of sum (s - A cos(2 pi u + phi0))^2 for phases u(t)
    given in turns: linear least squares in (a, b) of a cos + b sin."""
    c = np.cos(2 * np.pi * freq_turns)
    sn = np.sin(2 * np.pi * freq_turns)
    M = np.stack([c, sn], axis=-1)
    coef, *_ = np.linalg.lstsq(M, s, rcond=None)
    r = s - M @ coef
    return float(r @ r), coef


def _tiny(n, fs, f0, f1, seed, sigma=0.2):
    rng = np.random.default_rng(seed)
    t = (np.arange(n) - n / 2) / fs
    s = 0.9 * np.cos(1.1 + 2 * np.pi * (f0 * t + f1 * t * t / 2)) + rng.normal(0, sigma, n)
    return s, t


def test_brute_force_linear_phase():
    n, fs, f0 = 128, 100.0, 12.34
    s, t = _tiny(n, fs, f0, 0.0, 0)
    grid = np.linspace(f0 - 1, f0 + 1, 4001)
    vals = [_profile(s, t, g * t)[0] for g in grid]
    k = int(np.argmin(vals))
    res = optimize.minimize_scalar(lambda g: _profile(s, t, g * t)[0],
                                   bracket=(grid[k - 1], grid[k], grid[k + 1]),
                                   tol=1e-14)
    f_star, chi_star = res.x, res.fun
    lo = np.array([0.5, -math.pi, f0 - 1, 0, 0, 0])
    hi = np.array([1.3, math.pi, f0 + 1, 0, 0, 0])
    r = oracle.de_fit(s, fs, n / 2, lo, hi, 20, 400, seed=4)
    assert r["objective"] <= chi_star * (1 + 1e-12)
    assert r["objective"] <= min(vals)
    assert abs(r["x"][2] - f_star) < 1e-6
    _, coef = _profile(s, t, f_star * t)
    A = math.hypot(*coef)
    phi = math.atan2(-coef[1], coef[0])
    assert r["x"][0] == pytest.approx(A, rel=1e-6)
    assert math.remainder(r["x"][1] - phi, 2 * math.pi) == pytest.approx(0, abs=1e-6)


def test_brute_force_quadratic_phase():
    n, fs, f0, f1 = 256, 200.0, 31.7, 2.3
    s, t = _tiny(n, fs, f0, f1, 1)
    g0 = np.linspace(f0 - 0.6, f0 + 0.6, 241)
    g1 = np.linspace(f1 - 3.0, f1 + 3.0, 241)
    best = (np.inf, None)
    for a in g0:
        for b in g1:
            v = _profile(s, t, a * t + b * t * t / 2)[0]
            if v < best[0]:
                best = (v, (a, b))
    grid_min = best[0]

    def resid(p):
        u = p[0] * t + p[1] * t * t / 2
        return s - p[2] * np.cos(2 * np.pi * u) - p[3] * np.sin(2 * np.pi * u)

    _, coef = _profile(s, t, best[1][0] * t + best[1][1] * t * t / 2)
    sol = optimize.least_squares(resid, [best[1][0], best[1][1], coef[0], coef[1]],
                                 xtol=1e-15, ftol=1e-15, gtol=1e-15)
    chi_star = float(sol.fun @ sol.fun)
    lo = np.array([0.5, -math.pi, f0 - 0.6, f1 - 3.0, 0, 0])
    hi = np.array([1.3, math.pi, f0 + 0.6, f1 + 3.0, 0, 0])
    r = oracle.de_fit(s, fs, n / 2, lo, hi, 24, 600, seed=9)
    assert r["objective"] <= grid_min
    assert r["objective"] <= chi_star * (1 + 1e-12)
    assert abs(r["x"][2] - sol.x[0]) < 1e-6
    assert abs(r["x"][3] - sol.x[1]) < 1e-5
