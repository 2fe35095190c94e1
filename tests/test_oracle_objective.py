"""Pins of the oracle's chi-square objective (Eq. 2-2-2 / 2-2-4).

Each check rests on something other than the oracle's own formula:
  * A = 0 leaves the sum of squared samples (pins the summation);
  * the Dirichlet-kernel closed form of sum cos(a n + b) for a linear phase,
    evaluated with mpmath at 40 digits (pins cosine, f0, phi0, the time
    origin and the quadratic structure in A);
  * a signal whose phase is the integral of the frequency law
    f(t) = f0 + f1 t + f2 t^2 / 2, accumulated sample by sample with
    Simpson's rule in exact rationals (exact for a quadratic integrand) --
    the objective at the generating coefficients must vanish, which pins the
    factorials of the f1 and f2 terms and the sign conventions;
  * re-expanding the same phase about another reference sample leaves the
    objective unchanged (pins the time origin handling);
  * the noise statistics: E[chi2] = N sigma^2 at the truth (the objective
    converges to the noise power, Sec. 2.2);
  * symmetries of the cosine (period, mirror, sign of A).
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import synth

mpmath.mp.dps = 40


def _dirichlet(a, b, n):
    """sum_{k<n} cos(a k + b) in closed form (mpmath)."""
    a = mpmath.mpf(a)
    b = mpmath.mpf(b)
    half = a / 2
    if abs(mpmath.sin(half)) < mpmath.mpf(10) ** -30:
        return n * mpmath.cos(b)  # a is a multiple of 2 pi: every term is cos b
    return mpmath.sin(n * half) / mpmath.sin(half) * mpmath.cos(b + (n - 1) * half)


def _linear_closed_form(A, a, b, Ah, ah, bh, n):
    """sum (A cos(a k + b) - Ah cos(ah k + bh))^2 via products-to-sums."""
    t1 = A * A / 2 * (n + _dirichlet(2 * a, 2 * b, n))
    t2 = Ah * Ah / 2 * (n + _dirichlet(2 * ah, 2 * bh, n))
    t3 = A * Ah * (_dirichlet(a - ah, b - bh, n) + _dirichlet(a + ah, b + bh, n))
    return t1 + t2 - t3


def test_zero_amplitude_is_sum_of_squares():
    rng = np.random.default_rng(1)
    s = rng.normal(size=10007)
    x = [0.0, 1.3, 123.4, 0.7, 0.01, 0.0]
    got = oracle.chi2(s, 1000.0, 5003.5, x)
    ref = math.fsum(float(v) * float(v) for v in s)
    assert got == pytest.approx(ref, rel=1e-15)


@pytest.mark.parametrize("n,fs,ref", [(4096, 1000.0, 2048.0), (1001, 250.0, 500.5), (64, 1.0, 0.0)])
def test_linear_phase_dirichlet_closed_form(n, fs, ref):
    mp = mpmath.mpf
    A, f0, phi0 = mp("0.93"), mp("123.4567"), mp("1.234")
    a = 2 * mpmath.pi * f0 / fs
    b = phi0 - a * ref
    s = np.array([float(A * mpmath.cos(a * k + b)) for k in range(n)])
    cands = [(0.93, 1.234, 123.4567), (1.1, 0.3, 123.4567), (0.8, 2.0, 123.5),
             (1.05, -2.5, 121.0), (0.5, 6.0, 130.25)]
    for Ah, ph, fh in cands:
        ah = 2 * mpmath.pi * mp(fh) / fs
        bh = mp(ph) - ah * ref
        # the samples are FP64-rounded: account for that with the exact sum of
        # their rounding against the closed form's exact cosines
        exact = _linear_closed_form(A, a, b, mp(Ah), ah, bh, n)
        corr = mpmath.fsum((mp(float(s[k])) - A * mpmath.cos(a * k + b)) *
                           (mp(float(s[k])) + A * mpmath.cos(a * k + b) -
                            2 * mp(Ah) * mpmath.cos(ah * k + bh)) for k in range(n))
        want = float(exact + corr)
        got = oracle.chi2(s, fs, ref, [Ah, ph, fh, 0.0, 0.0, 0.0])
        # FP64 forms the phase with a rounding of a few ulp of its largest
        # magnitude; each residual moves by at most Ah times that, so the sum
        # of squares moves by at most 2 n (A + Ah) Ah eps_phi.
        max_phase = abs(ph) + 2 * math.pi * abs(fh) * max(ref, n - 1 - ref) / fs
        eps_phi = 4 * max_phase * 2.0 ** -53
        tol = 2 * n * (0.93 + Ah) * Ah * eps_phi
        assert abs(got - want) <= tol + 1e-15 * want


def _simpson_signal(n, fs, ref, A, phi0, f0, f1, f2, f3=0.0):
    """cos of phi0 + 2 pi * integral_0^t f(u) du, t = (k - ref)/fs, the
    integral accumulated with Simpson's rule in exact rationals (exact for
    the cubic frequency law f0 + f1 u + f2 u^2/2 + f3 u^3/6)."""
    F0, F1, F2, F3 = Fraction(f0), Fraction(f1), Fraction(f2), Fraction(f3)
    h = 1 / Fraction(fs)

    def f(u):
        return F0 + F1 * u + F2 * u * u / 2 + F3 * u * u * u / 6

    kref = int(ref)
    assert Fraction(ref) == kref
    turns = {kref: Fraction(0)}
    for k in range(kref, n - 1):        # forward from the reference sample
        u = (k - kref) * h
        turns[k + 1] = turns[k] + h / 6 * (f(u) + 4 * f(u + h / 2) + f(u + h))
    for k in range(kref, 0, -1):        # backward
        u = (k - kref) * h
        turns[k - 1] = turns[k] - h / 6 * (f(u - h) + 4 * f(u - h / 2) + f(u))
    out = np.empty(n)
    for k in range(n):
        fr = turns[k] - math.floor(turns[k])
        out[k] = float(A * mpmath.cos(mpmath.mpf(phi0) + 2 * mpmath.pi * mpmath.mpf(fr.numerator) / fr.denominator))
    return out


def test_integrated_frequency_law_vanishes_at_truth():
    n, fs, ref = 2000, 500.0, 1000.0
    A, phi0, f0, f1, f2 = 0.8, 2.1, 37.25, 3.5, -1.75
    s = _simpson_signal(n, fs, ref, A, phi0, f0, f1, f2)
    x = [A, phi0, f0, f1, f2, 0.0]
    assert oracle.chi2(s, fs, ref, x) < 1e-20
    # each term matters: a dropped or mis-scaled f1 / f2 term is far from zero
    for j, scale in [(3, 2.0), (4, 2.0), (4, 0.0), (3, 0.0)]:
        y = list(x)
        y[j] *= scale
        assert oracle.chi2(s, fs, ref, y) > 1.0


def test_quartic_frequency_law_vanishes_at_truth():
    # the fourth Taylor order of Sec. 3.2.1: slot 6 is f3 with phase 2 pi f3 t^4 / 24
    n, fs, ref = 2000, 500.0, 1000.0
    A, phi0, f0, f1, f2, f3 = 0.8, 2.1, 37.25, 3.5, -1.75, 1.5
    s = _simpson_signal(n, fs, ref, A, phi0, f0, f1, f2, f3)
    x = [A, phi0, f0, f1, f2, 0.0, f3]
    assert oracle.chi2(s, fs, ref, x) < 1e-20
    for j, scale in [(6, 2.0), (6, 0.0), (6, -1.0), (4, 0.0)]:
        y = list(x)
        y[j] *= scale
        assert oracle.chi2(s, fs, ref, y) > 1.0
    # the correlation objective sees the same phase
    xc = list(x)
    assert oracle.cor(s, fs, ref, xc) < oracle.cor(s, fs, ref, x[:6] + [0.0])


def test_quartic_reference_shift_invariance():
    rng = np.random.default_rng(8)
    n, fs = 3001, 1000.0
    s = rng.normal(size=n)
    phi0, f0, f1, f2, f3 = 0.4, 123.4, 2.0, -0.7, 0.3
    x1 = [1.3, phi0, f0, f1, f2, 0.0, f3]
    shifted = synth.shift_truth4(phi0, f0, f1, f2, f3, 0.9)
    x2 = [1.3, shifted[0], shifted[1], shifted[2], shifted[3], 0.0, shifted[4]]
    a = oracle.chi2(s, fs, 0.0, x1)
    b = oracle.chi2(s, fs, 900.0, x2)
    assert abs(a - b) <= 1e-9 * a


def test_reference_shift_invariance():
    b = synth.config1(3, n=20000)
    s = b.samples.astype(np.float64)
    x = b.truth.copy()
    x[0] *= 0.97
    x[2] += 0.01
    f_c = oracle.chi2(s, b.fs, b.ref, x)
    for new_ref in [0.0, 12345.0, 19999.5]:
        dt = (new_ref - b.ref) / b.fs
        p, g0, g1, g2 = synth.shift_truth(x[1], x[2], x[3], x[4], dt)
        y = [x[0], p, g0, g1, g2, 0.0]
        assert oracle.chi2(s, b.fs, new_ref, y) == pytest.approx(f_c, rel=1e-11)


def test_noise_power_at_truth():
    for seed in range(4):
        b = synth.config0(seed)
        f = oracle.chi2(b.samples, b.fs, b.ref, b.truth)
        n, s2 = b.n, b.sigma ** 2
        assert abs(f - n * s2) < 5 * math.sqrt(2 * n) * s2


def test_cosine_symmetries():
    b = synth.config0(1)
    x = np.array([1.02, 0.7, b.truth[2] + 0.3, b.truth[3] - 0.2, 0.0, 0.0])
    f = oracle.chi2(b.samples, b.fs, b.ref, x)
    y = x.copy(); y[1] += 2 * math.pi
    assert oracle.chi2(b.samples, b.fs, b.ref, y) == pytest.approx(f, rel=1e-12)
    y = -x; y[0] = x[0]; y[5] = 0.0
    assert oracle.chi2(b.samples, b.fs, b.ref, y) == pytest.approx(f, rel=1e-12)
    y = x.copy(); y[0] = -x[0]; y[1] += math.pi
    assert oracle.chi2(b.samples, b.fs, b.ref, y) == pytest.approx(f, rel=1e-12)


def test_quadratic_in_amplitude():
    # chi2(A) = sum s^2 - 2 A sum s c + A^2 sum c^2: equal second differences,
    # and for a linear phase sum c^2 = (N + D(2a, 2b)) / 2.
    n, fs, ref = 3000, 800.0, 1500.0
    rng = np.random.default_rng(4)
    s = rng.normal(size=n)
    ph, fh = 0.4, 77.7
    vals = [oracle.chi2(s, fs, ref, [A, ph, fh, 0, 0, 0]) for A in (-1.0, 0.0, 1.0, 2.0)]
    d2a = vals[3] - 2 * vals[2] + vals[1]
    d2b = vals[2] - 2 * vals[1] + vals[0]
    a = 2 * mpmath.pi * mpmath.mpf(fh) / fs
    b = mpmath.mpf(ph) - a * ref
    sc2 = float((n + _dirichlet(2 * a, 2 * b, n)) / 2)
    assert d2a == pytest.approx(2 * sc2, rel=1e-10)
    assert d2b == pytest.approx(2 * sc2, rel=1e-10)


def test_amplitude_slope_term():
    # With a constant-phase model (f = 0, phi0 = 0) the model is A + Adot t;
    # chi2 against samples equal to that line is zero, and a zero-slope model
    # leaves sum (Adot t)^2.
    n, fs, ref = 101, 10.0, 50.0
    t = (np.arange(n) - ref) / fs
    s = 0.5 + 0.25 * t
    assert oracle.chi2(s, fs, ref, [0.5, 0.0, 0.0, 0.0, 0.0, 0.25]) < 1e-28
    assert oracle.chi2(s, fs, ref, [0.5, 0.0, 0.0, 0.0, 0.0, 0.0]) == pytest.approx(
        math.fsum((0.25 * v) ** 2 for v in t), rel=1e-14)


def test_population_matches_single():
    b = synth.config0(2)
    pop = oracle.de_init(3, 0, 16, b.lo, b.hi)
    many = oracle.chi2_pop(b.samples, b.fs, b.ref, pop, nthreads=3)
    one = [oracle.chi2(b.samples, b.fs, b.ref, p) for p in pop]
    assert np.array_equal(many, np.array(one))


# ------------------------------------------------- correlation objective
def test_correlation_linear_phase_closed_form():
    # C = A_hat sum s cos(a_hat k + b_hat) with s = A cos(a k + b):
    # sum cos cos = (D(a - a_hat, b - b_hat) + D(a + a_hat, b + b_hat)) / 2
    mp = mpmath.mpf
    n, fs, ref = 3001, 500.0, 1500.0
    A, f0, phi0 = mp("0.7"), mp("61.25"), mp("2.5")
    a = 2 * mpmath.pi * f0 / fs
    b = phi0 - a * ref
    s = np.array([float(A * mpmath.cos(a * k + b)) for k in range(n)])
    for Ah, ph, fh in [(1.0, 2.5, 61.25), (1.3, 0.4, 61.0), (0.9, -1.0, 70.5)]:
        ah = 2 * mpmath.pi * mp(fh) / fs
        bh = mp(ph) - ah * ref
        C = mp(Ah) * A * (_dirichlet(a - ah, b - bh, n) + _dirichlet(a + ah, b + bh, n)) / 2
        want = float(1 / (mpmath.atan(C) + mpmath.pi / 2))
        got = oracle.cor(s, fs, ref, [Ah, ph, fh, 0, 0, 0])
        assert got == pytest.approx(want, rel=1e-13)


def test_correlation_tends_to_one_over_pi_and_orders_like_chi2():
    # at the truth C ~ N A^2 / 2 is large, so F -> 1/pi from above; F is a
    # decreasing function of C, and with a fixed amplitude chi2 = sum s^2 -
    # 2 C + A^2 sum cos^2, so near the truth both objectives rank candidates alike
    b = synth.config0(0)
    x = b.truth.copy()
    f = oracle.cor(b.samples, b.fs, b.ref, x)
    assert 1 / np.pi < f < 1 / np.pi + 1e-3
    worse = x.copy()
    worse[2] += 0.05
    assert oracle.cor(b.samples, b.fs, b.ref, worse) > f
    zero = x.copy()
    zero[0] = 0.0
    assert oracle.cor(b.samples, b.fs, b.ref, zero) == pytest.approx(2 / np.pi, rel=1e-15)  # C = 0
    neg = x.copy()
    neg[1] += np.pi  # anti-correlated model: C -> -C, F -> 1/(pi/2 - atan C) > 2/pi
    assert oracle.cor(b.samples, b.fs, b.ref, neg) > 2 / np.pi


def test_obj_pop_dispatch():
    b = synth.config0(1)
    pop = oracle.de_init(2, 0, 6, b.lo, b.hi)
    c = oracle.obj_pop(oracle.OBJ_COR, b.samples, b.fs, b.ref, pop)
    assert np.array_equal(c, [oracle.cor(b.samples, b.fs, b.ref, p) for p in pop])
    q = oracle.obj_pop(oracle.OBJ_CHI2, b.samples, b.fs, b.ref, pop)
    assert np.array_equal(q, oracle.chi2_pop(b.samples, b.fs, b.ref, pop))
