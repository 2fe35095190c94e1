"""Pins of the Cramer-Rao bound used to report f0 accuracy (synth/crlb.py).

  * f0, A and phi0 free: the bound equals the single-tone closed form
    sqrt(6) sigma / (pi A T sqrt(n)) (time origin at the block centre).
  * f0, f1 and f2 free as well: with a centred origin f0 decouples from the
    even terms (A, phi0, f1) and couples only to the t^3 term, so its variance
    grows by the (1,1) element of the inverse Gram matrix of (t, t^3) over a
    uniform span, [[1/12, 1/80], [1/80, 1/448]]^-1 = [[75, ...]]: 75 / 12, i.e.
    the standard deviation by 2.5.
  * The Fisher sum agrees with a Monte-Carlo spread of the least-squares
    estimate on a small block.
"""
import math

import numpy as np
import scipy.optimize

import synth
from synth.crlb import crlb_f0_block, crlb_f0_single_tone, fisher_crlb


def test_single_tone_closed_form():
    n, fs, A, sigma = 200_000, 50_000.0, 0.8, 0.5
    truth = [A, 1.1, 1234.5, 0.0, 0.0, 0.0, 0.0]
    got = fisher_crlb(n, fs, n / 2, truth, sigma, [0, 1, 2])[2]
    want = crlb_f0_single_tone(n, fs, A, sigma)
    assert abs(got / want - 1) < 1e-3, (got, want)


def test_cubic_phase_inflates_f0_bound_by_two_and_a_half():
    b = synth.config1(0)
    full = crlb_f0_block(b)  # A, phi0, f0, f1, f2 free
    single = crlb_f0_single_tone(b.n, b.fs, b.truth[0], b.sigma)
    assert abs(full / single - 2.5) < 0.01, full / single
    # the paper-scale bound is ~2.7e-4 Hz at 0 dB over 8 s
    assert 2e-4 < full < 4e-4


def test_monte_carlo_spread_matches_bound():
    rng = np.random.default_rng(5)
    n, fs, sigma = 2000, 1000.0, 0.7
    truth = np.array([1.0, 0.4, 123.4, 0.8, 0.0])
    t = (np.arange(n) - n / 2) / fs

    def model(x):
        return x[0] * np.cos(x[1] + 2 * np.pi * (x[2] * t + x[3] * t * t / 2))

    clean = model(truth)
    est = []
    for _ in range(300):
        s = clean + rng.normal(0, sigma, n)
        r = scipy.optimize.least_squares(lambda x: model(x) - s, truth[:4], x_scale=[1, 1, 0.01, 0.01],
                                         xtol=1e-12, ftol=1e-12)
        est.append(r.x[2])
    spread = float(np.std(est))
    bound = fisher_crlb(n, fs, n / 2, list(truth) + [0, 0], sigma, [0, 1, 2, 3])[2]
    # 300 draws: the sample standard deviation is within ~15 % of the bound
    assert abs(spread / bound - 1) < 0.15, (spread, bound)
    assert math.isfinite(bound)
