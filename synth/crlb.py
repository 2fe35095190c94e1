"""Cramer-Rao bounds of the synthetic blocks' parameters (reporting only).

For a block s_n = mu_n(theta) + w_n with white Gaussian noise of standard
deviation sigma, the Fisher information of the parameters theta is
J = (1 / sigma^2) sum_n grad mu_n grad mu_n^T, and the variance of any
unbiased estimate of theta_i is at least (J^-1)_ii.  The model is the one the
blocks are drawn from (Sec. 2.2, Eq. 2-2-1 with the Taylor phase of
Eq. 2-2-3):

    mu_n = (A + Adot t) cos phi(t),
    phi(t) = phi0 + 2 pi (f0 t + f1 t^2 / 2 + f2 t^3 / 6 + f3 t^4 / 24),
    t = (n - ref) / fs,

so with g = -(A + Adot t) sin phi:
    d mu / dA = cos phi,    d mu / dAdot = t cos phi,   d mu / dphi0 = g,
    d mu / df0 = 2 pi t g,  d mu / df1 = pi t^2 g,       d mu / df2 = pi t^3 g / 3,
    d mu / df3 = pi t^4 g / 12.

The bound is taken over the parameters a fit actually frees (the block's box
slots with lo < hi).  With f1 and f2 free the f0 estimate correlates with
them, so its bound is larger than the single-tone one (f0, A, phi0 only),
sqrt(6) sigma / (pi A T sqrt(n)).

This module evaluates the bound for reporting accuracy; it holds none of the
fit's arithmetic.
"""
import math

import numpy as np

SLOTS = ("A", "phi0", "f0", "f1", "f2", "Adot", "f3")


def _jacobian(n, fs, ref, truth, slots, chunk=1 << 16):
    """Columns d mu / d theta_j for j in slots, accumulated as J = G^T G in
    chunks (FP64)."""
    A, phi0, f0, f1, f2 = (float(truth[k]) for k in range(5))
    adot = float(truth[5]) if len(truth) > 5 else 0.0
    f3 = float(truth[6]) if len(truth) > 6 else 0.0
    J = np.zeros((len(slots), len(slots)))
    for a in range(0, n, chunk):
        t = (np.arange(a, min(n, a + chunk), dtype=np.float64) - ref) / fs
        phi = phi0 + 2 * math.pi * (f0 * t + f1 * t * t / 2 + f2 * t ** 3 / 6 + f3 * t ** 4 / 24)
        c, amp = np.cos(phi), A + adot * t
        g = -amp * np.sin(phi)
        cols = {0: c, 1: g, 2: 2 * math.pi * t * g, 3: math.pi * t * t * g, 4: math.pi * t ** 3 * g / 3,
                5: t * c, 6: math.pi * t ** 4 * g / 12}
        G = np.stack([cols[k] for k in slots], axis=1)
        J += G.T @ G
    return J


def fisher_crlb(n, fs, ref, truth, sigma, slots):
    """Standard deviations sqrt((J^-1)_ii) of the parameters in `slots`
    (indices into SLOTS) for n samples at rate fs about reference sample
    `ref`, noise sigma, evaluated at `truth`.  Returns {slot index: std}."""
    slots = list(slots)
    J = _jacobian(int(n), float(fs), float(ref), truth, slots) / float(sigma) ** 2
    cov = np.linalg.inv(J)
    return {k: math.sqrt(cov[i, i]) for i, k in enumerate(slots)}


def free_slots(lo, hi):
    """Slots a fit frees: box lo < hi."""
    return [k for k in range(min(len(lo), len(SLOTS))) if lo[k] < hi[k]]


def crlb_f0_block(b):
    """CRLB [Hz] of f0 for a synth.Block, over the parameters its box frees."""
    slots = free_slots(b.lo, b.hi)
    if 2 not in slots:
        raise ValueError("f0 is fixed by the box")
    return fisher_crlb(b.n, b.fs, b.ref, b.truth, b.sigma, slots)[2]


def crlb_f0_single_tone(n, fs, amp, sigma):
    """The single-tone bound (f0, A and phi0 free, block-centred origin):
    sqrt(6) sigma / (pi A T sqrt(n)) with T = n / fs."""
    T = n / fs
    return math.sqrt(6.0) * sigma / (math.pi * amp * T * math.sqrt(n))
