"""Observables derived from a fitted Taylor phase (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Coefficients follow Eq. (2-2-3): c0 = phi(0), c_i = phi^(i)(0) / i!.  In the
fit's units (phi0 [rad], f0 [Hz], f1 [Hz/s], f2 [Hz/s^2]):
    c0 = phi0, c1 = 2 pi f0, c2 = pi f1, c3 = pi f2 / 3.
"""
import math

import numpy as np

C_LIGHT = 299792458.0  # m/s


def coefs_from_fit(phi0, f0, f1, f2, f3=None):
    """(c0, c1, c2, c3) of Eq. (2-2-3) from the fit's parameters; with f3 also
    the fourth-order phase coefficient phi^(4)(0) / 4! = pi f3 / 12 (Sec. 3.2.1)."""
    c = (phi0, 2.0 * math.pi * f0, math.pi * f1, math.pi * f2 / 3.0)
    return c if f3 is None else c + (math.pi * f3 / 12.0,)


def fit_from_coefs(c0, c1, c2, c3, c4=None):
    """Inverse of :func:`coefs_from_fit`."""
    f = (c0, c1 / (2.0 * math.pi), c2 / math.pi, 3.0 * c3 / math.pi)
    return f if c4 is None else f + (12.0 * c4 / math.pi,)


def _c5(c):
    """Phase coefficients padded to the fourth order (c4 = 0 for a cubic)."""
    return tuple(c[:4]) + ((c[4],) if len(c) > 4 else (0.0,))


def phase(c, t):
    """phi(t) = c0 + c1 t + c2 t^2 + c3 t^3 (+ c4 t^4) [rad], Eq. (3-1-1)."""
    c = _c5(c)
    t = np.asarray(t, dtype=np.float64)
    return c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3 + c[4] * t ** 4


def phase_mod2pi(c, t):
    """Phase reduced to [0, 2 pi), as at the block borders of Eq. (3-1-2)."""
    return np.mod(phase(c, t), 2.0 * math.pi)


def freq_rad(c, t):
    """F(t) = d phi / dt = c1 + 2 c2 t + 3 c3 t^2 (+ 4 c4 t^3) [rad/s], Eq. (3-1-1)."""
    c = _c5(c)
    t = np.asarray(t, dtype=np.float64)
    return c[1] + 2.0 * c[2] * t + 3.0 * c[3] * t ** 2 + 4.0 * c[4] * t ** 3


def freq_hz(c, t):
    return freq_rad(c, t) / (2.0 * math.pi)


def phase_accel(c, t):
    """Second derivative of the phase, phi''(t) = 2 c2 + 6 c3 t (+ 12 c4 t^2) [rad/s^2]."""
    c = _c5(c)
    t = np.asarray(t, dtype=np.float64)
    return 2.0 * c[2] + 6.0 * c[3] * t + 12.0 * c[4] * t ** 2


def total_phase(c, t_start, t_end):
    """Phase change over [t_start, t_end] inside one block (numerator of Eq. 4-1-1)."""
    return float(phase(c, t_end) - phase(c, t_start))


def block_total_phase(c, T):
    """phi(T/2) - phi(-T/2), the per-block term of Eq. (4-1-2)."""
    return total_phase(c, -T / 2.0, T / 2.0)


def connect(cs, Ts):
    """Phase connection over consecutive blocks, Eq. (4-1-2).

    Returns (Phi_total [rad], F_int_dop [rad/s]) with T_c = sum of block lengths.
    """
    tot = 0.0
    for c, T in zip(cs, Ts):
        tot += block_total_phase(c, T)
    Tc = float(sum(Ts))
    return tot, tot / Tc


def los_accel(c, t, f_carrier, M2=1.0, three_way=False):
    """Line-of-sight acceleration from phi'' (Eq. 4-2-1) [m/s^2].

    1-way: phi'' = 2 pi f_c a / c;  3-way: phi'' = 4 pi M2 f_c a / c.
    """
    pa = phase_accel(c, t)
    k = 4.0 * math.pi * M2 * f_carrier if three_way else 2.0 * math.pi * f_carrier
    return pa * C_LIGHT / k
