"""Pins of the oracle's derived observables (Sec. 3.1.3, Sec. 4).

  * the paper's Appendix 1 worked example: from the printed Taylor
    coefficients of eleven consecutive 2 s Mars Express blocks, the border
    phases (mod 2 pi) and frequencies of Eq. (3-1-2) and the per-block total
    phase must reproduce the printed values to the printing precision
    (3 decimals; the printed coefficients are themselves rounded, which
    costs up to 2e-3);
  * closed forms of the cubic: the total phase over a symmetric block is
    2 (c1 T/2 + c3 (T/2)^3); the phase connection of Eq. (4-1-2) over
    contiguous blocks of one continuous cubic equals the phase change of
    that cubic end to end;
  * Eq. (4-2-1): a known line-of-sight acceleration gives the stated phi''.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import derived as d

GOLD = os.path.join(os.path.dirname(__file__), "golden")
TOL = 3e-3


def _wrapdiff(a, b):
    return abs(math.remainder(a - b, 2 * math.pi))


def test_appendix1_borders_and_total_phase():
    rows = np.loadtxt(os.path.join(GOLD, "app1_mex_blocks.txt"))
    T = 2.0
    assert rows.shape == (11, 9)
    for r in rows:
        c = r[:4]
        assert d.block_total_phase(c, T) == pytest.approx(r[4], abs=TOL)
        assert _wrapdiff(float(d.phase_mod2pi(c, -T / 2)), r[5]) < TOL
        assert float(d.freq_rad(c, -T / 2)) == pytest.approx(r[6], abs=TOL)
        assert _wrapdiff(float(d.phase_mod2pi(c, T / 2)), r[7]) < TOL
        assert float(d.freq_rad(c, T / 2)) == pytest.approx(r[8], abs=TOL)


def test_appendix1_continuity_within_noise():
    # adjacent borders agree to within the ~50 mrad phase noise the paper
    # quotes for MEX (Sec. 3.1.3), frequency to well under 1 rad/s
    rows = np.loadtxt(os.path.join(GOLD, "app1_mex_blocks.txt"))
    for a, b in zip(rows[:-1], rows[1:]):
        assert _wrapdiff(float(d.phase_mod2pi(a[:4], 1.0)), float(d.phase_mod2pi(b[:4], -1.0))) < 0.05
        assert abs(float(d.freq_rad(a[:4], 1.0) - d.freq_rad(b[:4], -1.0))) < 0.5


def test_unit_conversion_roundtrip():
    c = d.coefs_from_fit(1.0, 23321.0, -34.4, 0.03)
    assert c[1] == pytest.approx(2 * math.pi * 23321.0, rel=1e-15)
    assert c[2] == pytest.approx(math.pi * -34.4, rel=1e-15)
    assert c[3] == pytest.approx(math.pi * 0.03 / 3, rel=1e-15)
    back = d.fit_from_coefs(*c)
    assert np.allclose(back, (1.0, 23321.0, -34.4, 0.03), rtol=1e-14, atol=0)


def test_symmetric_block_total_closed_form():
    c = (0.3, 1234.5, -7.25, 0.125)
    for T in (0.5, 2.0, 8.0):
        h = T / 2
        assert d.block_total_phase(c, T) == pytest.approx(2 * (c[1] * h + c[3] * h ** 3), rel=1e-14)


def test_connection_of_contiguous_blocks():
    # one cubic over [0, sum T); each block re-expands it about its own
    # centre; the connected phase equals the end-to-end change of the cubic
    phi0, f0, f1, f2 = 0.7, 812.25, 1.5, -0.03
    Ts = [2.0, 4.0, 2.0, 8.0, 20.0]
    cs, t = [], 0.0
    for T in Ts:
        p, g0, g1, g2 = synth.shift_truth(phi0, f0, f1, f2, t + T / 2)
        cs.append(d.coefs_from_fit(p, g0, g1, g2))
        t += T
    tot, fint = d.connect(cs, Ts)
    Tc = sum(Ts)
    exact = 2 * math.pi * (f0 * Tc + f1 * Tc ** 2 / 2 + f2 * Tc ** 3 / 6)
    assert tot == pytest.approx(exact, rel=1e-12)
    assert fint == pytest.approx(exact / Tc, rel=1e-12)


def test_los_acceleration():
    fc, a = 8.4e9, 1.25
    phi2_1way = 2 * math.pi * fc / d.C_LIGHT * a
    c = (0.0, 0.0, phi2_1way / 2, 0.0)   # phi'' = 2 c2
    assert float(d.los_accel(c, 0.3, fc)) == pytest.approx(a, rel=1e-14)
    M2 = 880.0 / 749.0
    phi2_3way = 4 * math.pi * M2 * fc / d.C_LIGHT * a
    c = (0.0, 0.0, phi2_3way / 2, 0.0)
    assert float(d.los_accel(c, -0.3, fc, M2=M2, three_way=True)) == pytest.approx(a, rel=1e-14)
