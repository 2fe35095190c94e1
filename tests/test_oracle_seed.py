"""Pins of the range-determination and continuity oracle (Sec. 3.1.1, 3.1.3).

  * a noise-free real tone on an FFT bin gives that frequency and amplitude
    exactly (the image at -f is orthogonal on a bin);
  * off-bin tones: Candan's corrected interpolator is unbiased for one
    complex exponential; the real tone's image at -f shifts the estimate by
    far less than 1e-5 bins and the DTFT amplitude by at most
    A / (M sin(2 pi k / M)), the image's own magnitude;
  * a linear chirp gives f1 and a cubic phase gives f2 by the difference
    formulas (closed forms of the instantaneous frequency);
  * in white noise the frequency error stays within the Cramer-Rao bound the
    oracle reports, and the noise estimate recovers sigma;
  * border continuity is zero for one continuous phase split in two blocks,
    and returns a planted phase jump wrapped to (-pi, pi].
"""
import math

import numpy as np
import pytest

from oracle import seed

FS = 50_000.0


def _tone(M, k, A=0.7, phi=1.1):
    n = np.arange(M, dtype=np.float64)
    return A * np.cos(2 * math.pi * k * n / M + phi)


@pytest.mark.parametrize("M", [1024, 4096, 8192])
def test_on_bin_tone_is_exact(M):
    for k in (M // 8, M // 4 + 3, 3 * M // 8):
        f, A, sg, kb = seed.snippet_estimate(_tone(M, k), FS)
        assert kb == k
        assert abs(f - k * FS / M) < 1e-9 * FS / M
        assert abs(A - 0.7) < 1e-12
        assert sg < 1e-6


def test_off_bin_tone_within_image_bound():
    M = 4096
    rng = np.random.default_rng(3)
    for _ in range(100):
        k = rng.uniform(M / 8, 3 * M / 8)
        f, A, sg, kb = seed.snippet_estimate(_tone(M, k, 1.0, rng.uniform(0, 2 * math.pi)), FS)
        assert kb in (math.floor(k), math.ceil(k))
        assert abs(f * M / FS - k) < 1e-5
        assert abs(A - 1.0) <= 1.0 / (M * math.sin(2 * math.pi * k / M)) + 1e-12


def _chirp(N, f0, f1, f2, phi, ref, A=1.0, sigma=0.0, rng=None):
    t = (np.arange(N, dtype=np.float64) - ref) / FS
    x = A * np.cos(phi + 2 * math.pi * (f0 * t + f1 * t ** 2 / 2 + f2 * t ** 3 / 6))
    if sigma:
        x = x + rng.normal(0.0, sigma, N)
    return x


def test_chirp_rate_and_acceleration_by_differences():
    N, M = 400_000, 4096
    ref = N / 2
    for f0, f1, f2 in ((7000.0, 3.0, 0.0), (-12000.0, -4.0, 0.04), (15000.0, 0.5, -0.05)):
        x = _chirp(N, f0, f1, f2, 0.3, ref)
        r = seed.seed_block(x, FS, ref, M)
        # a real tone shows |f|: the estimate is the mirror image for f0 < 0
        sgn = 1.0 if f0 > 0 else -1.0
        dt = (N // 4) / FS
        bin_hz = FS / M
        # per-snippet error <= 1e-4 bin (chirp sweep inside a snippet is << 1 bin)
        assert abs(r["f0"] - sgn * f0) < 1e-4 * bin_hz + abs(f1) * 1e-6
        assert abs(r["f1"] - sgn * f1) < 2e-4 * bin_hz / (2 * dt) + abs(f2) * dt
        assert abs(r["f2"] - sgn * f2) < 4e-4 * bin_hz / dt ** 2
        assert abs(r["A"] - 1.0) < 1e-3


def test_noise_errors_within_reported_bound():
    N, M = 400_000, 4096
    rng = np.random.default_rng(5)
    z0, z1, s_rel = [], [], []
    for _ in range(24):
        f0 = rng.uniform(3000, 20000)
        f1 = rng.uniform(-5, 5)
        sigma = 1.0 / math.sqrt(2.0)  # 0 dB
        x = _chirp(N, f0, f1, 0.0, rng.uniform(0, 6.28), N / 2, sigma=sigma, rng=rng)
        r = seed.seed_block(x, FS, N / 2, M)
        z0.append((r["f0"] - f0) / r["sd_f0"])
        z1.append((r["f1"] - f1) / r["sd_f1"])
        s_rel.append(r["sigma"] / sigma - 1)
    assert np.max(np.abs(z0)) < 5 and np.max(np.abs(z1)) < 5
    assert 0.3 < np.std(z0) < 2.0
    assert np.max(np.abs(s_rel)) < 0.05


def test_snippet_outside_block_is_rejected():
    with pytest.raises(ValueError):
        seed.seed_block(np.zeros(1000), FS, 500.0, 1024)


def _fit(phi0, f0, f1, f2, tl, tr):
    return {"phi0": phi0, "f0": f0, "f1": f1, "f2": f2, "t_left": tl, "t_right": tr}


def _shift(phi0, f0, f1, f2, dt):
    # the same cubic phase re-expanded about t = dt
    return (phi0 + 2 * math.pi * (f0 * dt + f1 * dt ** 2 / 2 + f2 * dt ** 3 / 6),
            f0 + f1 * dt + f2 * dt ** 2 / 2, f1 + f2 * dt, f2)


def test_border_continuity():
    T = 2.0
    a = (0.4, 1234.5, 0.8, 0.01)
    b = _shift(*a, T)  # next block's centre is T later
    fa = _fit(*a, -T / 2, T / 2)
    fb = _fit(*b, -T / 2, T / 2)
    dphi, dfreq = seed.border_continuity(fa, fb)
    assert abs(dphi) < 1e-9 and abs(dfreq) < 1e-12
    for jump, want in ((0.3, -0.3), (2 * math.pi + 0.1, -0.1), (-2 * math.pi - 0.2, 0.2)):
        fb2 = dict(fb, phi0=fb["phi0"] + jump)
        dphi, _ = seed.border_continuity(fa, fb2)
        assert abs(dphi - want) < 1e-9
    fb3 = dict(fb, f0=fb["f0"] + 0.05)
    assert abs(seed.border_continuity(fa, fb3)[1] + 0.05) < 1e-12


def _r(**kw):
    base = dict(A=2.0, f0=1000.0, f1=-4.0, f2=0.02, sd_f0=0.01, sd_f1=0.003, sd_f2=0.004, sd_A=0.001)
    base.update(kw)
    return base


def test_seed_box_paper_rule_hand_worked():
    lo, hi = seed.seed_box(_r(), "paper", 10.0, 8.0, slope=True)
    want_lo = [1.8, 0.0, 900.0, -4.4, -150 / math.pi, -0.05, 0.0]
    want_hi = [2.2, 2 * math.pi, 1100.0, -3.6, 150 / math.pi, 0.05, 0.0]
    assert np.allclose(lo, want_lo, rtol=0, atol=1e-12) and np.allclose(hi, want_hi, rtol=0, atol=1e-12)
    # f1 near zero: the printed 10 % would collapse the range; nsig standard errors floor it
    lo, hi = seed.seed_box(_r(f1=0.001), "paper", 10.0, 8.0)
    assert math.isclose(hi[3] - lo[3], 0.06, rel_tol=1e-12)
    assert lo[5] == hi[5] == 0.0


def test_seed_box_sigma_rule_hand_worked():
    lo, hi = seed.seed_box(_r(), "sigma", 10.0, 8.0)
    want_lo = [1.8, 0.0, 999.9, -4.03, -0.02, 0.0, 0.0]
    want_hi = [2.2, 2 * math.pi, 1000.1, -3.97, 0.06, 0.0, 0.0]
    assert np.allclose(lo, want_lo, rtol=0, atol=1e-12) and np.allclose(hi, want_hi, rtol=0, atol=1e-12)
    lo, hi = seed.seed_box(_r(sd_A=0.05), "sigma", 10.0, 8.0)
    assert math.isclose(hi[0] - lo[0], 1.0, rel_tol=1e-12)  # 10 sd_A beats 10 %


def test_predict_is_the_same_phase():
    c = [1.0, 0.7, 1234.5, 0.8, 0.01, 0.0]
    for dt in (2.0, -3.0, 8.0):
        p = seed.predict(c, dt)
        for t in (-1.0, 0.0, 0.5):
            a = c[1] + 2 * math.pi * (c[2] * (dt + t) + c[3] * (dt + t) ** 2 / 2 + c[4] * (dt + t) ** 3 / 6)
            b = p[1] + 2 * math.pi * (p[2] * t + p[3] * t ** 2 / 2 + p[4] * t ** 3 / 6)
            assert abs(math.remainder(a - b, 2 * math.pi)) < 1e-8


def test_running_box_properties():
    c = [1.0, 0.3, 5000.0, 2.5, 0.0, 0.0]
    n, fs = 400_000, 50_000.0
    T = n / fs
    glo = [0.9, 0.3 - math.pi, 4999.5, 2.4, -0.01, 0.0]
    ghi = [1.1, 0.3 + math.pi, 5000.5, 2.6, 0.01, 0.0]
    # warm rule: given half-widths times 0.7 around the prediction at the new centre
    lo, hi = seed.running_box(c, T / 2, n, fs, n / 2, glo, ghi, 0.7, False)
    pred = seed.predict(c, T)
    for j in range(5):
        assert math.isclose((hi[j] + lo[j]) / 2, pred[j], rel_tol=1e-12, abs_tol=1e-12)
        assert math.isclose(hi[j] - lo[j], 0.7 * (ghi[j] - glo[j]), rel_tol=1e-9)
    # running range: a constant frequency rate sweeps |f1| T over the new block,
    # centred on the prediction at the block centre
    lo, hi = seed.running_box(c, T / 2, n, fs, n / 2, glo, ghi, 0.7, True)
    assert math.isclose(hi[2] - lo[2], abs(c[3]) * T, rel_tol=1e-12)
    assert math.isclose((hi[2] + lo[2]) / 2, pred[2], rel_tol=1e-14)
    assert math.isclose(hi[3] - lo[3], 0.7 * 0.2, rel_tol=1e-9)  # no f2: the floor
    assert math.isclose(hi[0] - lo[0], 0.2, rel_tol=1e-12)
