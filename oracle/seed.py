"""Range determination and continuity checking around the fit (FP64, NumPy).

TEST INFRASTRUCTURE ONLY (part of the oracle).  It shares no code with the
HIP path.

Sec. 3.1.1 (initial range): the instantaneous frequency at the block centre
comes from an FFT of a short piece of data at the centre, the frequency rate
from a central difference of three equally spaced frequency estimates, and
the amplitude from the same FFT.  Written out here as:

  * snippet k (k = -1, 0, +1) holds M samples centred on ref + k * spacing;
  * its periodogram peak bin k* is the argmax of |X_b|^2 over 1 <= b < M/2
    (lowest b on ties), X = numpy.fft.fft of the snippet;
  * the peak is refined between bins with Candan's estimator for a
    rectangular window, d = tan(pi/M)/(pi/M) * Re[(X_{k*-1} - X_{k*+1}) /
    (2 X_{k*} - X_{k*-1} - X_{k*+1})], f = (k* + d) fs / M;
  * the amplitude is 2 |sum_n x_n exp(-2 pi i f n / fs)| / M at that f;
  * the noise variance is the snippet's mean power minus the tone's,
    mean(x^2) - A^2 / 2 (floored at 0);
  * a snippet's frequency belongs to the mid-time of its samples; with
    dt = spacing / fs, f1 = (f_+ - f_-) / (2 dt), f2 = (f_+ - 2 f_c + f_-) / dt^2,
    and f0 is the middle snippet's frequency f_c moved to ref with f1.

Standard errors use the single-tone Cramer-Rao bound with the measured
noise: sd_f = sqrt(6) sigma / (pi A T_s sqrt(M)) with T_s = M / fs, then the
difference formulas propagate it.

Sec. 3.1.3 (continuity): phase and frequency of adjacent blocks at their
common border, Eq. (3-1-2).
"""
import math

import numpy as np


def snippet_estimate(x, fs):
    """(f [Hz], A, sigma, k*) of one snippet (the steps listed above)."""
    x = np.asarray(x, dtype=np.float64)
    M = x.size
    X = np.fft.fft(x)
    half = M // 2
    pw = np.abs(X[1:half]) ** 2
    k = 1 + int(np.argmax(pw))
    d = 0.0
    num = X[k - 1] - X[k + 1]  # 0 <= k - 1 and k + 1 <= M / 2 < M
    den = 2.0 * X[k] - X[k - 1] - X[k + 1]
    if den != 0:
        d = math.tan(math.pi / M) / (math.pi / M) * float(np.real(num / den))
    f = (k + d) * fs / M
    n = np.arange(M, dtype=np.float64)
    ang = 2.0 * math.pi * f * n / fs
    Y = np.sum(x * np.cos(ang)) - 1j * np.sum(x * np.sin(ang))
    A = 2.0 * abs(Y) / M
    var = max(float(np.mean(x * x)) - A * A / 2.0, 0.0)
    return f, A, math.sqrt(var), k


def seed_block(s, fs, ref, M, spacing=0):
    """Initial-range estimates of Sec. 3.1.1 for the block ``s``.

    Snippet centres: ref - spacing, ref, ref + spacing (spacing = N // 4 when
    0), each snippet [c - M/2, c + M/2) with c = floor(centre).  Returns a dict
    with the per-snippet estimates and f0, f1, f2, A, sigma and their
    standard errors."""
    s = np.asarray(s)
    N = s.size
    if spacing <= 0:
        spacing = N // 4
    out = {"f": [], "amp": [], "noise": [], "bin": [], "t": []}
    for k in (-1, 0, 1):
        c = int(math.floor(ref)) + k * spacing
        lo = c - M // 2
        if lo < 0 or lo + M > N:
            raise ValueError("snippet outside the block")
        f, A, sg, b = snippet_estimate(s[lo:lo + M], fs)
        out["f"].append(f)
        out["amp"].append(A)
        out["noise"].append(sg)
        out["bin"].append(b)
        out["t"].append((lo + (M - 1) / 2.0 - ref) / fs)  # mid-time of the snippet's samples
    dt = spacing / fs
    fm, fc, fp = out["f"]
    f1 = (fp - fm) / (2.0 * dt)
    f0 = fc - f1 * out["t"][1]  # the middle snippet sits half a sample before ref (even M)
    A = out["amp"][1]
    sigma = out["noise"][1]
    Ts = M / fs
    sd_f = math.sqrt(6.0) * sigma / (math.pi * A * Ts * math.sqrt(M)) if A > 0 else math.inf
    out.update(f0=f0, f1=f1, f2=(fp - 2.0 * fc + fm) / (dt * dt), A=A, sigma=sigma,
               sd_f0=sd_f, sd_f1=math.sqrt(2.0) * sd_f / (2.0 * dt), sd_f2=math.sqrt(6.0) * sd_f / (dt * dt),
               sd_A=sigma * math.sqrt(2.0 / M))
    return out


def border_continuity(fit_a, fit_b):
    """Eq. (3-1-2) at the border of block a (left) and block b (right):
    (phase difference wrapped to (-pi, pi] [rad], frequency difference [Hz]).
    fit_x holds phi0, f0, f1, f2 (and optionally f3) at its own reference and
    t_left / t_right."""
    def ph(x, t):
        return x["phi0"] + 2.0 * math.pi * (x["f0"] * t + x["f1"] * t * t / 2.0 + x["f2"] * t ** 3 / 6.0
                                            + x.get("f3", 0.0) * t ** 4 / 24.0)

    def fr(x, t):
        return x["f0"] + x["f1"] * t + x["f2"] * t * t / 2.0 + x.get("f3", 0.0) * t ** 3 / 6.0

    d = ph(fit_a, fit_a["t_right"]) - ph(fit_b, fit_b["t_left"])
    d = math.remainder(d, 2.0 * math.pi)
    return d, fr(fit_a, fit_a["t_right"]) - fr(fit_b, fit_b["t_left"])


def seed_box(r, rule, nsig, T, slope=False):
    """Search box (lo[6], hi[6]) from seed estimates ``r`` (a dict as returned
    by seed_block).  rule "paper" takes Sec. 3.1.1's widths as printed: phi0
    over one turn [0, 2 pi], f0 and A +-10 %, f1 +-10 % floored at nsig
    standard errors (no width is printed for it), f2 from c3 in [-50, 50]
    rad/s^3, i.e. +-150/pi Hz/s^2; rule "sigma" takes nsig standard errors for
    f0, f1, f2 and max(10 %, nsig sd_A) for A.  Adot: +-0.2 A / T with slope."""
    mid = [r["A"], math.pi, r["f0"], r["f1"], 0.0, 0.0, 0.0]
    half = [0.0, math.pi, 0.0, 0.0, 0.0, 0.2 * r["A"] / T if slope else 0.0, 0.0]
    if rule == "paper":
        half[0] = 0.1 * r["A"]
        half[2] = 0.1 * abs(r["f0"])
        half[3] = max(0.1 * abs(r["f1"]), nsig * r["sd_f1"])
        half[4] = 150.0 / math.pi
    else:
        half[0] = max(0.1 * r["A"], nsig * r["sd_A"])
        half[2] = nsig * r["sd_f0"]
        half[3] = nsig * r["sd_f1"]
        mid[4] = r["f2"]
        half[4] = nsig * r["sd_f2"]
    return [m - h for m, h in zip(mid, half)], [m + h for m, h in zip(mid, half)]


def predict(c, dt):
    """The fitted phase (A, phi0, f0, f1, f2, Adot[, f3]) re-expanded dt seconds
    later (exact Taylor shift of the quartic; phi0 reduced to [0, 2 pi))."""
    A, phi0, f0, f1, f2, Ad = c[:6]
    f3 = c[6] if len(c) > 6 else 0.0
    ph = phi0 + 2.0 * math.pi * (f0 * dt + f1 * dt * dt / 2.0 + f2 * dt ** 3 / 6.0 + f3 * dt ** 4 / 24.0)
    out = [A + Ad * dt, ph % (2.0 * math.pi), f0 + f1 * dt + f2 * dt * dt / 2.0 + f3 * dt ** 3 / 6.0,
           f1 + f2 * dt + f3 * dt * dt / 2.0, f2 + f3 * dt, Ad]
    return out + [f3] if len(c) > 6 else out


def running_box(c, t_since, n, fs, ref, given_lo, given_hi, narrow, extrapolate):
    """Box of a track's next block from the previous fit ``c``.

    t_since: seconds from the previous fit's reference sample to the end of
    its block (the new block's first sample).  Warm rule: the given box's
    half-widths times ``narrow`` around the prediction at the new reference.
    Running-range rule of Sec. 3.1.1 (extrapolate): f0 spans the previous
    fit's frequency F(t) = f0 + f1 t + f2 t^2 / 2 from the new block's start
    to its end, f1 likewise f1 + f2 t, each widened to at least the warm
    half-width around the interval's middle; A is the prediction +-10 %."""
    pred = predict(c, t_since + ref / fs)
    lo, hi = list(given_lo), list(given_hi)
    half = [(h - l) / 2.0 for l, h in zip(given_lo, given_hi)]
    for j in range(min(len(half), len(pred))):
        if half[j] > 0:
            lo[j] = pred[j] - narrow * half[j]
            hi[j] = pred[j] + narrow * half[j]
    if extrapolate:
        ta, tb = t_since, t_since + n / fs
        g3 = c[6] if len(c) > 6 else 0.0
        F = lambda t: c[2] + c[3] * t + c[4] * t * t / 2.0 + g3 * t ** 3 / 6.0  # noqa: E731
        R = lambda t: c[3] + c[4] * t + g3 * t * t / 2.0  # noqa: E731
        for j, g in ((2, F), (3, R)):
            if half[j] > 0:
                a, b = sorted((g(ta), g(tb)))
                m = (a + b) / 2.0
                lo[j] = min(a, m - narrow * half[j])
                hi[j] = max(b, m + narrow * half[j])
        if half[0] > 0:
            lo[0] = pred[0] - 0.1 * abs(pred[0])
            hi[0] = pred[0] + 0.1 * abs(pred[0])
    return lo, hi
