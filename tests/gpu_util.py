"""Shared helpers of the GPU tests (device context, tensors, tolerances)."""
import math

import numpy as np

import synth
from paper_1906_10598_amd import phasetrack as ptk

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        _CTX = ptk.Context(0)
    return _CTX


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def block_of(b: synth.Block, samples_dev, ref=None, stream=None, lo=None, hi=None):
    return ptk.make_block(samples_dev, b.fs, b.lo if lo is None else lo, b.hi if hi is None else hi,
                          ref=b.ref if ref is None else ref, stream=b.stream if stream is None else stream)


def settings_of(b: synth.Block, gens=None, precision=ptk.PT_PREC_FP64, **kw):
    de = b.de
    args = dict(pop=de.pop, max_gens=de.max_gens if gens is None else gens, F=de.F, CR=de.CR, seed=de.seed,
                vtr=de.vtr, rel_tol=de.rel_tol, window=de.window, precision=precision)
    args.update(kw)
    return ptk.make_settings(**args)


def phase_rounding_bound(s, pop, fs, ref):
    """Largest change of chi^2 that FP64 rounding of the phase can cause:
    each side forms phi with an error of a few ulp of |phi| <= phi_max, which
    moves every residual by at most A * eps_phi, so chi^2 moves by at most
    2 sum|rho| A eps_phi <= 2 sqrt(n chi^2) A eps_phi."""
    n = np.asarray(s).size
    tmax = max(abs(ref), abs(n - 1 - ref)) / fs
    pop = np.atleast_2d(pop)
    phi_max = (np.abs(pop[:, 1]) + 2 * math.pi * (np.abs(pop[:, 2]) * tmax + np.abs(pop[:, 3]) * tmax ** 2 / 2
                                                  + np.abs(pop[:, 4]) * tmax ** 3 / 6))
    return 8 * phi_max * 2.0 ** -53, np.abs(pop[:, 0])


# Per-sample error of the model cosine [relative to A, or rad of phase] of the
# FP64 arithmetics beyond the phase rounding: the per-sample cosine path
# ~1e-16 turns; the phasor path is used only where its dropped terms stay
# below 1e-12 turns, its quadratic correction below 1e-11 and its recurrence
# rounding below 1e-12.
MODEL_PHASE_ERR = {ptk.PT_ARITH_FP64_POLY: 1e-13,
                   ptk.PT_ARITH_FP64_PHASOR: 2 * math.pi * 1e-12 + 1e-11 + 1e-12 + 1e-13}


def model_phase_err(c=None):
    """MODEL_PHASE_ERR of the arithmetic the context's last evaluation used."""
    return MODEL_PHASE_ERR.get(ptk.pt_ctx_last_arithmetic((c or ctx()).handle), 1e-13)


def assert_chi2_close(got, ref, n, amp=1.0, rel=1e-10, eps_phi=None, floor=1e-13):
    """Objectives agree within `rel` relative, with an absolute floor
    n (floor A)^2 (floor: per-sample phase error of the arithmetic, see
    MODEL_PHASE_ERR).  For noise-free data, where chi^2 -> 0 and a relative
    error is undefined, pass eps_phi (per-candidate phase rounding, see
    phase_rounding_bound): the bound becomes
    2 sqrt(n chi^2) A (eps_phi + floor) + n (floor A)^2."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    amp = np.broadcast_to(np.asarray(amp, dtype=np.float64), ref.shape)
    err = np.abs(got - ref)
    tol = np.maximum(rel * np.abs(ref), n * (floor * amp) ** 2)
    if eps_phi is not None:
        tol = np.maximum(tol, 2 * np.sqrt(n * np.abs(ref)) * amp * (eps_phi + floor) + n * (floor * amp) ** 2)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (
        f"{bad.size} objectives outside tolerance; worst rel err "
        f"{float(np.max(err / np.maximum(np.abs(ref), 1e-300))):.3e} at {int(bad[0])}: "
        f"gpu {got[bad[0]]!r} oracle {ref[bad[0]]!r} tol {tol[bad[0]]!r}")


def random_population(rng, lo, hi, P, far=0):
    """P members uniform in the box, plus `far` members well outside it."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    ns = lo.size
    pop = lo + rng.random((P, ns)) * (hi - lo)
    for k in range(min(far, P)):
        w = hi - lo
        pop[k] = lo + (rng.random(ns) * 5 - 2) * np.where(w > 0, w, 1.0)
        for j in (5, 6):  # amplitude slope and quartic term stay off when their box is fixed
            if j < ns and hi[j] == lo[j]:
                pop[k, j] = lo[j]
    return pop


def crlb_f0(b: synth.Block):
    """Cramer-Rao bound on f0 [Hz] of a block over the parameters its box
    frees (Fisher information of the signal model, synth.crlb): with f1 and
    f2 free it is 2.5x the single-tone bound."""
    from synth.crlb import crlb_f0_block

    return crlb_f0_block(b)


# Mixed precision, noise-free FP32 samples of the model at the truth:
# chi^2 / (n A^2) is the mean square of the mixed path's per-sample model
# error.  With the hi/lo split of the linear phase term the FP32 local phase
# stays below one turn, so each of its ~4 roundings is uniform within half an
# ulp of 2^-24 turns: variance 4 (2^-24)^2 / 12 turns^2, (2 pi)^2 times that
# = 4.7e-14 rad^2; the FP32 cosine (1.1e-8), the FP32 samples and residual
# (ulp 6e-8 at |s| < 1) add ~1e-15.  Bound 1e-13.  Without the split the FP32
# product b1 j reaches 0.4 S turns (f0 near 20 kHz at 50 kHz): roundings at an
# ulp of 2^-21 or 2^-20 give 5e-13 (S = 16) and 3e-12 (S = 32) in a CPU
# emulation of the same steps, against 1.2e-14 with it.
MIXED_NOISE_FREE = 1e-13


def mixed_rel_at_optimum(n, chi2, amp, spl=32):
    """Bound on the mixed path's relative chi^2 error at a fitted optimum of
    an n-sample block (chi2: its objective, amp: the amplitude, spl: samples
    per lane, 32 at most).  There the residuals rho are noise of variance
    s^2 = chi2 / n, independent of the mixed model's per-sample error e
    (rms e_m <= sqrt(MIXED_NOISE_FREE) A = 3.2e-7 A), so chi^2 moves by
    2 sum rho e + sum e^2, of rms 2 s e_m sqrt(n): relative 2 (e_m / s) / sqrt(n).
    The FP32 lane sums of spl terms add a relative rounding of rms
    2^-24 / sqrt(3) per addition, 2e-8 spl / sqrt(n) over the block.  The
    bound is five times the sum of the two rms figures: 1.2e-8 for the
    paper-scale block at 0 dB, 1.2e-7 for a 50 000-sample block at 15 dB."""
    s = math.sqrt(chi2 / n)
    e_m = math.sqrt(MIXED_NOISE_FREE) * amp
    return 5.0 * (2.0 * e_m / s + 2e-8 * spl) / math.sqrt(n)
