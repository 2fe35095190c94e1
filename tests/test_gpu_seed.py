"""GPU parity of the initial-range estimation (Sec. 3.1.1) against the oracle.

pt_seed_block runs an FFT of three snippets on the device; the oracle does
the same steps with numpy's FFT.  Peak bins must agree exactly (the test
inputs keep the top two bins far apart); frequencies within 1e-8 Hz
(rounding of two different FFTs moves Candan's ratio by ~1e-13 bins);
amplitudes within 1e-10 relative; noise estimates within 1e-9.  The seeded
box must then cover the truth (up to the real-signal mirror) and lead the
DE to it.
"""
import math

import numpy as np
import pytest
import torch

import oracle.seed as oseed
import synth
from gpu_util import block_of, crlb_f0, ctx, settings_of, to_dev
from paper_1906_10598_amd import phasetrack as ptk

pytestmark = pytest.mark.gpu


def _mirror(truth, f0_est):
    """The truth in the orientation the real-signal spectrum reports (f0 > 0)."""
    t = np.array(truth, dtype=np.float64)
    if t[2] * f0_est < 0:
        t[1:5] = -t[1:5]
        t[6:] = -t[6:]
    return t


def _check(b, M, spacing=0, samples=None, on_device=True):
    s = b.samples if samples is None else samples
    ten = torch.from_numpy(np.ascontiguousarray(s))
    blk = block_of(b, ten.cuda() if on_device else ten)
    r = ptk.pt_seed_block(ctx().handle, blk, M, spacing, ptk.current_stream())
    o = oseed.seed_block(np.asarray(s, dtype=np.float64), b.fs, b.ref, M, spacing)
    print(f"[seed {b.name} M={M} spacing={spacing} dev={on_device}] bins {list(r.bin)} "
          f"df {[r.f[k] - o['f'][k] for k in range(3)]}", flush=True)
    assert list(r.bin) == o["bin"]
    assert r.snippet == M
    for k in range(3):
        assert abs(r.f[k] - o["f"][k]) < 1e-8
        assert abs(r.amp[k] - o["amp"][k]) <= 1e-10 * o["amp"][k]
        assert abs(r.noise[k] - o["noise"][k]) < 1e-9
        assert r.t[k] == pytest.approx(o["t"][k], rel=0, abs=1e-15)
    dt = (spacing or b.n // 4) / b.fs
    assert abs(r.f0 - o["f0"]) < 1e-8 * (1 + abs(r.t[1]) / dt)
    assert abs(r.f1 - o["f1"]) < 1e-8 / dt
    assert abs(r.f2 - o["f2"]) < 4e-8 / dt ** 2
    for k in ("A", "sigma", "sd_f0", "sd_f1", "sd_f2", "sd_A"):
        assert getattr(r, k) == pytest.approx(o[k], rel=1e-8, abs=1e-12)
    return r, o


def test_paper_blocks_every_snippet_size():
    mx = ptk.pt_seed_max_snippet(ctx().handle)
    assert mx >= 1024
    sizes = sorted({64, 1024, min(4096, mx), mx})
    for seed in range(2):
        b = synth.config1(seed)
        for M in sizes:
            _check(b, M)


def test_dtypes_host_pointer_and_spacing():
    b = synth.config1(2)
    _check(b, 2048, samples=b.samples.astype(np.float64))
    _check(b, 2048, on_device=False)
    _check(b, 2048, spacing=150_000)
    _check(b, 2048, spacing=1000)  # overlapping snippets are allowed


def test_ragged_block_and_reference():
    b = synth.config1(3, n=100_003)
    _check(b, 1024)
    bb = synth.config1(3, n=100_003)
    bb.ref = 40_000.5
    _check(bb, 512)


def test_invalid_options():
    b = synth.config1(0, n=10_000)
    blk = block_of(b, to_dev(b.samples))
    h = ctx().handle
    for M, sp in ((1000, 0), (32, 0), (1 << 20, 0), (4096, 4000), (2048, -1)):
        with pytest.raises(ptk.PtError):
            ptk.pt_seed_block(h, blk, M, sp)


def test_seeded_box_covers_truth_and_fit_converges():
    mx = ptk.pt_seed_max_snippet(ctx().handle)
    for seed in range(3):
        b = synth.config1(seed)
        dev = to_dev(b.samples)
        r = ptk.pt_seed_block(ctx().handle, block_of(b, dev), mx, 0, ptk.current_stream())
        truth = _mirror(b.truth, r.f0)
        box = ptk.pt_seed_box(r, ptk.PT_RANGE_SIGMA, 10.0, b.n / b.fs)
        lo, hi = np.array(box.lo), np.array(box.hi)
        z = [(r.f0 - truth[2]) / r.sd_f0, (r.f1 - truth[3]) / r.sd_f1, (r.f2 - truth[4]) / r.sd_f2]
        print(f"[seed {seed}] z(f0, f1, f2) = {np.round(z, 2).tolist()} box f2 +-{(hi[4] - lo[4]) / 2:.3f}",
              flush=True)
        assert np.all(lo[[0, 2, 3, 4]] < truth[[0, 2, 3, 4]]) and np.all(truth[[0, 2, 3, 4]] < hi[[0, 2, 3, 4]])
        f = ctx().fit_block(block_of(b, dev, lo=lo, hi=hi), settings_of(b))
        sig = crlb_f0(b)
        print(f"[seed {seed}] seeded fit f0 err {f.coef[2] - truth[2]:.3e} Hz = "
              f"{(f.coef[2] - truth[2]) / sig:.2f} CRLB, flags {f.flags}", flush=True)
        assert abs(f.coef[2] - truth[2]) < 5 * sig
        assert not (f.flags & ptk.PT_FLAG_AT_BOUND)
