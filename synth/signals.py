"""Synthetic sample blocks and their truths.

Recipe (also stated in the design notes):
  * tiny block: N = 4096 FP64 samples at fs = 1 kHz,
    s[n] = A cos(phi0 + 2 pi (f0 t + f1 t^2 / 2)) + N(0, sigma^2), t = n / fs,
    A = 1, phi0 ~ U(0, 2 pi), f0 ~ U(50, 450) Hz, f1 ~ U(-0.5, 0.5) Hz/s,
    sigma = 0.3; DE: P = 32, F = 0.5, CR = 0.9, 200 generations; box
    +-(0.2 A, pi, 2 Hz, 1 Hz/s) around the truth, f2 fixed at 0.
  * paper-scale block: N = 400 000 samples at fs = 50 kHz (8 s), cubic phase
    with f0 ~ U(-20, 20) kHz, f1 ~ U(-5, 5) Hz/s, f2 ~ U(-0.05, 0.05) Hz/s^2,
    A = 1, per-sample SNR 0 dB (sigma = A / sqrt 2).  The FP64 signal is
    peak-normalised and quantised to int16, q = round(32767 s / max|s|), and
    stored as FP32 q / 32767.  DE: P = 40, 2000 generations; box
    +-(10 % of A, pi, 0.5 Hz, 0.1 Hz/s, 0.01 Hz/s^2) around the truth.
  * batch: 64 independent blocks, N log-uniform in [50 000, 400 000] at
    50 kHz, truths as the paper-scale block, SNR ~ U(-5, 10) dB, P = 40,
    1500 generations.
  * serving stream: 16 tracks with a continuous cubic phase over the whole
    track, contiguous blocks with N drawn from {1e5, 2e5, 4e5, 1e6}, Poisson
    arrivals at an aggregate 20 blocks/s; int16 with a fixed full scale of
    A + 6 sigma per track (a receiver of fixed gain).

The truths are drawn at the block start (t = n / fs) and reported at the
block's reference sample (the block centre N / 2, Sec. 2.2) by an exact
polynomial shift evaluated in extended precision; the search box is centred
on the shifted truth with unchanged widths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import List, Optional

import numpy as np

NSLOT = 7  # A, phi0 [rad], f0 [Hz], f1 [Hz/s], f2 [Hz/s^2], Adot [1/s], f3 [Hz/s^3]
_SEED_BASE = 0x19061059


@dataclass
class DESettings:
    pop: int
    max_gens: int
    F: float = 0.5
    CR: float = 0.9
    seed: int = 0
    vtr: float = -math.inf
    rel_tol: float = 0.0
    window: int = 0


@dataclass
class Block:
    samples: np.ndarray           # FP32 or FP64, contiguous
    fs: float
    ref: float                    # reference sample (time origin), N / 2
    truth: np.ndarray             # 6 slots at the reference sample
    lo: np.ndarray                # 6 slots
    hi: np.ndarray                # 6 slots
    de: DESettings
    sigma: float                  # noise std in data units
    stream: int = 0               # DE random-stream id of this block
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.samples.size)


def _rng(config_index: int, track: int, seed: int) -> np.random.Generator:
    return np.random.default_rng([_SEED_BASE, 0x8000 * config_index + track, seed])


def shift_truth(phi0, f0, f1, f2, dt):
    """Coefficients of the same cubic phase re-expanded about t = dt.

    phi(t) = phi0 + 2 pi (f0 t + f1 t^2/2 + f2 t^3/6); the shifted set
    satisfies phi(dt + u) = phi0' + 2 pi (f0' u + f1' u^2/2 + f2' u^3/6).
    Evaluated with exact rationals so the truth carries no rounding beyond
    the final conversion; phi0' is returned modulo 2 pi.
    """
    F0, F1, F2, D = Fraction(f0), Fraction(f1), Fraction(f2), Fraction(dt)
    turns = F0 * D + F1 * D * D / 2 + F2 * D * D * D / 6
    frac = turns - math.floor(turns)
    phi = math.fmod(phi0 + 2.0 * math.pi * float(frac), 2.0 * math.pi)
    f0n = float(F0 + F1 * D + F2 * D * D / 2)
    f1n = float(F1 + F2 * D)
    return phi, f0n, f1n, float(F2)


def shift_truth4(phi0, f0, f1, f2, f3, dt):
    """shift_truth for a quartic phase (f3 t^4 / 24 added): returns
    (phi0', f0', f1', f2', f3) about t = dt, exact rationals."""
    F0, F1, F2, F3, D = Fraction(f0), Fraction(f1), Fraction(f2), Fraction(f3), Fraction(dt)
    turns = F0 * D + F1 * D ** 2 / 2 + F2 * D ** 3 / 6 + F3 * D ** 4 / 24
    frac = turns - math.floor(turns)
    phi = math.fmod(phi0 + 2.0 * math.pi * float(frac), 2.0 * math.pi)
    return (phi, float(F0 + F1 * D + F2 * D ** 2 / 2 + F3 * D ** 3 / 6), float(F1 + F2 * D + F3 * D ** 2 / 2),
            float(F2 + F3 * D), float(F3))


def block_from_phase(n, fs, amp, phi0, f0, f1, f2, sigma, rng, quantise, t0=0.0, full_scale=None, f3=0.0):
    """Samples amp * cos(phase(t0 + k/fs)) + noise for k < n (phase at absolute time).

    quantise: int16 codes q / 32767 as FP32, with the block's own peak as full
    scale, or a fixed ``full_scale`` (a receiver with fixed gain; values beyond
    it clip)."""
    k = np.arange(n, dtype=np.float64)
    t = t0 + k / fs
    # phase in turns with exact-integer removal of f0*t0 style large parts
    turns = f0 * t + f1 * t * t / 2.0 + f2 * t * t * t / 6.0
    if f3:
        turns = turns + f3 * t ** 4 / 24.0
    turns = turns - np.floor(turns)
    s = amp * np.cos(phi0 + 2.0 * np.pi * turns)
    if sigma > 0:
        s = s + rng.normal(0.0, sigma, size=n)
    scale = 1.0
    if quantise:
        peak = float(np.max(np.abs(s))) if full_scale is None else float(full_scale)
        q = np.rint(32767.0 * np.clip(s / peak, -1.0, 1.0))
        s = (q / 32767.0).astype(np.float32)
        scale = 1.0 / peak
    return s, scale


def config0(seed: int = 0) -> Block:
    """Tiny FP64 block (4096 samples at 1 kHz, quadratic phase)."""
    rng = _rng(0, 0, seed)
    n, fs, A, sigma = 4096, 1000.0, 1.0, 0.3
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    f0 = rng.uniform(50.0, 450.0)
    f1 = rng.uniform(-0.5, 0.5)
    s, _ = block_from_phase(n, fs, A, phi0, f0, f1, 0.0, sigma, rng, quantise=False)
    ref = n / 2.0
    p, g0, g1, g2 = shift_truth(phi0, f0, f1, 0.0, ref / fs)
    truth = np.array([A, p, g0, g1, 0.0, 0.0, 0.0])
    half = np.array([0.2 * A, math.pi, 2.0, 1.0, 0.0, 0.0, 0.0])
    de = DESettings(pop=32, max_gens=200, F=0.5, CR=0.9, seed=(_SEED_BASE ^ 0xDE) + seed)
    return Block(np.ascontiguousarray(s, dtype=np.float64), fs, ref, truth, truth - half,
                 truth + half, de, sigma, stream=0, name="tiny-4096-fp64")


def _paper_truth(rng):
    f0 = rng.uniform(-20000.0, 20000.0)
    f1 = rng.uniform(-5.0, 5.0)
    f2 = rng.uniform(-0.05, 0.05)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    return phi0, f0, f1, f2


def _paper_block(n, fs, snr_db, rng, gens, seed, stream, name):
    A = 1.0
    sigma = A / math.sqrt(2.0) * 10.0 ** (-snr_db / 20.0)
    phi0, f0, f1, f2 = _paper_truth(rng)
    s, scale = block_from_phase(n, fs, A, phi0, f0, f1, f2, sigma, rng, quantise=True)
    ref = n / 2.0
    p, g0, g1, g2 = shift_truth(phi0, f0, f1, f2, ref / fs)
    a = A * scale
    truth = np.array([a, p, g0, g1, g2, 0.0, 0.0])
    half = np.array([0.1 * a, math.pi, 0.5, 0.1, 0.01, 0.0, 0.0])
    de = DESettings(pop=40, max_gens=gens, F=0.5, CR=0.9, seed=(_SEED_BASE ^ 0xDE) + seed)
    return Block(s, fs, ref, truth, truth - half, truth + half, de, sigma * scale,
                 stream=stream, name=name, meta={"snr_db": snr_db})


def config1(seed: int = 0, n: int = 400_000) -> Block:
    """Paper-scale block: 400 000 int16-quantised FP32 samples at 50 kHz, cubic phase."""
    rng = _rng(1, 0, seed)
    return _paper_block(n, 50_000.0, 0.0, rng, 2000, seed, 0, f"paper-{n}-fp32")


def config3(seed: int = 0, nblocks: int = 64, gens: int = 1500) -> List[Block]:
    """64 independent blocks of uneven length (log-uniform 50 000 .. 400 000)."""
    out = []
    for b in range(nblocks):
        rng = _rng(3, b, seed)
        n = int(round(math.exp(rng.uniform(math.log(50_000), math.log(400_000)))))
        snr = rng.uniform(-5.0, 10.0)
        out.append(_paper_block(n, 50_000.0, snr, rng, gens, seed, b, f"batch-{b}-{n}"))
    return out


def config4_stream(seed: int = 0, ntracks: int = 16, nblocks: int = 160,
                   rate: float = 20.0, lengths=(100_000, 200_000, 400_000, 1_000_000),
                   fs: float = 50_000.0) -> List[dict]:
    """Arrivals of contiguous blocks from tracks with a continuous cubic phase.

    Returns a list of dicts sorted by arrival time, each holding the block
    (samples, truth at its centre, the full box of the paper-scale config
    around the truth) plus its track, sequence number and arrival time [s].
    """
    rng = _rng(4, 0, seed)
    tracks = []
    for k in range(ntracks):
        trng = _rng(4, 1 + k, seed)
        phi0, f0, f1, f2 = _paper_truth(trng)
        snr = 0.0
        tracks.append({"phi0": phi0, "f0": f0, "f1": f1, "f2": f2, "t": 0.0, "seq": 0,
                       "rng": trng, "snr": snr})
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=nblocks))
    order = rng.integers(0, ntracks, size=nblocks)
    out = []
    for idx in range(nblocks):
        k = int(order[idx])
        tr = tracks[k]
        n = int(lengths[int(rng.integers(0, len(lengths)))])
        A = 1.0
        sigma = A / math.sqrt(2.0)
        t0 = tr["t"]
        s, scale = block_from_phase(n, fs, A, tr["phi0"], tr["f0"], tr["f1"], tr["f2"], sigma,
                                    tr["rng"], quantise=True, t0=t0, full_scale=A + 6.0 * sigma)
        ref = n / 2.0
        p, g0, g1, g2 = shift_truth(tr["phi0"], tr["f0"], tr["f1"], tr["f2"], t0 + ref / fs)
        a = A * scale
        truth = np.array([a, p, g0, g1, g2, 0.0, 0.0])
        half = np.array([0.1 * a, math.pi, 0.5, 0.1, 0.01, 0.0, 0.0])
        blk = Block(s, fs, ref, truth, truth - half, truth + half,
                    DESettings(pop=40, max_gens=3000, F=0.5, CR=0.9,
                               seed=(_SEED_BASE ^ 0xDE) + seed, rel_tol=1e-9, window=50),
                    sigma * scale, stream=(k << 32) | tr["seq"], name=f"track{k}-seq{tr['seq']}",
                    meta={"track": k, "seq": tr["seq"], "t0": t0, "scale": scale})
        out.append({"arrival": float(arrivals[idx]), "track": k, "seq": tr["seq"], "block": blk})
        tr["t"] = t0 + n / fs
        tr["seq"] += 1
    return out


def config_quartic(seed: int = 0, n: int = 1_000_000) -> Block:
    """Perigee-like block (Sec. 3.2.1): 20 s at 50 kHz whose phase needs the
    fourth Taylor order.  f0 ~ U(-20, 20) kHz, f1 ~ U(-5, 5) Hz/s,
    f2 ~ U(-0.05, 0.05) Hz/s^2, |f3| ~ U(2e-4, 1e-3) Hz/s^3 with a random sign
    (0.5 to 2.6 rad of quartic phase at the block ends), 0 dB, int16 with the
    block's peak as full scale.  Box: the paper-scale half-widths plus
    f3 +- 2e-4 Hz/s^3; DE P = 40, 2000 generations."""
    rng = _rng(5, 0, seed)
    fs, A = 50_000.0, 1.0
    sigma = A / math.sqrt(2.0)
    phi0, f0, f1, f2 = _paper_truth(rng)
    f3 = float(rng.uniform(2e-4, 1e-3) * rng.choice([-1.0, 1.0]))
    s, scale = block_from_phase(n, fs, A, phi0, f0, f1, f2, sigma, rng, quantise=True, f3=f3)
    ref = n / 2.0
    p, g0, g1, g2, g3 = shift_truth4(phi0, f0, f1, f2, f3, ref / fs)
    a = A * scale
    truth = np.array([a, p, g0, g1, g2, 0.0, g3])
    half = np.array([0.1 * a, math.pi, 0.5, 0.1, 0.01, 0.0, 2e-4])
    de = DESettings(pop=40, max_gens=2000, F=0.5, CR=0.9, seed=(_SEED_BASE ^ 0xDE) + seed)
    return Block(s, fs, ref, truth, truth - half, truth + half, de, sigma * scale,
                 stream=0, name=f"quartic-{n}-fp32")
