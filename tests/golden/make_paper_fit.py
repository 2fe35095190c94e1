"""Write tests/golden/paper_fit_seed<k>.json: the oracle's full fit of the
paper-scale block and the exact least-squares minimiser next to it; with
`--kind cor`, paper_fit_cor_seed<k>.json: the oracle's full fit of the same
block under the correlation objective (Eq. 2-2-5, amplitude fixed at the
truth as Eq. 2-2-6 asks); with `--kind quartic`, quartic_fit_seed<k>.json:
the oracle's full fit of the 20 s quartic-phase block (Sec. 3.2.1) and its
least-squares minimiser.

Calls only oracle/ (the FP64 CPU reference) and NumPy; nothing here touches
the HIP library.  For synth.config1(seed) -- 400 000 int16-quantised samples
at 50 kHz, cubic phase, 0 dB, DE/rand/1/bin with P = 40, F = 0.5, CR = 0.9
and 2000 generations (Sec. 1.2, Table 4; Sec. 1.3's 400K-sample block) -- it
stores

  * the oracle fit: best member, chi^2 (Eq. 2-2-4), generations, flags and
    the best-so-far history every 100 generations;
  * the continuous minimiser of the same chi^2 inside the same box:
    Gauss-Newton steps from the oracle's best member on the residuals
    s_n - A cos(phi(t_n)) in FP64, and its chi^2 evaluated by the oracle.

Usage: python tests/golden/make_paper_fit.py [--kind chi2|cor|quartic] [seed ...]   (default: chi2, 0)
About a minute per seed on 8 cores (the quartic block three).
"""
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def polish(b, x0, iters=8):
    """Minimiser of chi^2 over the box's free slots by Gauss-Newton steps
    from x0: residuals r_n = s_n - A cos(phi(t_n)) in FP64, Jacobian
    dr/dtheta written out, normal equations solved with column scaling."""
    s = b.samples.astype(np.float64)
    t = (np.arange(b.n, dtype=np.float64) - b.ref) / b.fs
    free = [j for j in (0, 1, 2, 3, 4, 6) if j < len(b.lo) and b.lo[j] < b.hi[j]]
    x = np.zeros(7)
    x[: len(x0)] = x0
    for _ in range(iters):
        phi = x[1] + 2 * math.pi * (x[2] * t + x[3] * t * t / 2 + x[4] * t ** 3 / 6 + x[6] * t ** 4 / 24)
        c, sn = np.cos(phi), np.sin(phi)
        r = s - x[0] * c
        g = x[0] * sn  # dr/dphi
        cols = {0: -c, 1: g, 2: 2 * math.pi * t * g, 3: math.pi * t * t * g, 4: math.pi * t ** 3 * g / 3,
                6: math.pi * t ** 4 * g / 12}
        J = np.stack([cols[j] for j in free], axis=1)
        d = np.sqrt(np.sum(J * J, axis=0))
        step = np.linalg.solve((J / d).T @ (J / d), -(J / d).T @ r) / d
        x[free] += step
    return x


def fixed_amplitude_box(b):
    """The correlation objective's box (Eq. 2-2-6): amplitude fixed at the
    truth, no amplitude slope."""
    lo, hi = b.lo.copy(), b.hi.copy()
    lo[0] = hi[0] = b.truth[0]
    lo[5] = hi[5] = 0.0
    return lo, hi


def main(seeds, kind="chi2"):
    for seed in seeds:
        b = synth.config_quartic(seed) if kind == "quartic" else synth.config1(seed)
        lo, hi = fixed_amplitude_box(b) if kind == "cor" else (b.lo, b.hi)
        obj = oracle.OBJ_COR if kind == "cor" else oracle.OBJ_CHI2
        s64 = b.samples.astype(np.float64)
        t0 = time.time()
        r = oracle.de_fit(s64, b.fs, b.ref, lo, hi, b.de.pop, b.de.max_gens, F=b.de.F, CR=b.de.CR,
                          seed=b.de.seed, stream=b.stream, objective=obj)
        dt = time.time() - t0
        name = {"chi2": "config1", "cor": "config1", "quartic": "config_quartic"}[kind]
        out = {
            "block": f"synth.{name}({seed})", "kind": kind, "n": b.n, "fs": b.fs, "ref": b.ref,
            "de": {"pop": b.de.pop, "max_gens": b.de.max_gens, "F": b.de.F, "CR": b.de.CR, "seed": b.de.seed,
                   "stream": b.stream},
            "box": {"lo": [float(v) for v in lo], "hi": [float(v) for v in hi]},
            "oracle_fit": {"x": [float(v) for v in r["x"]], "objective": float(r["objective"]),
                           "generations": int(r["generations"]), "flags": int(r["flags"]),
                           "hist_every_100": [float(v) for v in r["hist"][::100]], "seconds": dt},
            "truth": [float(v) for v in b.truth],
        }
        msg = f"{kind} seed {seed}: oracle fit {dt:.1f} s, f0 {r['x'][2]!r}, objective {r['objective']!r}"
        if kind != "cor":
            # the least-squares minimiser is chi^2's; the correlation objective's
            # optimum differs from it by the amplitude it fixes
            xp = polish(b, r["x"])
            free = [j for j in range(len(b.lo)) if b.lo[j] < b.hi[j]]
            inside = bool(all(b.lo[j] <= xp[j] <= b.hi[j] for j in free))
            out["minimiser"] = {"x": [float(v) for v in xp], "objective": float(oracle.chi2(s64, b.fs, b.ref, xp)),
                                "inside_box": inside}
            msg += f"; minimiser f0 {xp[2]!r} (diff {r['x'][2] - xp[2]:.3e} Hz), chi2 {out['minimiser']['objective']!r}"
        prefix = {"chi2": "paper_fit", "cor": "paper_fit_cor", "quartic": "quartic_fit"}[kind]
        with open(os.path.join(HERE, f"{prefix}_seed{seed}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(msg, flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    kind = "chi2"
    if args[:1] == ["--kind"]:
        kind, args = args[1], args[2:]
    main([int(a) for a in args] or [0], kind)
