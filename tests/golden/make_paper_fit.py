"""Write tests/golden/paper_fit_seed<k>.json: the oracle's full fit of the
paper-scale block and the exact least-squares minimiser next to it.

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

Usage: python tests/golden/make_paper_fit.py [seed ...]   (default: 0)
About a minute per seed on 8 cores.
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
    free = [j for j in range(5) if b.lo[j] < b.hi[j]]
    x = np.array(x0, dtype=np.float64)
    for _ in range(iters):
        phi = x[1] + 2 * math.pi * (x[2] * t + x[3] * t * t / 2 + x[4] * t ** 3 / 6)
        c, sn = np.cos(phi), np.sin(phi)
        r = s - x[0] * c
        g = x[0] * sn  # dr/dphi
        cols = {0: -c, 1: g, 2: 2 * math.pi * t * g, 3: math.pi * t * t * g, 4: math.pi * t ** 3 * g / 3}
        J = np.stack([cols[j] for j in free], axis=1)
        d = np.sqrt(np.sum(J * J, axis=0))
        step = np.linalg.solve((J / d).T @ (J / d), -(J / d).T @ r) / d
        x[free] += step
    return x


def main(seeds):
    for seed in seeds:
        b = synth.config1(seed)
        s64 = b.samples.astype(np.float64)
        t0 = time.time()
        r = oracle.de_fit(s64, b.fs, b.ref, b.lo, b.hi, b.de.pop, b.de.max_gens, F=b.de.F, CR=b.de.CR,
                          seed=b.de.seed, stream=b.stream)
        dt = time.time() - t0
        xp = polish(b, r["x"])
        inside = bool(np.all(xp[:5] >= b.lo[:5]) and np.all(xp[:5] <= b.hi[:5]))
        out = {
            "block": f"synth.config1({seed})", "n": b.n, "fs": b.fs, "ref": b.ref,
            "de": {"pop": b.de.pop, "max_gens": b.de.max_gens, "F": b.de.F, "CR": b.de.CR, "seed": b.de.seed,
                   "stream": b.stream},
            "oracle_fit": {"x": [float(v) for v in r["x"]], "objective": float(r["objective"]),
                           "generations": int(r["generations"]), "flags": int(r["flags"]),
                           "hist_every_100": [float(v) for v in r["hist"][::100]], "seconds": dt},
            "minimiser": {"x": [float(v) for v in xp], "objective": float(oracle.chi2(s64, b.fs, b.ref, xp)),
                          "inside_box": inside},
            "truth": [float(v) for v in b.truth],
        }
        path = os.path.join(HERE, f"paper_fit_seed{seed}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"seed {seed}: oracle fit {dt:.1f} s, f0 {r['x'][2]!r} vs minimiser {xp[2]!r} "
              f"(diff {r['x'][2] - xp[2]:.3e} Hz), chi2 {r['objective']!r} vs {out['minimiser']['objective']!r}",
              flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0])
