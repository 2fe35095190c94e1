"""Plain FP64 CPU oracle of the phase-tracking fit (arXiv:1906.10598).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only users; the product library never imports,
links or calls it, and it imports nothing from the product.

Contents
  * ``liboracle.so`` (``oracle.c``): Philox4x32-10, the chi-square objective
    of Eq. (2-2-4) over the model of Eq. (2-2-2), the correlation objective
    of Eq. (2-2-5) over the constant-amplitude model of Eq. (2-2-6), and DE/rand/1/bin
    (Sec. 1.2, Table 4), all in FP64.
  * :mod:`oracle.derived`: the observables of Sec. 3.1.3 and Sec. 4
    (instantaneous phase and frequency, total-count phase, integration
    Doppler, line-of-sight acceleration), in NumPy FP64.

Parameter vectors have seven slots (ORC_NSLOT): A, phi0 [rad], f0 [Hz],
f1 [Hz/s], f2 [Hz/s^2], Adot [1/s], f3 [Hz/s^3]; t_n = (n - ref) / fs.
"""
import ctypes
import os

import numpy as np

from . import derived  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
NSLOT = 7
OBJ_CHI2, OBJ_COR = 0, 1
TAG_INIT, TAG_MUT, TAG_XOVER = 1, 2, 3
FLAG_CONVERGED, FLAG_MAXGEN, FLAG_VTR, FLAG_AT_BOUND = 1, 2, 4, 8

_lib = None


class _DeCfg(ctypes.Structure):
    _fields_ = [
        ("P", ctypes.c_int),
        ("max_gens", ctypes.c_int),
        ("F", ctypes.c_double),
        ("CR", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_uint64),
        ("vtr", ctypes.c_double),
        ("rel_tol", ctypes.c_double),
        ("window", ctypes.c_int),
        ("lo", ctypes.c_double * NSLOT),
        ("hi", ctypes.c_double * NSLOT),
        ("objective", ctypes.c_int),
    ]


def lib():
    """Load liboracle.so, compiling it first only if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build

            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_draw_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_chi2.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, dp]
        L.orc_chi2.restype = ctypes.c_double
        L.orc_chi2_pop.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                   dp, ctypes.c_int, dp, ctypes.c_int]
        L.orc_cor.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, dp]
        L.orc_cor.restype = ctypes.c_double
        L.orc_obj_pop.argtypes = [ctypes.c_int, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  dp, ctypes.c_int, dp, ctypes.c_int]
        L.orc_de_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ip, ip, ip, ip, dp]
        L.orc_de_trial.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, dp, ctypes.c_int, ip, ctypes.c_double,
                                   ctypes.c_double, dp, dp, dp]
        L.orc_de_init.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, dp, dp, dp]
        L.orc_de_fit.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(_DeCfg), ctypes.c_int, dp, dp, ip, ip, dp, dp, dp]
        L.orc_de_fit.restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def centre_ref(n: int) -> float:
    """Reference sample of the block centre: N/2 (Sec. 2.2, phase origin at the block centre)."""
    return n / 2.0


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (Salmon et al. 2011); returns 4 uint32 words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def draw_words(seed, stream, i, g, tag, call):
    o = (ctypes.c_uint32 * 4)()
    lib().orc_draw_words(seed, stream, i, g, tag, call, o)
    return [int(v) for v in o]


def chi2(s, fs, ref, x):
    """chi^2 of one candidate (Eq. 2-2-4), FP64 with Neumaier summation."""
    s = _f64(s)
    x = _pad(x)[0].copy()
    return lib().orc_chi2(_dptr(s), s.size, float(fs), float(ref), _dptr(x))


def cor(s, fs, ref, x):
    """Correlation objective of Eq. (2-2-5): 1 / (arctan(C) + pi/2), C = sum s (A + Adot t) cos phi."""
    s = _f64(s)
    x = _pad(x)[0].copy()
    return lib().orc_cor(_dptr(s), s.size, float(fs), float(ref), _dptr(x))


def obj_pop(kind, s, fs, ref, pop, nthreads=0):
    s = _f64(s)
    pop = _pad(pop)
    out = np.empty(pop.shape[0], dtype=np.float64)
    lib().orc_obj_pop(int(kind), _dptr(s), s.size, float(fs), float(ref), _dptr(pop), pop.shape[0],
                      _dptr(out), int(nthreads))
    return out


def _padv(v):
    """A parameter vector or bound of <= NSLOT slots, missing slots 0."""
    v = np.asarray(v, dtype=np.float64).ravel()
    if v.size < NSLOT:
        v = np.concatenate([v, np.zeros(NSLOT - v.size)])
    return _f64(v)


def _pad(pop):
    pop = np.asarray(pop, dtype=np.float64)
    if pop.ndim == 1:
        pop = pop[None, :]
    if pop.shape[1] < NSLOT:
        pop = np.concatenate([pop, np.zeros((pop.shape[0], NSLOT - pop.shape[1]))], axis=1)
    return _f64(pop)


def chi2_pop(s, fs, ref, pop, nthreads=0):
    """chi^2 of every row of ``pop`` (P x <= NSLOT, missing slots are 0)."""
    s = _f64(s)
    pop = _pad(pop)
    out = np.empty(pop.shape[0], dtype=np.float64)
    lib().orc_chi2_pop(_dptr(s), s.size, float(fs), float(ref), _dptr(pop), pop.shape[0],
                       _dptr(out), int(nthreads))
    return out


def active_slots(lo, hi):
    lo, hi = _padv(lo), _padv(hi)
    return [j for j in range(NSLOT) if lo[j] < hi[j]]


def de_draws(seed, stream, g, i, P, D):
    r1, r2, r3, jr = (ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int())
    U = np.empty(D, dtype=np.float64)
    lib().orc_de_draws(seed, stream, g, i, P, D, ctypes.byref(r1), ctypes.byref(r2),
                       ctypes.byref(r3), ctypes.byref(jr), _dptr(U))
    return r1.value, r2.value, r3.value, jr.value, U


def de_trial(pop, i, r1, r2, r3, jrand, U, act, F, CR, lo, hi):
    pop = _pad(pop)
    U = _f64(U)
    act_a = (ctypes.c_int * len(act))(*act)
    lo = _padv(lo)
    hi = _padv(hi)
    out = np.empty(NSLOT, dtype=np.float64)
    lib().orc_de_trial(_dptr(pop), i, r1, r2, r3, jrand, _dptr(U), len(act), act_a, F, CR,
                       _dptr(lo), _dptr(hi), _dptr(out))
    return out


def de_init(seed, stream, P, lo, hi):
    lo = _padv(lo)
    hi = _padv(hi)
    out = np.empty((P, NSLOT), dtype=np.float64)
    lib().orc_de_init(seed, stream, P, _dptr(lo), _dptr(hi), _dptr(out))
    return out


def de_fit(s, fs, ref, lo, hi, P, max_gens, F=0.5, CR=0.9, seed=0, stream=0,
           vtr=-np.inf, rel_tol=0.0, window=0, nthreads=0, objective=OBJ_CHI2):
    """Full DE/rand/1/bin fit; returns a dict with best, objective, history, population."""
    s = _f64(s)
    cfg = _DeCfg()
    cfg.P, cfg.max_gens, cfg.F, cfg.CR = P, max_gens, F, CR
    cfg.seed, cfg.stream, cfg.vtr, cfg.rel_tol, cfg.window = seed, stream, vtr, rel_tol, window
    cfg.objective = objective
    lo, hi = _padv(lo), _padv(hi)
    for j in range(NSLOT):
        cfg.lo[j] = float(lo[j])
        cfg.hi[j] = float(hi[j])
    best = np.empty(NSLOT)
    bf = ctypes.c_double()
    gens = ctypes.c_int()
    flags = ctypes.c_int()
    pop = np.empty((P, NSLOT))
    fpop = np.empty(P)
    hist = np.empty(max_gens + 1)
    rc = lib().orc_de_fit(_dptr(s), s.size, float(fs), float(ref), ctypes.byref(cfg),
                          int(nthreads), _dptr(best), ctypes.byref(bf), ctypes.byref(gens),
                          ctypes.byref(flags), _dptr(pop), _dptr(fpop), _dptr(hist))
    if rc != 0:
        raise ValueError("oracle de_fit: invalid arguments")
    return {"x": best, "objective": bf.value, "generations": gens.value, "flags": flags.value,
            "pop": pop, "fpop": fpop, "hist": hist[: gens.value + 1]}
