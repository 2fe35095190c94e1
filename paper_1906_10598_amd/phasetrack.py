"""ctypes binding of libphasetrack.so (the C ABI declared in include/phasetrack.h).

Argument marshalling only: every step of the fit runs in the library's HIP
kernels.  The entry points keep the C names (``pt_fit_block`` ...);
:class:`Context` adds a little convenience for torch tensors (device memory
and the current HIP stream come from torch, nothing else does).

Loading fails loudly when the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

NSLOT = 7  # A, phi0, f0, f1, f2, Adot, f3
MAX_POP = 1024
PT_NOALLOC_SCRATCH_BYTES = 4 << 20  # device array of pt_objective_noalloc
PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_EBUSY, PT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PT_F32, PT_F64 = 0, 1
PT_PREC_FP64, PT_PREC_MIXED = 0, 1
PT_FLAG_CONVERGED, PT_FLAG_MAXGEN, PT_FLAG_VTR, PT_FLAG_AT_BOUND = 1, 2, 4, 8
PT_FLAG_ABANDONED, PT_FLAG_DISCONTINUOUS = 16, 32
PT_RANGE_PAPER, PT_RANGE_SIGMA = 0, 1
PT_RUN_WARM, PT_RUN_EXTRAPOLATE = 0, 1
PT_LAUNCH_AUTO, PT_LAUNCH_GRAPH, PT_LAUNCH_PERSISTENT = 0, 1, 2
PT_FP64_AUTO, PT_FP64_POLY = 0, 1
PT_OBJ_CHI2, PT_OBJ_COR = 0, 1
PT_ARITH_FP64_POLY, PT_ARITH_MIXED, PT_ARITH_FP64_PHASOR = 0, 1, 2
PT_FUSION_OFF, PT_FUSION_LEAD, PT_FUSION_LAST, PT_FUSION_AUTO = 0, 1, 2, 3

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libphasetrack.so")


class PtError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


class pt_box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * NSLOT), ("hi", ctypes.c_double * NSLOT)]


class pt_de_settings(ctypes.Structure):
    _fields_ = [
        ("pop", ctypes.c_int32),
        ("max_gens", ctypes.c_int32),
        ("F", ctypes.c_double),
        ("CR", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("vtr", ctypes.c_double),
        ("rel_tol", ctypes.c_double),
        ("window", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("objective", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class pt_block(ctypes.Structure):
    _fields_ = [
        ("samples", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("dtype", ctypes.c_int32),
        ("on_device", ctypes.c_int32),
        ("fs", ctypes.c_double),
        ("ref", ctypes.c_double),
        ("stream", ctypes.c_uint64),
        ("box", pt_box),
    ]


class pt_fit(ctypes.Structure):
    _fields_ = [
        ("coef", ctypes.c_double * NSLOT),
        ("objective", ctypes.c_double),
        ("generations", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("ref", ctypes.c_double),
        ("t_left", ctypes.c_double),
        ("t_right", ctypes.c_double),
        ("phase_centre", ctypes.c_double),
        ("phase_left", ctypes.c_double),
        ("phase_right", ctypes.c_double),
        ("freq_left", ctypes.c_double),
        ("freq_right", ctypes.c_double),
        ("total_phase", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: (list(getattr(self, k)) if k == "coef" else getattr(self, k)) for k, _ in self._fields_}


class pt_server_config(ctypes.Structure):
    _fields_ = [
        ("max_slots", ctypes.c_int32),
        ("gens_per_step", ctypes.c_int32),
        ("max_pending", ctypes.c_int32),
        ("spl", ctypes.c_int32),
        ("cpg", ctypes.c_int32),
        ("range_rule", ctypes.c_int32),
        ("warm_narrow", ctypes.c_double),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("de", pt_de_settings),
        ("seed_first", ctypes.c_int32),
        ("seed_snippet", ctypes.c_int32),
        ("seed_nsig", ctypes.c_double),
        ("max_attempts", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("enlarge", ctypes.c_double),
        ("qc_phase_rad", ctypes.c_double),
        ("qc_freq_hz", ctypes.c_double),
    ]


class pt_server_result(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_uint64),
        ("track", ctypes.c_int32),
        ("warm", ctypes.c_int32),
        ("t_submit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("box", pt_box),
        ("fit", pt_fit),
        ("attempts", ctypes.c_int32),
        ("qc", ctypes.c_int32),
        ("border_dphi", ctypes.c_double),
        ("border_dfreq", ctypes.c_double),
    ]


class pt_seed_opts(ctypes.Structure):
    _fields_ = [("snippet", ctypes.c_int32), ("reserved", ctypes.c_int32), ("spacing", ctypes.c_int64)]


class pt_seed(ctypes.Structure):
    _fields_ = [
        ("f", ctypes.c_double * 3),
        ("amp", ctypes.c_double * 3),
        ("noise", ctypes.c_double * 3),
        ("t", ctypes.c_double * 3),
        ("bin", ctypes.c_int32 * 3),
        ("snippet", ctypes.c_int32),
        ("f0", ctypes.c_double),
        ("f1", ctypes.c_double),
        ("f2", ctypes.c_double),
        ("A", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("sd_f0", ctypes.c_double),
        ("sd_f1", ctypes.c_double),
        ("sd_f2", ctypes.c_double),
        ("sd_A", ctypes.c_double),
    ]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p
_CTX = ctypes.c_void_p


def _signatures(L):
    i32, i64 = ctypes.c_int, ctypes.c_int64
    spec = {
        "pt_version": ([], i32),
        "pt_last_error": ([], ctypes.c_char_p),
        "pt_ctx_create": ([i32, ctypes.POINTER(_CTX)], i32),
        "pt_ctx_destroy": ([_CTX], None),
        "pt_fit_block": ([_CTX, ctypes.POINTER(pt_block), ctypes.POINTER(pt_de_settings), _VP,
                          ctypes.POINTER(pt_fit)], i32),
        "pt_fit_batch": ([_CTX, ctypes.POINTER(pt_block), i32, ctypes.POINTER(pt_de_settings), _VP,
                          ctypes.POINTER(pt_fit)], i32),
        "pt_objective": ([_CTX, ctypes.POINTER(pt_block), _VP, i32, i32, i32, _VP, _VP], i32),
        "pt_objective_noalloc": ([_CTX, ctypes.POINTER(pt_block), _VP, i32, i32, i32, _VP, _VP], i32),
        "pt_last_population": ([_CTX, i32, _DP, _DP, i32], i32),
        "pt_last_history": ([_CTX, i32, _DP, i32, ctypes.POINTER(i32)], i32),
        "pt_phase": ([ctypes.POINTER(pt_fit), _DP, i64, _DP, _DP, _DP, _DP], i32),
        "pt_total_phase": ([ctypes.POINTER(pt_fit), ctypes.c_double, ctypes.c_double, _DP, _DP], i32),
        "pt_connect_phase": ([ctypes.POINTER(pt_fit), i32, _DP, _DP], i32),
        "pt_los_accel": ([ctypes.POINTER(pt_fit), ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                          _DP], i32),
        "pt_continuity": ([ctypes.POINTER(pt_fit), ctypes.POINTER(pt_fit), _DP, _DP], i32),
        "pt_seed_max_snippet": ([_CTX], i32),
        "pt_seed_block": ([_CTX, ctypes.POINTER(pt_block), ctypes.POINTER(pt_seed_opts), _VP,
                           ctypes.POINTER(pt_seed)], i32),
        "pt_seed_box": ([ctypes.POINTER(pt_seed), i32, ctypes.c_double, ctypes.c_double, i32,
                         ctypes.POINTER(pt_box)], i32),
        "pt_time_objective": ([_CTX, ctypes.POINTER(pt_block), _VP, i32, i32, i32, _VP, _DP], i32),
        "pt_server_create": ([_CTX, ctypes.POINTER(pt_server_config), ctypes.POINTER(_CTX)], i32),
        "pt_server_destroy": ([_CTX], None),
        "pt_server_submit": ([_CTX, i32, ctypes.POINTER(pt_block), ctypes.POINTER(ctypes.c_uint64)], i32),
        "pt_server_step": ([_CTX, _VP, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "pt_server_poll": ([_CTX, ctypes.POINTER(pt_server_result), i32, ctypes.POINTER(i32)], i32),
        "pt_server_stats": ([_CTX, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_uint64)],
                            i32),
        "pt_server_clock": ([_CTX], ctypes.c_double),
        "pt_ctx_set_launch_mode": ([_CTX, i32], i32),
        "pt_ctx_set_fp64_method": ([_CTX, i32], i32),
        "pt_ctx_last_launch": ([_CTX, ctypes.POINTER(i32)], i32),
        "pt_ctx_last_arithmetic": ([_CTX, ctypes.POINTER(i32)], i32),
        "pt_ctx_last_geometry": ([_CTX, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "pt_ctx_set_step_fusion": ([_CTX, i32], i32),
        "pt_ctx_set_timing": ([_CTX, i32], i32),
        "pt_ctx_kernel_stats": ([_CTX, ctypes.POINTER(i64), _DP], i32),
        "pt_ctx_last_fit_launches": ([_CTX, ctypes.POINTER(i64)], i32),
        "pt_ctx_get_tile": ([_CTX, i64, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "pt_ctx_set_tile": ([_CTX, i32, i32], i32),
        "pt_ctx_autotune": ([_CTX, i64, i32, i32, _VP, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
    }
    for name, (args, res) in spec.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res


def lib():
    """The loaded library.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libphasetrack.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        _signatures(L)
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != PT_OK:
        raise PtError(rc, where, lib().pt_last_error().decode(errors="replace"))


# ----------------------------------------------------------------- C names
def pt_version() -> int:
    return lib().pt_version()


def pt_last_error() -> str:
    return lib().pt_last_error().decode(errors="replace")


def pt_ctx_create(device: int = 0):
    h = _CTX()
    _check(lib().pt_ctx_create(device, ctypes.byref(h)), "pt_ctx_create")
    return h


def pt_ctx_destroy(ctx) -> None:
    lib().pt_ctx_destroy(ctx)


def pt_fit_block(ctx, block: pt_block, de: pt_de_settings, stream=None) -> pt_fit:
    out = pt_fit()
    _check(lib().pt_fit_block(ctx, ctypes.byref(block), ctypes.byref(de), stream, ctypes.byref(out)),
           "pt_fit_block")
    return out


def pt_fit_batch(ctx, blocks: Sequence[pt_block], de: pt_de_settings, stream=None):
    arr = (pt_block * len(blocks))(*blocks)
    out = (pt_fit * len(blocks))()
    _check(lib().pt_fit_batch(ctx, arr, len(blocks), ctypes.byref(de), stream, out), "pt_fit_batch")
    return list(out)


def pt_objective(ctx, block: pt_block, pop_ptr: int, P: int, precision: int, out_ptr: int, stream=None,
                 objective: int = PT_OBJ_CHI2):
    _check(lib().pt_objective(ctx, ctypes.byref(block), pop_ptr, P, precision, objective, stream, out_ptr),
           "pt_objective")


def pt_objective_noalloc(ctx, block: pt_block, pop_ptr: int, P: int, precision: int, out_ptr: int, stream=None,
                         objective: int = PT_OBJ_CHI2):
    _check(lib().pt_objective_noalloc(ctx, ctypes.byref(block), pop_ptr, P, precision, objective, stream,
                                      out_ptr), "pt_objective_noalloc")


def pt_last_population(ctx, index: int, P: int):
    import numpy as np

    pop = np.empty((P, NSLOT))
    f = np.empty(P)
    _check(lib().pt_last_population(ctx, index, pop.ctypes.data_as(_DP), f.ctypes.data_as(_DP), P),
           "pt_last_population")
    return pop, f


def pt_last_history(ctx, index: int, n: int):
    import numpy as np

    h = np.empty(max(n, 1))
    cnt = ctypes.c_int()
    _check(lib().pt_last_history(ctx, index, h.ctypes.data_as(_DP), n, ctypes.byref(cnt)), "pt_last_history")
    return h[: cnt.value]


def pt_phase(fit: pt_fit, t):
    import numpy as np

    t = np.ascontiguousarray(t, dtype=np.float64)
    outs = [np.empty_like(t) for _ in range(4)]
    _check(lib().pt_phase(ctypes.byref(fit), t.ctypes.data_as(_DP), t.size,
                          *[o.ctypes.data_as(_DP) for o in outs]), "pt_phase")
    return tuple(outs)


def pt_total_phase(fit: pt_fit, t_start: float, t_end: float):
    d, f = ctypes.c_double(), ctypes.c_double()
    _check(lib().pt_total_phase(ctypes.byref(fit), t_start, t_end, ctypes.byref(d), ctypes.byref(f)),
           "pt_total_phase")
    return d.value, f.value


def pt_connect_phase(fits: Sequence[pt_fit]):
    arr = (pt_fit * len(fits))(*fits)
    d, f = ctypes.c_double(), ctypes.c_double()
    _check(lib().pt_connect_phase(arr, len(fits), ctypes.byref(d), ctypes.byref(f)), "pt_connect_phase")
    return d.value, f.value


def pt_los_accel(fit: pt_fit, t: float, f_carrier_hz: float, M2: float = 1.0, three_way: bool = False):
    a = ctypes.c_double()
    _check(lib().pt_los_accel(ctypes.byref(fit), t, f_carrier_hz, M2, int(three_way), ctypes.byref(a)),
           "pt_los_accel")
    return a.value


def pt_time_objective(ctx, block: pt_block, pop_ptr: int, P: int, precision: int, reps: int, stream=None):
    ms = ctypes.c_double()
    _check(lib().pt_time_objective(ctx, ctypes.byref(block), pop_ptr, P, precision, reps, stream,
                                   ctypes.byref(ms)), "pt_time_objective")
    return ms.value


def pt_server_create(ctx, cfg: pt_server_config):
    h = _CTX()
    _check(lib().pt_server_create(ctx, ctypes.byref(cfg), ctypes.byref(h)), "pt_server_create")
    return h


def pt_server_destroy(srv) -> None:
    lib().pt_server_destroy(srv)


def pt_server_submit(srv, track: int, block: pt_block):
    """Returns the ticket, or None when the queue is full (PT_EBUSY)."""
    t = ctypes.c_uint64()
    rc = lib().pt_server_submit(srv, track, ctypes.byref(block), ctypes.byref(t))
    if rc == PT_EBUSY:
        return None
    _check(rc, "pt_server_submit")
    return t.value


def pt_server_step(srv, stream=None):
    a, p = ctypes.c_int(), ctypes.c_int()
    _check(lib().pt_server_step(srv, stream, ctypes.byref(a), ctypes.byref(p)), "pt_server_step")
    return a.value, p.value


def pt_server_poll(srv, max_results: int = 256):
    out = (pt_server_result * max_results)()
    n = ctypes.c_int()
    _check(lib().pt_server_poll(srv, out, max_results, ctypes.byref(n)), "pt_server_poll")
    return [out[k] for k in range(n.value)]


def pt_server_stats(srv):
    a, p, u = ctypes.c_int(), ctypes.c_int(), ctypes.c_uint64()
    _check(lib().pt_server_stats(srv, ctypes.byref(a), ctypes.byref(p), ctypes.byref(u)), "pt_server_stats")
    return a.value, p.value, u.value


def pt_server_clock(srv) -> float:
    return lib().pt_server_clock(srv)


def make_server_config(de: pt_de_settings, max_slots: int = 64, gens_per_step: int = 32,
                       max_pending: int = 4096, spl: int = 16, cpg: int = 4, warm_narrow: float = 0.7,
                       hbm_budget_bytes: int = 64 << 30, range_rule: int = PT_RUN_WARM, seed_first: bool = False,
                       seed_snippet: int = 0, seed_nsig: float = 10.0, max_attempts: int = 1,
                       enlarge: float = 2.0, qc_phase_rad: float = 0.0, qc_freq_hz: float = 0.0) -> pt_server_config:
    c = pt_server_config()
    c.max_slots, c.gens_per_step, c.max_pending = max_slots, gens_per_step, max_pending
    c.spl, c.cpg, c.warm_narrow, c.hbm_budget_bytes = spl, cpg, warm_narrow, hbm_budget_bytes
    c.de = de
    c.range_rule, c.seed_first, c.seed_snippet, c.seed_nsig = range_rule, int(seed_first), seed_snippet, seed_nsig
    c.max_attempts, c.enlarge, c.qc_phase_rad, c.qc_freq_hz = max_attempts, enlarge, qc_phase_rad, qc_freq_hz
    return c


def pt_continuity(a: pt_fit, b: pt_fit):
    """(border phase jump [rad, wrapped], border frequency jump [Hz]) of adjacent blocks a, b."""
    dp, df = ctypes.c_double(), ctypes.c_double()
    _check(lib().pt_continuity(ctypes.byref(a), ctypes.byref(b), ctypes.byref(dp), ctypes.byref(df)),
           "pt_continuity")
    return dp.value, df.value


def pt_seed_max_snippet(ctx) -> int:
    return lib().pt_seed_max_snippet(ctx)


def pt_seed_block(ctx, block: pt_block, snippet: int = 0, spacing: int = 0, stream=None) -> pt_seed:
    o = pt_seed_opts()
    o.snippet, o.spacing = snippet, spacing
    out = pt_seed()
    _check(lib().pt_seed_block(ctx, ctypes.byref(block), ctypes.byref(o), stream, ctypes.byref(out)),
           "pt_seed_block")
    return out


def pt_seed_box(seed: pt_seed, rule: int, nsig: float, T: float, slope: bool = False) -> pt_box:
    b = pt_box()
    _check(lib().pt_seed_box(ctypes.byref(seed), rule, nsig, T, int(slope), ctypes.byref(b)), "pt_seed_box")
    return b


def pt_ctx_set_launch_mode(ctx, mode: int):
    _check(lib().pt_ctx_set_launch_mode(ctx, mode), "pt_ctx_set_launch_mode")


def pt_ctx_set_fp64_method(ctx, method: int):
    _check(lib().pt_ctx_set_fp64_method(ctx, method), "pt_ctx_set_fp64_method")


def pt_ctx_fit_launches(ctx) -> int:
    n = ctypes.c_int64()
    _check(lib().pt_ctx_last_fit_launches(ctx, ctypes.byref(n)), "pt_ctx_last_fit_launches")
    return n.value


def pt_ctx_last_launch(ctx) -> int:
    m = ctypes.c_int()
    _check(lib().pt_ctx_last_launch(ctx, ctypes.byref(m)), "pt_ctx_last_launch")
    return m.value


def pt_ctx_set_step_fusion(ctx, mode: int):
    """PT_FUSION_AUTO (default), PT_FUSION_LEAD, PT_FUSION_LAST or PT_FUSION_OFF."""
    _check(lib().pt_ctx_set_step_fusion(ctx, int(mode)), "pt_ctx_set_step_fusion")


def pt_ctx_last_arithmetic(ctx) -> int:
    m = ctypes.c_int32()
    _check(lib().pt_ctx_last_arithmetic(ctx, ctypes.byref(m)), "pt_ctx_last_arithmetic")
    return m.value


def pt_ctx_last_geometry(ctx):
    """(samples per lane, candidates per workgroup) of the most recent fit or
    objective evaluation."""
    spl, cpg = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().pt_ctx_last_geometry(ctx, ctypes.byref(spl), ctypes.byref(cpg)), "pt_ctx_last_geometry")
    return spl.value, cpg.value


def pt_ctx_set_timing(ctx, on: bool):
    _check(lib().pt_ctx_set_timing(ctx, int(on)), "pt_ctx_set_timing")


def pt_ctx_kernel_stats(ctx):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(lib().pt_ctx_kernel_stats(ctx, ctypes.byref(n), ctypes.byref(ms)), "pt_ctx_kernel_stats")
    return n.value, ms.value


def pt_ctx_get_tile(ctx, n: int, P: int, precision: int):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().pt_ctx_get_tile(ctx, n, P, precision, ctypes.byref(a), ctypes.byref(b)), "pt_ctx_get_tile")
    return a.value, b.value


def pt_ctx_set_tile(ctx, spl: int, cpg: int):
    _check(lib().pt_ctx_set_tile(ctx, spl, cpg), "pt_ctx_set_tile")


def pt_ctx_autotune(ctx, n: int, P: int, precision: int, stream=None):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(lib().pt_ctx_autotune(ctx, n, P, precision, stream, ctypes.byref(a), ctypes.byref(b)),
           "pt_ctx_autotune")
    return a.value, b.value


# ------------------------------------------------------------ conveniences
def make_box(lo, hi) -> pt_box:
    """Box from lo / hi sequences of up to NSLOT slots (missing slots fixed at 0)."""
    b = pt_box()
    for j in range(NSLOT):
        b.lo[j] = float(lo[j]) if j < len(lo) else 0.0
        b.hi[j] = float(hi[j]) if j < len(hi) else 0.0
    return b


def make_settings(pop: int, max_gens: int, F: float = 0.5, CR: float = 0.9, seed: int = 0,
                  vtr: float = -math.inf, rel_tol: float = 0.0, window: int = 0,
                  precision: int = PT_PREC_FP64, objective: int = PT_OBJ_CHI2) -> pt_de_settings:
    s = pt_de_settings()
    s.pop, s.max_gens, s.F, s.CR, s.seed = pop, max_gens, F, CR, seed
    s.vtr, s.rel_tol, s.window, s.precision = vtr, rel_tol, window, precision
    s.objective = objective
    return s


def make_block(samples, fs: float, lo, hi, ref: Optional[float] = None, stream: int = 0) -> pt_block:
    """pt_block over a torch tensor on the GPU (FP32 or FP64, contiguous)."""
    import torch

    if not isinstance(samples, torch.Tensor):
        raise TypeError("samples must be a torch tensor")
    if not samples.is_contiguous():
        raise ValueError("samples must be contiguous")
    if samples.dtype == torch.float32:
        dt = PT_F32
    elif samples.dtype == torch.float64:
        dt = PT_F64
    else:
        raise TypeError("samples must be float32 or float64")
    b = pt_block()
    b.samples = samples.data_ptr()
    b.n = samples.numel()
    b.dtype = dt
    b.on_device = 1 if samples.is_cuda else 0
    b.fs = float(fs)
    b.ref = float("nan") if ref is None else float(ref)
    b.stream = int(stream)
    b.box = make_box(lo, hi)
    b._samples = samples  # the block only holds a raw pointer: keep the tensor alive with it
    return b


def current_stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Owning wrapper of a pt_ctx handle."""

    def __init__(self, device: int = 0):
        # torch and this library share the process's HIP runtime; torch must
        # bring up its device state first (when the library initialises the
        # runtime first, torch afterwards reports no devices)
        try:
            import torch

            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        self.handle = pt_ctx_create(device)
        self.device = device

    def close(self):
        if self.handle is not None:
            pt_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fit_block(self, block: pt_block, de: pt_de_settings) -> pt_fit:
        return pt_fit_block(self.handle, block, de, current_stream())

    def fit_batch(self, blocks, de: pt_de_settings):
        return pt_fit_batch(self.handle, blocks, de, current_stream())

    def objective(self, block: pt_block, pop, precision: int = PT_PREC_FP64, objective: int = PT_OBJ_CHI2):
        """Objective (chi^2 or correlation) of each row of ``pop`` (torch FP64 tensor P x 6 on the GPU)."""
        import torch

        if pop.dim() == 2 and pop.shape[1] < NSLOT:  # missing slots are 0
            pop = torch.nn.functional.pad(pop, (0, NSLOT - pop.shape[1]))
        pop = pop.contiguous()
        if pop.dtype != torch.float64 or pop.dim() != 2 or pop.shape[1] != NSLOT or not pop.is_cuda:
            raise ValueError(f"pop must be a CUDA float64 tensor of shape (P, <= {NSLOT})")
        out = torch.empty(pop.shape[0], dtype=torch.float64, device=pop.device)
        pt_objective(self.handle, block, pop.data_ptr(), pop.shape[0], precision, out.data_ptr(),
                     current_stream(), objective)
        return out
