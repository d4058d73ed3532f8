"""ctypes binding of the C ABI in ``include/pp.h`` (argument marshalling only).

Every function keeps the name of the C entry point it wraps and raises
``PPError`` on a non-zero status.  Device memory and streams come from the
caller (PyTorch tensors' ``data_ptr()`` and ``cuda_stream``); all computation
runs in the HIP library ``libpp_hip.so``.  There is no fallback: if the library
is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Sequence

from .build import LIB_PATH

PP_OK = 0
PP_ERR_INVALID_ARG = 1
PP_ERR_OUT_OF_MEMORY = 2
PP_ERR_DEVICE = 3
PP_ERR_NOT_FINITE = 4
PP_ERR_STATE = 5
STATUS_NAMES = {0: "PP_OK", 1: "PP_ERR_INVALID_ARG", 2: "PP_ERR_OUT_OF_MEMORY", 3: "PP_ERR_DEVICE",
                4: "PP_ERR_NOT_FINITE", 5: "PP_ERR_STATE"}

PP_FP64 = 0
PP_MIXED = 1

PP_GRAPH = 1
PP_AUTOTUNE = 2
PP_CHECK = 4

EXPORTS = ("pp_create", "pp_field", "pp_field_noalloc", "pp_push", "pp_step_batched", "pp_diagnostics", "pp_invalidate",
           "pp_get_tuning", "pp_set_tuning", "pp_time_field", "pp_set_profiling", "pp_get_profile",
           "pp_sync", "pp_device_bytes", "pp_destroy", "pp_last_error", "pp_abi_version")


class PPError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class Bunch(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n", ctypes.c_int64), ("weight", ctypes.c_double),
                ("softening", ctypes.c_double), ("dt", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "q", "m")]


class Diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("n", ctypes.c_int64), ("time", ctypes.c_double),
        ("kinetic", ctypes.c_double), ("potential", ctypes.c_double), ("total", ctypes.c_double),
        ("momentum", ctypes.c_double * 3), ("com", ctypes.c_double * 3), ("com_velocity", ctypes.c_double * 3),
        ("emittance", ctypes.c_double * 3), ("emittance_centered", ctypes.c_double * 3),
        ("x_rms", ctypes.c_double * 3), ("x_max", ctypes.c_double * 3), ("v_rms", ctypes.c_double * 3),
        ("v_max", ctypes.c_double * 3), ("nonfinite", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, typ in self._fields_:
            val = getattr(self, name)
            out[name] = list(val) if hasattr(typ, "_length_") else val
        return out


class Tuning(ctypes.Structure):
    _fields_ = [("i_per_lane", ctypes.c_int32), ("sum_tile", ctypes.c_int32), ("chunk_pairs_log2", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("symmetric", ctypes.c_int32),
                ("far_split", ctypes.c_int32), ("sym_split", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("sym_rounds", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("evaluations", ctypes.c_int64), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("pairs", ctypes.c_double)]


_LIB = None
_VP = ctypes.c_void_p
ABI_VERSION = 4  # PP_ABI_VERSION of include/pp.h


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (once).  Raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build(); "
                           "this package has no CPU fallback")
    L = ctypes.CDLL(path)
    st = ctypes.c_int
    sig = {
        "pp_create": ([ctypes.POINTER(_VP), ctypes.POINTER(Bunch), ctypes.c_int32, ctypes.c_int64,
                       ctypes.POINTER(State), ctypes.c_int, _VP], st),
        "pp_field": ([_VP, _VP, _VP, _VP, _VP], st),
        "pp_field_noalloc": ([ctypes.c_int64, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                              _VP, _VP, _VP, _VP, _VP], st),
        "pp_push": ([_VP, ctypes.c_int64], st),
        "pp_step_batched": ([_VP, ctypes.c_int64, ctypes.c_uint32], st),
        "pp_diagnostics": ([_VP, ctypes.POINTER(Diag)], st),
        "pp_invalidate": ([_VP], st),
        "pp_get_tuning": ([_VP, ctypes.POINTER(Tuning)], st),
        "pp_set_tuning": ([_VP, ctypes.POINTER(Tuning)], st),
        "pp_time_field": ([_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], st),
        "pp_set_profiling": ([_VP, ctypes.c_int32], st),
        "pp_get_profile": ([_VP, ctypes.POINTER(Profile)], st),
        "pp_sync": ([_VP], st),
        "pp_device_bytes": ([_VP], ctypes.c_int64),
        "pp_destroy": ([_VP], st),
        "pp_last_error": ([_VP], ctypes.c_char_p),
        "pp_abi_version": ([], ctypes.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.pp_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {L.pp_abi_version()}, this binding expects {ABI_VERSION}: "
                           "rebuild it with __graft_entry__.build()")
    _LIB = L
    return L


def _check(status: int, ctx) -> None:
    if status != PP_OK:
        raise PPError(status, pp_last_error(ctx))


def pp_abi_version() -> int:
    return load().pp_abi_version()


def pp_last_error(ctx=None) -> str:
    return load().pp_last_error(ctx).decode()


def pp_create(bunches: Sequence[Sequence[float]], n_total: int, state: Sequence[int], precision: int,
              stream: int | None = None):
    """bunches: (offset, n, weight, softening, dt) per bunch; state: 8 device
    pointers (x, y, z, vx, vy, vz, q, m); returns the context handle."""
    arr = (Bunch * len(bunches))(*[Bunch(int(o), int(n), float(w), float(e), float(d))
                                   for (o, n, w, e, d) in bunches])
    st = State(*[int(p) for p in state])
    ctx = _VP()
    status = load().pp_create(ctypes.byref(ctx), arr, len(bunches), int(n_total), ctypes.byref(st),
                              int(precision), _VP(stream or 0) if stream else None)
    if status != PP_OK:
        raise PPError(status, pp_last_error(None))
    return ctx


def pp_field(ctx, ex: int, ey: int, ez: int, phi: int | None = None) -> None:
    _check(load().pp_field(ctx, ex, ey, ez, phi or None), ctx)


NOALLOC_MAX_N = 65536  # PP_NOALLOC_MAX_N of include/pp.h


def pp_field_noalloc(n: int, x: int, y: int, z: int, q: int, weight: float, softening: float, precision: int,
                     ex: int, ey: int, ez: int, phi: int | None = None, stream: int | None = None) -> None:
    """Context-free, allocation-free field of one bunch (device pointers)."""
    _check(load().pp_field_noalloc(int(n), x, y, z, q, float(weight), float(softening), int(precision),
                                   ex, ey, ez, phi or None, _VP(stream) if stream else None), None)


def pp_push(ctx, n_steps: int) -> None:
    _check(load().pp_push(ctx, int(n_steps)), ctx)


def pp_step_batched(ctx, n_steps: int, flags: int = 0) -> None:
    _check(load().pp_step_batched(ctx, int(n_steps), int(flags)), ctx)


def pp_diagnostics(ctx, n_bunches: int) -> List[dict]:
    out = (Diag * n_bunches)()
    _check(load().pp_diagnostics(ctx, out), ctx)
    return [d.as_dict() for d in out]


def pp_invalidate(ctx) -> None:
    _check(load().pp_invalidate(ctx), ctx)


def pp_get_tuning(ctx) -> dict:
    t = Tuning()
    _check(load().pp_get_tuning(ctx, ctypes.byref(t)), ctx)
    return t.as_dict()


def pp_set_tuning(ctx, **kw) -> None:
    cur = pp_get_tuning(ctx)
    cur.update(kw)
    t = Tuning(**cur)
    _check(load().pp_set_tuning(ctx, ctypes.byref(t)), ctx)


def pp_time_field(ctx, n_reps: int = 3):
    ms, pairs = ctypes.c_double(), ctypes.c_double()
    _check(load().pp_time_field(ctx, int(n_reps), ctypes.byref(ms), ctypes.byref(pairs)), ctx)
    return ms.value, pairs.value


def pp_set_profiling(ctx, enable: bool) -> None:
    _check(load().pp_set_profiling(ctx, 1 if enable else 0), ctx)


def pp_get_profile(ctx) -> dict:
    p = Profile()
    _check(load().pp_get_profile(ctx, ctypes.byref(p)), ctx)
    return {"evaluations": p.evaluations, "launches": p.launches, "total_ms": p.total_ms, "pairs": p.pairs}


def pp_sync(ctx) -> None:
    _check(load().pp_sync(ctx), ctx)


def pp_device_bytes(ctx=None) -> int:
    """Device bytes held by ctx, or by every live context when ctx is None."""
    return int(load().pp_device_bytes(ctx))


def pp_destroy(ctx) -> None:
    if ctx:
        _check(load().pp_destroy(ctx), None)


def exported_symbols(path: str = LIB_PATH) -> Iterable[str]:
    lib = ctypes.CDLL(path)
    return [n for n in EXPORTS if hasattr(lib, n)]
