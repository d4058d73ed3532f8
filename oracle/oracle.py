"""Python access to the plain FP64 CPU oracle (``pp_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the checker for the HIP path, not
part of it: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this module.  It imports nothing from the
``paper_2502_10640_amd`` package and the package imports nothing from here.

Functions follow arXiv 2502.10640 Sec. 2.1 (Eqs. (A)-(H)) and Sec. 2.2/3.2
(Eq. (I) and the beam observables); the C file states each one's definition.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pp_oracle.c")
LIB_PATH = os.path.join(_HERE, "libpporacle.so")

CFLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-shared", "-fPIC"]


def build(src: str = _SRC, out: str = LIB_PATH) -> str:
    """Compile the oracle into a shared library with gcc; returns its path."""
    cmd = ["gcc", *CFLAGS, "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


class DiagRecord(ctypes.Structure):
    """Mirror of ``oracle_diag_t``."""
    _fields_ = [
        ("kinetic", ctypes.c_double),
        ("potential", ctypes.c_double),
        ("total", ctypes.c_double),
        ("momentum", ctypes.c_double * 3),
        ("com", ctypes.c_double * 3),
        ("com_velocity", ctypes.c_double * 3),
        ("emittance", ctypes.c_double * 3),
        ("emittance_centered", ctypes.c_double * 3),
        ("x_rms", ctypes.c_double * 3),
        ("x_max", ctypes.c_double * 3),
        ("v_rms", ctypes.c_double * 3),
        ("v_max", ctypes.c_double * 3),
        ("nonfinite", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, typ in self._fields_:
            val = getattr(self, name)
            out[name] = list(val) if hasattr(typ, "_length_") else val
        return out


_P = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int64)


class Oracle:
    """ctypes handle on one build of the oracle library."""

    def __init__(self, lib_path: str = LIB_PATH):
        if not os.path.exists(lib_path):
            if lib_path != LIB_PATH:
                raise FileNotFoundError(lib_path)
            build()
        self.lib = ctypes.CDLL(lib_path)
        L = self.lib
        L.oracle_field.argtypes = [ctypes.c_int64, _P, _P, _P, _P, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_int64, _PI, _P, _P, _P, _P, _P, _P]
        L.oracle_field.restype = None
        L.oracle_vv.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int64, _P, _P, _P, ctypes.c_int]
        L.oracle_vv.restype = None
        L.oracle_diag.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P,
                                  ctypes.c_double, ctypes.c_double, ctypes.POINTER(DiagRecord)]
        L.oracle_diag.restype = None
        L.oracle_coulomb_k.argtypes = []
        L.oracle_coulomb_k.restype = ctypes.c_double
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None

    @staticmethod
    def _d(a: np.ndarray):
        return a.ctypes.data_as(_P)

    @staticmethod
    def _arr(a, n=None) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.float64)
        if n is not None and a.shape != (n,):
            raise ValueError(f"expected shape ({n},), got {a.shape}")
        return a

    @property
    def k(self) -> float:
        return self.lib.oracle_coulomb_k()

    def num_threads(self) -> int:
        return self.lib.oracle_num_threads()

    def set_num_threads(self, n: int) -> None:
        """Thread count of later calls (n >= 1); results do not depend on it."""
        if n < 1:
            raise ValueError("thread count must be >= 1")
        self.lib.oracle_set_num_threads(int(n))

    def field(self, x, y, z, q, w: float, eps: float, recv=None, want_phi=False,
              want_amag=False, want_pmag=False):
        """E (and optionally phi, A, P) at receivers ``recv`` (all if None).
        A and P are the sums of the magnitudes of the terms of E and of phi."""
        x = self._arr(x)
        n = x.shape[0]
        y, z, q = self._arr(y, n), self._arr(z, n), self._arr(q, n)
        if recv is None:
            nr, rp = n, None
        else:
            recv = np.ascontiguousarray(recv, dtype=np.int64)
            if recv.size and (recv.min() < 0 or recv.max() >= n):
                raise IndexError("receiver index out of range")
            nr, rp = recv.shape[0], recv.ctypes.data_as(_PI)
        ex, ey, ez = (np.empty(nr) for _ in range(3))
        phi = np.empty(nr) if want_phi else None
        amag = np.empty(nr) if want_amag else None
        pmag = np.empty(nr) if want_pmag else None
        self.lib.oracle_field(n, self._d(x), self._d(y), self._d(z), self._d(q), w, eps, nr, rp,
                              self._d(ex), self._d(ey), self._d(ez),
                              self._d(phi) if phi is not None else None,
                              self._d(amag) if amag is not None else None,
                              self._d(pmag) if pmag is not None else None)
        out = {"ex": ex, "ey": ey, "ez": ez}
        if want_phi:
            out["phi"] = phi
        if want_amag:
            out["amag"] = amag
        if want_pmag:
            out["pmag"] = pmag
        return out

    def vv(self, state: "OracleState", n_steps: int) -> None:
        """Advance ``state`` in place by ``n_steps`` Velocity Verlet steps."""
        s = state
        self.lib.oracle_vv(s.n, *(self._d(a) for a in (s.x, s.y, s.z, s.vx, s.vy, s.vz, s.q, s.m)),
                           s.w, s.eps, s.dt, int(n_steps),
                           self._d(s.ax), self._d(s.ay), self._d(s.az), int(s.a_valid))
        s.a_valid = True
        s.step += int(n_steps)

    def diag(self, x, y, z, vx, vy, vz, q, m, w: float, eps: float) -> dict:
        x = self._arr(x)
        n = x.shape[0]
        arrs = [x] + [self._arr(a, n) for a in (y, z, vx, vy, vz, q, m)]
        rec = DiagRecord()
        self.lib.oracle_diag(n, *(self._d(a) for a in arrs), w, eps, ctypes.byref(rec))
        return rec.as_dict()

    def diag_state(self, s: "OracleState") -> dict:
        return self.diag(s.x, s.y, s.z, s.vx, s.vy, s.vz, s.q, s.m, s.w, s.eps)


@dataclass
class OracleState:
    """FP64 state of one bunch as the oracle integrates it (copies its inputs)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    q: np.ndarray
    m: np.ndarray
    w: float
    eps: float
    dt: float
    ax: np.ndarray = None
    ay: np.ndarray = None
    az: np.ndarray = None
    a_valid: bool = False
    step: int = 0

    def __post_init__(self):
        for f in ("x", "y", "z", "vx", "vy", "vz", "q", "m"):
            setattr(self, f, np.array(getattr(self, f), dtype=np.float64, copy=True))
        n = self.x.shape[0]
        for f in ("ax", "ay", "az"):
            if getattr(self, f) is None:
                setattr(self, f, np.zeros(n))

    @property
    def n(self) -> int:
        return self.x.shape[0]

    def copy(self) -> "OracleState":
        c = OracleState(self.x, self.y, self.z, self.vx, self.vy, self.vz, self.q, self.m,
                        self.w, self.eps, self.dt, self.ax.copy(), self.ay.copy(), self.az.copy(),
                        self.a_valid, self.step)
        return c


_DEFAULT = None


def default() -> Oracle:
    """Process-wide oracle instance (builds the library on first use)."""
    global _DEFAULT
    if _DEFAULT is None:
        _DEFAULT = Oracle()
    return _DEFAULT
