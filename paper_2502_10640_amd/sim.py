"""Device-resident simulation of one or more bunches through the C ABI.

PyTorch provides the device memory (FP64 SoA tensors) and the stream; every
step of the method runs in the HIP library via ``pp``.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from . import pp
from .workloads import Bunch, concat

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "q", "m")


class Simulation:
    """Owns device copies of the bunches' state and a library context."""

    def __init__(self, bunches: Sequence[Bunch], precision: str = "mixed", device: str = "cuda:0",
                 tuning: dict | None = None, gap: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the PP library runs on the GPU only")
        self.torch = torch
        self.device = torch.device(device)
        self.bunches = list(bunches)
        self.precision = precision
        arrays, offsets = concat(self.bunches)
        if gap:
            # leave `gap` unused slots after every bunch (exercises offset tables with holes)
            arrays, offsets = _with_gaps(arrays, offsets, gap)
        self.offsets = offsets
        self.n_total = int(arrays[0].shape[0])
        prec = pp.PP_MIXED if precision == "mixed" else pp.PP_FP64
        desc = [(off, n, b.weight, b.softening, b.dt) for (off, n), b in zip(offsets, self.bunches)]
        # the context lives on this device and enqueues on this stream; every call
        # below runs with both current, so torch's own work (copies, zero fills)
        # is ordered with the library's
        self.stream = torch.cuda.current_stream(self.device)
        with self._on():
            self.t = {name: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
                      for name, a in zip(FIELDS, arrays)}
            self.ctx = pp.pp_create(desc, self.n_total, [self.t[k].data_ptr() for k in FIELDS], prec,
                                    self.stream.cuda_stream)
            if tuning:
                pp.pp_set_tuning(self.ctx, **tuning)

    def _on(self):
        """Make this simulation's device and stream current (a context manager)."""
        import contextlib
        stack = contextlib.ExitStack()
        stack.enter_context(self.torch.cuda.device(self.device))
        stack.enter_context(self.torch.cuda.stream(self.stream))
        return stack

    # -- the C entry points ------------------------------------------------
    def field(self, want_phi: bool = False):
        torch = self.torch
        with self._on():
            out = {k: torch.zeros(self.n_total, dtype=torch.float64, device=self.device) for k in ("ex", "ey", "ez")}
            if want_phi:
                out["phi"] = torch.zeros(self.n_total, dtype=torch.float64, device=self.device)
            pp.pp_field(self.ctx, out["ex"].data_ptr(), out["ey"].data_ptr(), out["ez"].data_ptr(),
                        out["phi"].data_ptr() if want_phi else None)
        return out

    def push(self, n_steps: int) -> None:
        with self._on():
            pp.pp_push(self.ctx, n_steps)

    def step_batched(self, n_steps: int, graph: bool = True, autotune: bool = False, check: bool = False) -> None:
        flags = (pp.PP_GRAPH if graph else 0) | (pp.PP_AUTOTUNE if autotune else 0) | (pp.PP_CHECK if check else 0)
        with self._on():
            pp.pp_step_batched(self.ctx, n_steps, flags)

    def diagnostics(self) -> List[dict]:
        with self._on():
            return pp.pp_diagnostics(self.ctx, len(self.bunches))

    def invalidate(self) -> None:
        pp.pp_invalidate(self.ctx)

    def tuning(self) -> dict:
        return pp.pp_get_tuning(self.ctx)

    def set_tuning(self, **kw) -> None:
        with self._on():
            pp.pp_set_tuning(self.ctx, **kw)

    def sync(self) -> None:
        with self._on():
            pp.pp_sync(self.ctx)

    # -- host views ---------------------------------------------------------
    def host(self, name: str) -> np.ndarray:
        self.sync()
        with self._on():
            return self.t[name].cpu().numpy()

    def bunch_slice(self, b: int) -> slice:
        off, n = self.offsets[b]
        return slice(off, off + n)

    def close(self) -> None:
        if getattr(self, "ctx", None):
            with self._on():
                pp.pp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False


def _with_gaps(arrays, offsets, gap):
    out = [[] for _ in arrays]
    new_off, pos = [], 0
    for (off, n) in offsets:
        for k, a in enumerate(arrays):
            out[k].append(a[off:off + n])
            fill = 1.0 if k == 7 else 0.0   # gap particles get m = 1 so nothing is singular
            out[k].append(np.full(gap, fill))
        new_off.append((pos, n))
        pos += n + gap
    return [np.concatenate(o) for o in out], new_off
