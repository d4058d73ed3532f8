"""Failure handling of the C ABI on the GPU, forced from the host: the
PP_FAULT_INJECT hook makes the N-th device allocation or kernel launch of a
context fail before it reaches the device (nothing faults, every launched
kernel completes).  For every N the failing call returns
PP_ERR_OUT_OF_MEMORY or PP_ERR_DEVICE, every later call PP_ERR_STATE,
pp_destroy succeeds and the process holds no device memory of the library
afterwards (pp_device_bytes, and hipMemGetInfo within a small slack).

Also: the device-memory accounting of live contexts, and pp_invalidate
re-centring the mixed path's frame on a bunch that has moved far away.
"""
import numpy as np
import pytest

from oracle.oracle import default
from paper_2502_10640_amd import pp
from paper_2502_10640_amd import workloads as wl
from tests.test_gpu_parity import Sim, check_field, oracle_field, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    pp.load()
    return torch


def _calls(sim, prec):
    """A typical run: field, pushes, graph replays, diagnostics (lazy
    allocations), a change to the symmetric schedule (new work list, slots,
    sort buffers), an invalidation, a checked step, a sync."""
    sym = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3 if prec == "mixed" else 0, "graph_steps": 2}
    return [("field", lambda: sim.field(want_phi=True)),
            ("push", lambda: sim.push(2)),
            ("step_graph", lambda: sim.step_batched(4, graph=True)),
            ("diagnostics", lambda: sim.diagnostics()),
            ("set_tuning", lambda: sim.set_tuning(**sym)),
            ("field_sym", lambda: sim.field(want_phi=True)),
            ("step_sym_graph", lambda: sim.step_batched(4, graph=True)),
            ("invalidate", lambda: sim.invalidate()),
            ("step_checked", lambda: sim.step_batched(1, graph=False, check=True)),
            ("sync", lambda: sim.sync())]


def _run(b, prec):
    """Statuses of create and of each call of the run, in order."""
    out = []
    try:
        sim = Sim([b], prec, tuning={"graph_steps": 2})
    except pp.PPError as e:
        return [("create", e.status)]
    out.append(("create", pp.PP_OK))
    try:
        for name, op in _calls(sim, prec):
            try:
                op()
                out.append((name, pp.PP_OK))
            except pp.PPError as e:
                out.append((name, e.status))
    finally:
        sim.close()
    return out


@pytest.mark.parametrize("kind", ["alloc", "launch"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_injected_fault_breaks_the_context_cleanly(gpu, monkeypatch, prec, kind):
    torch = gpu
    b = wl.workload("gaussian_65536", n_override=700)[0]
    expect = pp.PP_ERR_OUT_OF_MEMORY if kind == "alloc" else pp.PP_ERR_DEVICE
    say(f"injected {kind} failures, {prec}, every position of a typical run")
    monkeypatch.delenv("PP_FAULT_INJECT", raising=False)
    # one clean run first: the runtime's own first-use set-up (code objects,
    # queues) is not the library's memory
    assert all(c == pp.PP_OK for _, c in _run(b, prec))
    torch.cuda.synchronize()
    base_bytes = pp.pp_device_bytes(None)
    free0, _ = torch.cuda.mem_get_info()
    where = {}
    n = 0
    while True:
        n += 1
        assert n < 2000, "the run never completes"
        monkeypatch.setenv("PP_FAULT_INJECT", f"{kind}:{n}")
        res = _run(b, prec)
        codes = [c for _, c in res]
        failed = [i for i, c in enumerate(codes) if c != pp.PP_OK]
        if not failed:
            break  # N is past the run's last allocation or launch
        first = failed[0]
        assert codes[first] == expect, (n, res)
        # every call after the failing one reports the broken context
        assert all(c == pp.PP_ERR_STATE for c in codes[first + 1:]), (n, res)
        where[res[first][0]] = where.get(res[first][0], 0) + 1
        assert pp.pp_device_bytes(None) == base_bytes, (n, res)
    monkeypatch.delenv("PP_FAULT_INJECT")
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    print(f"    {n - 1} failure positions, by call: {where}; free memory change {free1 - free0} B", flush=True)
    # the run allocates in create, diagnostics and the tuning change, and launches in every call
    # that computes (the tuning change only builds lists and allocates)
    if kind == "alloc":
        assert {"create", "diagnostics", "set_tuning"} <= set(where)
    else:
        assert {"create", "field", "push", "step_graph", "diagnostics", "field_sym", "step_sym_graph",
                "step_checked"} <= set(where)
    assert pp.pp_device_bytes(None) == base_bytes
    assert free1 >= free0 - (64 << 20)


def test_device_bytes_accounting(gpu):
    torch = gpu
    b = wl.workload("cold_sphere_2048", n_override=3000)[0]
    say("pp_device_bytes of live contexts")
    before = pp.pp_device_bytes(None)
    with Sim([b], "mixed") as s1, Sim([b], "fp64") as s2:
        n1, n2 = pp.pp_device_bytes(s1.ctx), pp.pp_device_bytes(s2.ctx)
        assert n1 > 0 and n2 > 0
        assert pp.pp_device_bytes(None) == before + n1 + n2
        s1.diagnostics()  # lazy diagnostics buffers
        assert pp.pp_device_bytes(s1.ctx) > n1
        s1.set_tuning(symmetric=1, fused=0, i_per_lane=1, far_split=3)  # slots and sort buffers
        assert pp.pp_device_bytes(s1.ctx) > n1
        # the context's own scratch: at least the acceleration (24 B) and mirror (28 B) per particle
        assert n1 >= 52 * b.n
    assert pp.pp_device_bytes(None) == before


def test_invalidate_recentres_the_mixed_frame(gpu):
    """A bunch moved 10^4 of its radii away after create: the field stays
    within tolerance with the stale frame, and after pp_invalidate (which
    re-centres the mixed path's frame) it is as accurate as at the origin (the
    pair-stage times of the three cases are printed: the near/far split finds
    fewer far groups in the stale frame).  A non-finite position makes
    pp_invalidate report PP_ERR_NOT_FINITE and leaves the context usable."""
    torch = gpu
    orc = default()
    b = wl.workload("gaussian_65536", n_override=6000)[0]
    shift = 1e4 * float(np.abs(b.x).max())
    moved = b.copy()
    moved.x = b.x + shift
    say(f"invalidate re-centres the frame after a shift of {shift:.3e} m")
    ref = oracle_field(orc, moved)
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3}
    with Sim([b], "mixed", tuning=tun) as sim:
        at_origin = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        ms_origin, _ = pp.pp_time_field(sim.ctx, 3)
        with sim._on():
            sim.t["x"] += shift
        stale = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        ms_stale, _ = pp.pp_time_field(sim.ctx, 3)
        sim.invalidate()
        fresh = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        ms_fresh, _ = pp.pp_time_field(sim.ctx, 3)
        with sim._on():
            sim.t["y"][17] = float("nan")
        with pytest.raises(pp.PPError) as e:
            sim.invalidate()
        assert e.value.status == pp.PP_ERR_NOT_FINITE
        with sim._on():
            sim.t["y"][17] = b.y[17]
        sim.invalidate()
        sim.sync()
    e_stale = check_field(stale, ref, 1e-5, "stale frame")
    e_fresh = check_field(fresh, ref, 1e-5, "re-centred frame")
    print(f"    pair stage: at the origin {ms_origin:.3f} ms, moved {ms_stale:.3f} ms, re-centred {ms_fresh:.3f} ms",
          flush=True)
    # re-centred, the mixed path is as accurate as for a bunch at its frame's origin (about 1e-7)
    assert e_fresh[0] <= 3e-7
    assert np.all(np.isfinite(at_origin["ex"]))
