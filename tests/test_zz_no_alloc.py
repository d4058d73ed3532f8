"""The allocation-free entry point pp_field_noalloc (GPU, through the C ABI).

Two calls in a row on one device, the second with a smaller bunch, in both
precisions: each result equals pp_field's on a context of the same bunch with
the ordered-pair tiling the allocation-free path uses, bit for bit, and both
are within the field tolerance of the CPU FP64 oracle (1e-12 FP64, 1e-5
mixed; relative L2 and the condition-aware max, potential per particle).
The calls allocate no device memory (no context is created; pp_device_bytes
stays unchanged).  A hipGraph captured around the call replays to the eager
result, with other calls on the same scratch between the replays.
"""
import numpy as np
import pytest

from oracle.oracle import default
from paper_2502_10640_amd import pp
from paper_2502_10640_amd import workloads as wl
from tests.test_gpu_parity import Sim, check_field, mixed_charge_bunch, oracle_field, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
PREC = {"fp64": pp.PP_FP64, "mixed": pp.PP_MIXED}
ORDERED = {"symmetric": 0, "fused": 0, "i_per_lane": 1, "sum_tile": 64, "chunk_pairs_log2": 22, "grid_per_cu": 4,
           "far_split": 0, "sym_split": 1}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    pp.load()
    return torch


def _inputs(torch, b):
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(b, k))).to(dev) for k in ("x", "y", "z", "q")}
    out = {k: torch.full((b.n,), float("nan"), dtype=torch.float64, device=dev) for k in ("ex", "ey", "ez", "phi")}
    return t, out


def _call(b, prec, t, out, stream=None):
    pp.pp_field_noalloc(b.n, t["x"].data_ptr(), t["y"].data_ptr(), t["z"].data_ptr(), t["q"].data_ptr(),
                        b.weight, b.softening, PREC[prec], out["ex"].data_ptr(), out["ey"].data_ptr(),
                        out["ez"].data_ptr(), out["phi"].data_ptr(), stream)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_field_equals_pp_field_on_two_calls(gpu, prec):
    torch = gpu
    orc = default()
    first = wl.workload("gaussian_65536", n_override=5000)[0]
    second = mixed_charge_bunch(1200, seed=31)   # smaller, unlike charges, no softening
    for b in (first, second):
        say(f"pp_field_noalloc {prec} n={b.n}")
        before = pp.pp_device_bytes(None)
        t, out = _inputs(torch, b)
        stream = torch.cuda.current_stream().cuda_stream
        _call(b, prec, t, out, stream)
        torch.cuda.synchronize()
        assert pp.pp_device_bytes(None) == before
        got = {k: v.cpu().numpy() for k, v in out.items()}
        with Sim([b], prec, tuning=ORDERED) as sim:
            ref_ctx = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        for k in ("ex", "ey", "ez", "phi"):
            np.testing.assert_array_equal(got[k], ref_ctx[k], err_msg=f"{prec} n={b.n} {k}")
        check_field(got, oracle_field(orc, b), TOL[prec], f"noalloc {prec} n={b.n}")


def test_noalloc_rejects_sizes_beyond_its_scratch(gpu):
    torch = gpu
    dev = torch.device("cuda:0")
    z = torch.zeros(4, dtype=torch.float64, device=dev)
    p = z.data_ptr()
    say("pp_field_noalloc argument checks")
    for n in (0, pp.NOALLOC_MAX_N + 1):
        with pytest.raises(pp.PPError) as e:
            pp.pp_field_noalloc(n, p, p, p, p, 1.0, 0.0, pp.PP_MIXED, p, p, p)
        assert e.value.status == pp.PP_ERR_INVALID_ARG and "allocation-free" in e.value.message
    with pytest.raises(pp.PPError) as e:
        pp.pp_field_noalloc(4, p, p, p, p, -1.0, 0.0, pp.PP_FP64, p, p, p)
    assert e.value.status == pp.PP_ERR_INVALID_ARG


def test_noalloc_under_graph_capture(gpu):
    """Captured in a hipGraph (the caller that cannot allocate): every replay
    gives the eager result, with calls on other inputs between replays."""
    torch = gpu
    b = wl.workload("cold_sphere_2048")[0]
    other = wl.workload("gaussian_65536", n_override=3000)[0]
    say("pp_field_noalloc captured in a hipGraph, 3 replays")
    t, out = _inputs(torch, b)
    t2, out2 = _inputs(torch, other)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        _call(b, "mixed", t, out, s.cuda_stream)   # first call on the device outside the capture
    torch.cuda.synchronize()
    eager = {k: v.cpu().numpy() for k, v in out.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        _call(b, "mixed", t, out, torch.cuda.current_stream().cuda_stream)
    for rep in range(3):
        for v in out.values():
            v.fill_(float("nan"))
        _call(other, "mixed", t2, out2, torch.cuda.current_stream().cuda_stream)  # same scratch, other bunch
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in eager:
            np.testing.assert_array_equal(out[k].cpu().numpy(), eager[k], err_msg=f"replay {rep} {k}")
