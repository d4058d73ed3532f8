"""The fused small-bunch schedule (tuning field `fused`: one workgroup
computes each receiver's whole field and applies the update; one kernel per
step) against the CPU FP64 oracle, and its bitwise equivalences.

Tolerances as in test_gpu_parity: fields 1e-12 (FP64) and 1e-5 (mixed) in
the relative L2 and condition-aware norms, the potential per particle;
trajectories relative to the rms of r and v.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleState, default
from paper_2502_10640_amd import pp
from paper_2502_10640_amd import workloads as wl
from tests.test_gpu_parity import RAGGED, Sim, check_field, gpu_field, mixed_charge_bunch, oracle_field, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
PRECS = ["fp64", "mixed"]
# (receivers per workgroup, workgroup size in units of 256 threads)
FUSED = [(4, 1), (8, 2), (16, 4), (32, 1), (32, 4)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    pp.load()
    return torch


@pytest.fixture(scope="module")
def orc():
    return default()


def tun(receivers, k=1, **kw):
    return {"symmetric": 0, "far_split": 0, "sym_split": 1, "fused": receivers, "i_per_lane": k, **kw}


def _state(b):
    return OracleState(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.q, b.m, b.weight, b.softening, b.dt)


@pytest.mark.parametrize("receivers,k", FUSED)
@pytest.mark.parametrize("prec", PRECS)
def test_fused_field_parity_ragged_batch(orc, prec, receivers, k):
    """Ragged bunches of 1..2049 particles with gaps, the paper's 12^3 lattice
    (no softening) and unlike charges in one batch."""
    bunches = [wl.cold_sphere(n, 30e-6 * (1 + i % 3), 2e4 * n, 1e-3, 0.01, 0, seed=700 + i, name=f"f{n}")
               for i, n in enumerate(RAGGED)]
    bunches += [wl.paper_cube(12), mixed_charge_bunch(1500, seed=23)]
    say(f"fused field {prec} receivers={receivers} threads={256 * k} sizes={[b.n for b in bunches]} gap=4")
    with Sim(bunches, prec, gap=4, tuning=tun(receivers, k)) as sim:
        assert sim.tuning()["fused"] == receivers
        full = gpu_field(sim)
        slices = [sim.bunch_slice(i) for i in range(len(bunches))]
        mask = np.ones(sim.n_total, bool)
        for sl in slices:
            mask[sl] = False
    assert np.all(full["ex"][mask] == 0) and np.all(full["phi"][mask] == 0)
    for i, b in enumerate(bunches):
        got = {key: v[slices[i]] for key, v in full.items()}
        if b.n == 1:
            assert got["ex"][0] == 0 and got["phi"][0] == 0
            continue
        check_field(got, oracle_field(orc, b), TOL[prec], f"fused n={b.n}")


@pytest.mark.parametrize("prec", PRECS)
def test_fused_push_graph_split_and_trajectory(orc, prec):
    """push == step_batched (graph and eager) == 7 + 13 steps, bitwise; the
    trajectory against the oracle's."""
    b = wl.workload("gaussian_65536", n_override=3000)[0]
    t = tun(8, graph_steps=4)
    say(f"fused push/graph/split {prec}")
    res = []
    for mode in ("push", "graph", "plain", "split"):
        with Sim([b], prec, tuning=t) as sim:
            if mode == "push":
                sim.push(20)
            elif mode == "split":
                sim.push(7)
                sim.step_batched(13, graph=True)
            else:
                sim.step_batched(20, graph=(mode == "graph"))
            res.append({key: sim.host(key) for key in ("x", "y", "z", "vx", "vy", "vz")})
    for r in res[1:]:
        for key in r:
            np.testing.assert_array_equal(res[0][key], r[key])
    s = _state(b)
    orc.vv(s, 20)
    r_rms = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    er = max(np.abs(res[0][key] - getattr(s, key)).max() for key in ("x", "y", "z")) / r_rms
    ev = max(np.abs(res[0][key] - getattr(s, key)).max() for key in ("vx", "vy", "vz")) / v_rms
    print(f"    fused trajectory: max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e}", flush=True)
    tol_r, tol_v = (1e-12, 1e-11) if prec == "fp64" else (1e-8, 1e-6)
    assert er <= tol_r and ev <= tol_v


@pytest.mark.parametrize("prec", PRECS)
def test_fused_batch_equals_separate_contexts_bitwise(prec):
    bunches = [wl.workload("gaussian_65536", n_override=n)[0] for n in (70, 700, 1300, 5000)]
    t = tun(16, 2)
    say(f"fused batch == separate {prec}")
    with Sim(bunches, prec, tuning=t) as sim:
        sim.push(3)
        batched = [np.concatenate([sim.host(key)[sim.bunch_slice(i)] for key in ("x", "vx", "vz")])
                   for i in range(len(bunches))]
    for i, b in enumerate(bunches):
        with Sim([b], prec, tuning=t) as one:
            one.push(3)
            alone = np.concatenate([one.host(key) for key in ("x", "vx", "vz")])
        np.testing.assert_array_equal(batched[i], alone)


@pytest.mark.parametrize("prec", PRECS)
def test_fused_diagnostics_and_graph_replays(orc, prec):
    """Diagnostics on the fused schedule against the oracle's on the GPU's
    state, and graph replays with eager work between them equal one-step
    pushes of a twin context."""
    b = wl.paper_cube(16)
    t = tun(4, graph_steps=5)
    say(f"fused diagnostics and graph replays {prec}")
    with Sim([b], prec, tuning=t) as g, Sim([b], prec, tuning=t) as e:
        for rep in range(3):
            g.step_batched(5, graph=True)
            for _ in range(5):
                e.push(1)
            d = g.diagnostics()[0]
            g.field(want_phi=True)
            for key in ("x", "vx", "z", "vz"):
                np.testing.assert_array_equal(g.host(key), e.host(key), err_msg=f"replay {rep} {key}")
        st = {key: g.host(key) for key in ("x", "y", "z", "vx", "vy", "vz")}
    ref = orc.diag(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], b.q, b.m, b.weight, b.softening)
    for key in ("potential", "total"):
        rel = abs(d[key] - ref[key]) / abs(ref[key])
        print(f"    {key}: rel {rel:.2e}", flush=True)
        assert rel <= TOL[prec]
    assert abs(d["kinetic"] - ref["kinetic"]) / abs(ref["kinetic"]) <= 1e-13
