"""GPU parity at the benchmark's and the paper's own configurations, at full
size, against the CPU FP64 oracle (trajectories, diagnostics and fields).

* the 65 536-particle Gaussian bunch: the first 10 Velocity Verlet steps of
  both precisions against the oracle's (Eqs. (G)/(H)), then the 1000-step
  total-energy gap between the mixed and the FP64 path through the library's
  own diagnostics;
* the 1 048 576-particle cold sphere: the same energy gap over 20 steps;
* the paper's 16^3 lattice cube (Sec. 2.1 setup: side 0.1 mm, n0 = 5e16 m^-3,
  no softening, dt = 1e-13 s) for 1000 steps, to t = 0.1 ns, the first sample
  of the paper's emittance series (Eq. (I));
* the paper's macro-particle sweep (Sec. 2.2: 4^3 .. 32^3 cubes) as one batch
  on its default tiling, fields at step 0 and after 10 steps, and trajectories;
* the PP baseline of the paper's PIC comparison (Sec. 3.2: 8^3 = 512 particles,
  dt = 1e-12 s, 100 steps) with the observables Sec. 3.2 plots;
* the 64-bunch sweep: sampled fields after 10 steps.

Tolerances.  Fields: the workload definition's 1e-12 (FP64) and 1e-5 (mixed).
Trajectories (max over particles, relative to the rms of the quantity): the
velocity is a time integral of the field, so its error is bounded by the
field's relative error, and the position error by that times the displacement
over r_rms (below 1 here); FP64 1e-12 for r and 1e-11 for v, mixed 1e-6 for r
and 1e-5 for v.  Beam moments (Eq. (I), rms, max) relative to their scale
(r_rms, v_rms or r_rms v_rms): FP64 1e-10, mixed 1e-5.  Total energy: FP64
1e-12, mixed 1e-6 (the energy gate).
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleState, default
from paper_2502_10640_amd import pp
from paper_2502_10640_amd import workloads as wl
from tests._metrics import cond_max, l2_rel, phi_cond_max, vec
from tests.test_gpu_parity import Sim, check_field, oracle_field, say

pytestmark = pytest.mark.gpu

TOL_FIELD = {"fp64": 1e-12, "mixed": 1e-5}
TOL_R = {"fp64": 1e-12, "mixed": 1e-6}
TOL_V = {"fp64": 1e-11, "mixed": 1e-5}
TOL_MOM = {"fp64": 1e-10, "mixed": 1e-5}
TOL_E = {"fp64": 1e-12, "mixed": 1e-6}
PRECS = ["fp64", "mixed"]
STATE = ("x", "y", "z", "vx", "vy", "vz")


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


def _state(b):
    return OracleState(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.q, b.m, b.weight, b.softening, b.dt)


def _host_state(sim, sl=None):
    out = {k: sim.host(k) for k in STATE}
    return out if sl is None else {k: v[sl] for k, v in out.items()}


def traj_errors(g, s):
    """max_i |dr_i| / r_rms and max_i |dv_i| / v_rms of a GPU state g against an
    oracle state s (one bunch); the rms are the oracle's."""
    r_rms = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    dr = np.sqrt(sum((g[k] - getattr(s, k)) ** 2 for k in ("x", "y", "z")))
    dv = np.sqrt(sum((g[k] - getattr(s, k)) ** 2 for k in ("vx", "vy", "vz")))
    return float(dr.max() / r_rms), float(dv.max() / v_rms)


MOMENT_KEYS = ("emittance", "emittance_centered", "x_rms", "x_max", "v_rms", "v_max")


def moment_errors(d, ref, r_rms, v_rms):
    """Largest error of the beam moments of Eq. (I) and Sec. 3.2 (per axis),
    each relative to its scale: r_rms for positions, v_rms for velocities,
    r_rms v_rms for emittances."""
    scale = {"emittance": r_rms * v_rms, "emittance_centered": r_rms * v_rms, "x_rms": r_rms, "x_max": r_rms,
             "v_rms": v_rms, "v_max": v_rms}
    return {k: float(np.abs(np.array(d[k]) - np.array(ref[k])).max() / scale[k]) for k in MOMENT_KEYS}


# ---------------------------------------------------------------------------
# the 65 536-particle Gaussian bunch
# ---------------------------------------------------------------------------

C2_STEPS = 10


@pytest.fixture(scope="module")
def c2_oracle(orc):
    """The oracle's first 10 steps of the full Gaussian bunch (4.7e10 pairs)
    and its diagnostics at the end."""
    b = wl.workload("gaussian_65536")[0]
    say(f"oracle: gaussian_65536, {C2_STEPS} steps (CPU, {orc.num_threads()} threads)")
    s = _state(b)
    orc.vv(s, C2_STEPS)
    return b, s, orc.diag_state(s)


@pytest.mark.parametrize("prec", PRECS)
def test_gaussian_65536_first_steps_against_oracle(c2_oracle, prec):
    """Full-size trajectory chain of the Gaussian bunch: the GPU path on its
    default tiling (graph replay, as the benchmark runs it) against the
    oracle's trajectory, element by element, and the total energy of the
    library's diagnostics against the oracle's."""
    b, s, dref = c2_oracle
    say(f"gaussian_65536 {prec}: {C2_STEPS} steps vs the oracle")
    with Sim([b], prec, tuning={"graph_steps": 5}) as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        sim.step_batched(C2_STEPS, graph=True)
        d = sim.diagnostics()[0]
        g = _host_state(sim)
    er, ev = traj_errors(g, s)
    de = abs(d["total"] - dref["total"]) / abs(dref["total"])
    print(f"    max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e} |dE_tot|/|E_tot|={de:.3e}", flush=True)
    assert d["step"] == C2_STEPS
    assert er <= TOL_R[prec] and ev <= TOL_V[prec]
    assert de <= TOL_E[prec]


def _energy_series(b_list, prec, n_steps, every, tuning=None):
    """Total energy per bunch from pp_diagnostics every `every` steps (hipGraph
    replay in between)."""
    out = []
    with Sim(b_list, prec, tuning=tuning) as sim:
        out.append([d["total"] for d in sim.diagnostics()])
        done = 0
        while done < n_steps:
            k = min(every, n_steps - done)
            sim.step_batched(k, graph=True)
            done += k
            ds = sim.diagnostics()
            assert all(d["step"] == done and d["nonfinite"] == 0 for d in ds)
            out.append([d["total"] for d in ds])
    return np.array(out)


def test_gaussian_65536_energy_gap_1000_steps():
    """Energy gate (ii): over the 1000 steps of the Gaussian workload the mixed
    path's total energy stays within 1e-6 of |E_tot(0)| of the FP64 path's,
    both from the library's FP64 diagnostics (sampled every 50 steps)."""
    b = wl.workload("gaussian_65536")[0]
    say("gaussian_65536: mixed vs fp64 total energy, 1000 steps, diagnostics every 50")
    tun = {"graph_steps": 50}
    e = {p: _energy_series([b], p, 1000, 50, tuning=tun)[:, 0] for p in PRECS}
    e0 = abs(e["fp64"][0])
    gap = float(np.max(np.abs(e["mixed"] - e["fp64"])) / e0)
    drift = {p: float(np.max(np.abs(e[p] - e[p][0])) / e0) for p in PRECS}
    print(f"    max_t|E_mixed - E_fp64|/|E0| = {gap:.3e}; drift fp64 {drift['fp64']:.3e} mixed {drift['mixed']:.3e}",
          flush=True)
    assert gap <= 1e-6


def test_cold_sphere_1m_energy_gap_20_steps():
    """Energy gate (ii) on the 1 048 576-particle sphere over 20 steps (every
    5 steps), both precisions on their default tilings."""
    b = wl.workload("cold_sphere_1m")[0]
    say("cold_sphere_1m: mixed vs fp64 total energy, 20 steps, diagnostics every 5")
    e = {p: _energy_series([b], p, 20, 5, tuning={"graph_steps": 5})[:, 0] for p in PRECS}
    e0 = abs(e["fp64"][0])
    gap = float(np.max(np.abs(e["mixed"] - e["fp64"])) / e0)
    drift = {p: float(np.max(np.abs(e[p] - e[p][0])) / e0) for p in PRECS}
    print(f"    max_t|E_mixed - E_fp64|/|E0| = {gap:.3e}; drift fp64 {drift['fp64']:.3e} mixed {drift['mixed']:.3e}",
          flush=True)
    assert gap <= 1e-6


# ---------------------------------------------------------------------------
# the paper's 16^3 cube to t = 0.1 ns
# ---------------------------------------------------------------------------

CUBE_STEPS = 1000


@pytest.fixture(scope="module")
def cube_oracle(orc):
    b = wl.paper_cube(16)
    say(f"oracle: paper cube 16^3, eps = 0, dt = 1e-13 s, {CUBE_STEPS} steps")
    s = _state(b)
    orc.vv(s, CUBE_STEPS)
    return b, s, orc.diag_state(s)


@pytest.mark.parametrize("prec", PRECS)
def test_paper_cube_16_to_first_emittance_sample(cube_oracle, prec):
    """The paper's own run (Sec. 2.1 setup) for its first 0.1 ns: positions and
    velocities of every particle, the emittance of Eq. (I) and the rms and
    maximum of x and v_x, against the oracle (default tiling, 200-step graphs
    as the paper-run benchmark replays them)."""
    b, s, dref = cube_oracle
    assert b.softening == 0.0 and b.dt == 1e-13
    say(f"paper cube 16^3 {prec}: {CUBE_STEPS} steps vs the oracle")
    with Sim([b], prec, tuning={"graph_steps": 200}) as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        sim.step_batched(CUBE_STEPS, graph=True)
        d = sim.diagnostics()[0]
        g = _host_state(sim)
    er, ev = traj_errors(g, s)
    r_rms = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    me = moment_errors(d, dref, r_rms, v_rms)
    de = abs(d["total"] - dref["total"]) / abs(dref["total"])
    print(f"    t={d['time']:.3e} s eps_x={d['emittance'][0]:.6e} (oracle {dref['emittance'][0]:.6e})", flush=True)
    print(f"    max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e} |dE|/|E|={de:.3e} moments {me}", flush=True)
    assert d["time"] == pytest.approx(1e-10, rel=1e-12, abs=0)
    assert er <= TOL_R[prec] and ev <= TOL_V[prec]
    assert max(me.values()) <= TOL_MOM[prec]
    assert de <= TOL_E[prec]


# ---------------------------------------------------------------------------
# the paper's macro-particle sweep as one batch, on its default tiling
# ---------------------------------------------------------------------------

def test_paper_np_batch_default_tiling_fields_and_trajectories(orc):
    """The 4^3 .. 32^3 cubes (no softening) as one batch on the tiling the
    library picks for them (the symmetric schedule with the near/far split,
    block pairs split in parts): every bunch's field and potential against the
    oracle at step 0 and at the GPU's state after 10 steps, and the 10-step
    trajectories against the oracle's."""
    bunches = wl.workload("paper_np_batch")
    steps = 10
    say(f"paper N_p batch {[b.n for b in bunches]}: default tiling, fields at steps 0 and {steps}, trajectories")
    with Sim(bunches, "mixed") as sim:
        t = sim.tuning()
        print(f"    tuning {t}", flush=True)
        assert t["symmetric"] == 1 and t["far_split"] > 0
        f0 = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        sim.step_batched(steps, graph=True)
        f1 = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        g = _host_state(sim)
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
    for k, b in enumerate(bunches):
        sl = slices[k]
        check_field({key: v[sl] for key, v in f0.items()}, oracle_field(orc, b), TOL_FIELD["mixed"],
                    f"{b.n} step 0")
        gk = {key: v[sl] for key, v in g.items()}
        at = orc.field(gk["x"], gk["y"], gk["z"], b.q, b.weight, b.softening, want_phi=True, want_amag=True,
                       want_pmag=True)
        check_field({key: v[sl] for key, v in f1.items()}, at, TOL_FIELD["mixed"], f"{b.n} step {steps}")
        s = _state(b)
        orc.vv(s, steps)
        er, ev = traj_errors(gk, s)
        print(f"    {b.n}: max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e}", flush=True)
        assert er <= TOL_R["mixed"] and ev <= TOL_V["mixed"]


# ---------------------------------------------------------------------------
# Sec. 3.2: the PP baseline of the PIC comparison, 512 particles, 100 steps
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def baseline_512_oracle(orc):
    """The oracle's run of the 8^3 cube at dt = 1e-12 s with its diagnostics
    every 10 steps (100 steps, 2.6e7 pairs)."""
    b = wl.paper_cube(8, dt=1e-12)
    s = _state(b)
    series = [orc.diag_state(s)]
    for _ in range(10):
        orc.vv(s, 10)
        series.append(orc.diag_state(s))
    return b, s, series


@pytest.mark.parametrize("prec", PRECS)
def test_paper_pic_comparison_baseline_512(baseline_512_oracle, prec):
    """Sec. 3.2's PP run (N_p = 8^3 in the 0.1 mm cube, dt = 1e-12 s, 100 steps)
    in full against the oracle: every 10 steps the emittance of Eq. (I), the
    rms and maximum of x and of v_x (the quantities Sec. 3.2 compares) and the
    total energy; at the end every particle's position and velocity."""
    b, s, series = baseline_512_oracle
    say(f"paper Sec. 3.2 baseline 8^3 {prec}: 100 steps vs the oracle")
    worst = {}
    with Sim([b], prec, tuning={"graph_steps": 10}) as sim:
        for k, dref in enumerate(series):
            if k:
                sim.step_batched(10, graph=True)
            d = sim.diagnostics()[0]
            assert d["step"] == 10 * k
            st = _host_state(sim)
            r_rms = math.sqrt(np.mean(st["x"] ** 2 + st["y"] ** 2 + st["z"] ** 2))
            v_rms = math.sqrt(np.mean(st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)) or 1.0
            me = moment_errors(d, dref, r_rms, v_rms)
            me["total"] = abs(d["total"] - dref["total"]) / abs(dref["total"])
            for key, v in me.items():
                worst[key] = max(worst.get(key, 0.0), v)
        g = _host_state(sim)
    er, ev = traj_errors(g, s)
    print(f"    max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e} worst over the series {worst}", flush=True)
    print(f"    eps_x(100 ps) = {series[-1]['emittance'][0]:.6e}", flush=True)
    assert er <= TOL_R[prec] and ev <= TOL_V[prec]
    assert worst.pop("total") <= TOL_E[prec]
    assert max(worst.values()) <= TOL_MOM[prec]


# ---------------------------------------------------------------------------
# the 64-bunch sweep after 10 steps
# ---------------------------------------------------------------------------

def test_sweep_64_sampled_fields_after_10_steps(orc):
    """The 64-bunch sweep on its default tiling: after 10 steps (graph
    replay; the far split's order is reused between its 8-step re-sorts) the
    field and potential at 16 sampled receivers per bunch against the oracle
    at the GPU's positions."""
    bunches = wl.workload("sweep_64")
    rng = np.random.default_rng(96)
    say(f"sweep_64: 10 steps, then sampled fields ({sum(b.n for b in bunches)} particles)")
    with Sim(bunches, "mixed") as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        sim.step_batched(10, graph=True)
        full = {k: v.cpu().numpy() for k, v in sim.field(want_phi=True).items()}
        pos = {k: sim.host(k) for k in ("x", "y", "z")}
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
    worst = 0.0
    for k, b in enumerate(bunches):
        sl = slices[k]
        recv = np.sort(rng.choice(b.n, 16, replace=False))
        got = {key: v[sl][recv] for key, v in full.items()}
        ref = orc.field(pos["x"][sl], pos["y"][sl], pos["z"][sl], b.q, b.weight, b.softening, recv=recv,
                        want_phi=True, want_amag=True, want_pmag=True)
        G, R = vec(got), vec(ref)
        e = max(l2_rel(G, R), cond_max(G, R, ref["amag"]), phi_cond_max(got["phi"], ref["phi"], ref["pmag"]))
        worst = max(worst, e)
        assert e <= TOL_FIELD["mixed"], (k, b.n, e)
    print(f"    worst over bunches {worst:.3e}", flush=True)
