"""GPU parity: the HIP library (through the C ABI) against the CPU FP64 oracle.

Tolerances (stated by the workload definition): field relative error
<= 1e-12 on the FP64 path and <= 1e-5 on the mixed path, in both the L2 and
the condition-aware max norm (tests/_metrics.py).  Equivalence tests are
bitwise.  Each test prints the case it runs before touching the GPU.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OracleState, default
from paper_2502_10640_amd import pp
from paper_2502_10640_amd import workloads as wl
from tests._metrics import cond_max, l2_rel, phi_cond_max, vec

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}
PRECS = ["fp64", "mixed"]
# the two-kernel ordered-pair schedule (small bunches default to the fused one)
ORDERED_TUNING = {"symmetric": 0, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 1}


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    pp.load()  # raises if the library is missing: there is no fallback
    return torch


@pytest.fixture(scope="module")
def orc():
    return default()


def say(msg):
    print(f"[case] {msg}", flush=True)


def Sim(*a, **k):
    from paper_2502_10640_amd.sim import Simulation
    return Simulation(*a, **k)


def gpu_field(sim, sl=None, phi=True):
    f = sim.field(want_phi=phi)
    h = {k: v.cpu().numpy() for k, v in f.items()}
    if sl is not None:
        h = {k: v[sl] for k, v in h.items()}
    return h


def oracle_field(orc, b, recv=None):
    return orc.field(b.x, b.y, b.z, b.q, b.weight, b.softening, recv=recv, want_phi=True, want_amag=True,
                     want_pmag=True)


def check_field(got, ref, tol, label):
    """Field: relative L2 and the condition-aware max; potential (when both
    sides have it): relative L2 and the per-particle max of |dphi_i| / P_i."""
    G, R = vec(got), vec(ref)
    e_l2 = l2_rel(G, R)
    e_cm = cond_max(G, R, ref["amag"])
    e_phi = l2_rel(got["phi"], ref["phi"]) if "phi" in got else 0.0
    e_pcm = phi_cond_max(got["phi"], ref["phi"], ref["pmag"]) if "phi" in got and "pmag" in ref else 0.0
    print(f"    {label}: l2={e_l2:.3e} cond_max={e_cm:.3e} phi_l2={e_phi:.3e} phi_cond_max={e_pcm:.3e}", flush=True)
    assert e_l2 <= tol, (label, e_l2)
    assert e_cm <= tol, (label, e_cm)
    assert e_phi <= tol, (label, e_phi)
    assert e_pcm <= tol, (label, e_pcm)
    return e_l2, e_cm


def mixed_charge_bunch(n=1500, seed=21):
    """Electrons and positive ions of different mass, no softening (bare Eq. (B))."""
    rng = np.random.default_rng(seed)
    x, y, z = wl.zero_mean(*wl.gaussian(n, 20e-6, rng))
    q = np.where(rng.random(n) < 0.7, -wl.E_CHARGE, 2 * wl.E_CHARGE)
    m = np.where(q < 0, wl.M_ELECTRON, 7.3e-27)
    vx, vy, vz = wl.maxwellian(n, 0.3, rng)
    return wl.Bunch(x, y, z, vx, vy, vz, q, m, 50.0, 0.0, 1e-14, 0, {"name": "mixed_charges"})


FIELD_CASES = {
    "cold_sphere_2048": lambda: wl.workload("cold_sphere_2048")[0],
    "gaussian_8192": lambda: wl.workload("gaussian_65536", n_override=8192)[0],
    "paper_cube_12^3_eps0": lambda: wl.paper_cube(12),
    "mixed_charges_1500_eps0": mixed_charge_bunch,
}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", list(FIELD_CASES))
def test_field_parity(orc, prec, case):
    b = FIELD_CASES[case]()
    say(f"field {case} {prec} n={b.n}")
    with Sim([b], prec) as sim:
        got = gpu_field(sim)
    check_field(got, oracle_field(orc, b), TOL[prec], f"{case}/{prec}")


RAGGED = [1, 2, 3, 63, 255, 256, 257, 511, 513, 777, 1025, 2049]


@pytest.mark.parametrize("sched", ["ordered", "symmetric_far"])
def test_three_hundred_small_bunches(orc, sched):
    """300 bunches of 1..100 particles in one context (nine bunch-index bits in
    the far split's sort keys, a long bunch table): every bunch's field against
    the oracle."""
    rng = np.random.default_rng(404)
    sizes = [int(v) for v in rng.integers(1, 101, 300)]
    bunches = [wl.cold_sphere(n, 20e-6, 1e4 * n, 1e-3, 0.01, 0, seed=5000 + k, name=f"s{k}")
               for k, n in enumerate(sizes)]
    tun = ORDERED_TUNING if sched == "ordered" else {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3}
    say(f"300 small bunches ({sched}), {sum(sizes)} particles")
    with Sim(bunches, "mixed", tuning=tun) as sim:
        full = gpu_field(sim)
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
    worst = 0.0
    for k, b in enumerate(bunches):
        got = {key: v[slices[k]] for key, v in full.items()}
        if b.n == 1:
            assert got["ex"][0] == 0 and got["phi"][0] == 0
            continue
        ref = oracle_field(orc, b)
        e = l2_rel(vec(got), vec(ref))
        worst = max(worst, e)
        assert e <= TOL["mixed"] and cond_max(vec(got), vec(ref), ref["amag"]) <= TOL["mixed"], (k, b.n, e)
        assert phi_cond_max(got["phi"], ref["phi"], ref["pmag"]) <= TOL["mixed"], (k, b.n)
    print(f"    worst relative L2 over the bunches {worst:.3e}", flush=True)


RAGGED_TUNINGS = {"ordered": {"symmetric": 0, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 1},
                  "symmetric": {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 1},
                  "symmetric_k4": {"symmetric": 1, "fused": 0, "i_per_lane": 4, "far_split": 0, "sym_split": 1},
                  "symmetric_k2_split4": {"symmetric": 1, "fused": 0, "i_per_lane": 2, "far_split": 0, "sym_split": 4}}


@pytest.mark.parametrize("sched", list(RAGGED_TUNINGS))
@pytest.mark.parametrize("prec", PRECS)
def test_ragged_batch_with_gaps(orc, prec, sched):
    bunches = [wl.cold_sphere(n, 30e-6 * (1 + k % 3), 2e4 * n, 1e-3, 0.01, 0, seed=300 + k, name=f"r{n}")
               for k, n in enumerate(RAGGED)]
    say(f"ragged batch {prec} {sched} sizes={RAGGED} gap=5")
    with Sim(bunches, prec, gap=5, tuning=RAGGED_TUNINGS[sched]) as sim:
        full = gpu_field(sim)
        for k, b in enumerate(bunches):
            sl = sim.bunch_slice(k)
            got = {key: v[sl] for key, v in full.items()}
            if b.n == 1:
                assert got["ex"][0] == 0 and got["phi"][0] == 0
                continue
            check_field(got, oracle_field(orc, b), TOL[prec], f"n={b.n}")
        # slots between bunches are never written
        mask = np.ones(sim.n_total, bool)
        for k in range(len(bunches)):
            mask[sim.bunch_slice(k)] = False
        assert mask.sum() == 5 * len(bunches)
        assert np.all(full["ex"][mask] == 0) and np.all(full["phi"][mask] == 0)


@pytest.mark.parametrize("prec", PRECS)
def test_every_tiling_within_tolerance(orc, prec):
    b = wl.workload("gaussian_65536", n_override=3000)[0]
    ref = oracle_field(orc, b)
    ks = (1, 2, 4, 8) if prec == "mixed" else (1, 2, 4)
    say(f"tilings {prec} n={b.n}")
    with Sim([b], prec) as sim:
        for k in ks:
            for ts in (32, 256):
                for cl in (16, 22):
                    for gpc in (1, 4):
                        sim.set_tuning(symmetric=0, fused=0, far_split=0, sym_split=1, i_per_lane=k, sum_tile=ts,
                                       chunk_pairs_log2=cl, grid_per_cu=gpc)
                        check_field(gpu_field(sim), ref, TOL[prec], f"K={k} ts={ts} cl={cl} gpc={gpc}")


def _state(b):
    return OracleState(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.q, b.m, b.weight, b.softening, b.dt)


@pytest.mark.parametrize("sched", ["default", "ordered"])
@pytest.mark.parametrize("prec", PRECS)
def test_push_parity(orc, prec, sched):
    b = wl.workload("gaussian_65536", n_override=1024)[0]
    steps = 25
    say(f"push {prec} {sched} n={b.n} steps={steps}")
    s = _state(b)
    orc.vv(s, steps)
    with Sim([b], prec, tuning=None if sched == "default" else ORDERED_TUNING) as sim:
        sim.push(steps)
        g = {k: sim.host(k) for k in ("x", "y", "z", "vx", "vy", "vz")}
    r_rms = math.sqrt(np.mean(s.x ** 2 + s.y ** 2 + s.z ** 2))
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    er = max(np.abs(g[k] - getattr(s, k)).max() for k in ("x", "y", "z")) / r_rms
    ev = max(np.abs(g[k] - getattr(s, k)).max() for k in ("vx", "vy", "vz")) / v_rms
    print(f"    trajectory: max|dr|/r_rms={er:.3e} max|dv|/v_rms={ev:.3e}", flush=True)
    tol_r, tol_v = (1e-12, 1e-11) if prec == "fp64" else (1e-8, 1e-6)
    assert er <= tol_r and ev <= tol_v


DIAG_SCALARS = ("kinetic", "potential", "total")
DIAG_VECTORS = ("com", "com_velocity", "emittance", "emittance_centered", "x_rms", "x_max", "v_rms", "v_max")


DIAG_TUNING = {"fp64": None, "mixed": None, "fp64_ordered": ORDERED_TUNING, "mixed_ordered": ORDERED_TUNING,
               "mixed_symmetric_far": {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3},
               "fp64_symmetric": {"symmetric": 1, "fused": 0, "i_per_lane": 1}}


@pytest.mark.parametrize("variant", list(DIAG_TUNING))
def test_diagnostics_parity(orc, variant):
    """GPU diagnostics against the oracle's on the GPU's own state."""
    prec = "fp64" if variant.startswith("fp64") else "mixed"
    b = wl.workload("gaussian_65536", n_override=4096)[0]
    say(f"diagnostics {variant} n={b.n}")
    with Sim([b], prec, tuning=DIAG_TUNING[variant]) as sim:
        sim.push(5)
        d = sim.diagnostics()[0]
        st = {k: sim.host(k) for k in ("x", "y", "z", "vx", "vy", "vz")}
    ref = orc.diag(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], b.q, b.m, b.weight, b.softening)
    tol_pe = TOL[prec]
    for k in DIAG_SCALARS:
        rel = abs(d[k] - ref[k]) / abs(ref[k])
        print(f"    {k}: gpu={d[k]:.12e} oracle={ref[k]:.12e} rel={rel:.2e}", flush=True)
        assert rel <= (1e-13 if k == "kinetic" else tol_pe)
    r_rms = math.sqrt(np.mean(st["x"] ** 2 + st["y"] ** 2 + st["z"] ** 2))
    v_rms = math.sqrt(np.mean(st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2))
    scale = {"com": r_rms, "x_rms": r_rms, "x_max": r_rms, "com_velocity": v_rms, "v_rms": v_rms,
             "v_max": v_rms, "emittance": r_rms * v_rms, "emittance_centered": r_rms * v_rms}
    for k in DIAG_VECTORS:
        # com and com_velocity are ~0 in the centre-of-mass frame: compare on the quantity's scale
        err = np.abs(np.array(d[k]) - np.array(ref[k])).max() / scale[k]
        print(f"    {k}: max err / scale = {err:.2e}", flush=True)
        assert err <= 1e-12, k
    pscale = (b.weight * b.m * np.sqrt(st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)).sum()
    assert np.abs(np.array(d["momentum"]) - ref["momentum"]).max() <= 1e-13 * pscale
    assert d["nonfinite"] == 0 and d["step"] == 5 and d["n"] == b.n
    assert d["time"] == pytest.approx(5 * b.dt, rel=1e-15, abs=0)


def test_diagnostics_write_only_the_callers_records():
    """pp_diagnostics fills exactly one pp_diag per bunch: a guard record after
    the caller's array stays untouched (an earlier version copied two doubles
    too many per record and corrupted the caller's heap)."""
    import ctypes
    bunches = [wl.workload("cold_sphere_2048", n_override=n)[0] for n in (300, 77, 1)]
    say("diagnostics guard record, 3 bunches")
    with Sim(bunches, "mixed") as sim:
        nb = len(bunches)
        buf = (pp.Diag * (nb + 1))()
        size = ctypes.sizeof(pp.Diag)
        ctypes.memset(ctypes.addressof(buf) + nb * size, 0x5A, size)
        st = pp.load().pp_diagnostics(sim.ctx, buf)
        assert st == pp.PP_OK, pp.pp_last_error(sim.ctx)
        assert ctypes.string_at(ctypes.addressof(buf) + nb * size, size) == b"\x5a" * size
        assert [buf[k].n for k in range(nb)] == [b.n for b in bunches]
        assert all(buf[k].nonfinite == 0 for k in range(nb))
        assert buf[2].potential == 0.0 and buf[0].potential > 0.0


@pytest.mark.parametrize("prec", PRECS)
def test_push_equals_step_batched_bitwise(prec):
    b = wl.workload("gaussian_65536", n_override=1500)[0]
    say(f"push == step_batched (graph, no graph) {prec}")
    res = []
    for mode in ("push", "graph", "plain"):
        with Sim([b], prec, tuning={"graph_steps": 4}) as sim:
            if mode == "push":
                sim.push(10)
            else:
                sim.step_batched(10, graph=(mode == "graph"))
            res.append(np.concatenate([sim.host(k) for k in ("x", "y", "z", "vx", "vy", "vz")]))
    np.testing.assert_array_equal(res[0], res[1])
    np.testing.assert_array_equal(res[0], res[2])


@pytest.mark.parametrize("prec", PRECS)
def test_batch_equals_separate_contexts_bitwise(prec):
    _batch_equals_separate(prec, {"i_per_lane": 1, "symmetric": 0, "fused": 0, "far_split": 0, "sym_split": 1})


def test_symmetric_far_batch_equals_separate_contexts_bitwise():
    # the sort keys, the coordinate bound, the boxes and the fold are all per bunch
    _batch_equals_separate("mixed", {"i_per_lane": 1, "symmetric": 1, "fused": 0, "far_split": 3, "sym_split": 1})


def test_fp64_symmetric_batch_equals_separate_contexts_bitwise():
    _batch_equals_separate("fp64", {"i_per_lane": 1, "symmetric": 1, "fused": 0, "far_split": 0, "sym_split": 1})


@pytest.mark.parametrize("prec", PRECS)
def test_split_symmetric_batch_equals_separate_contexts_bitwise(prec):
    _batch_equals_separate(prec, {"i_per_lane": 1, "symmetric": 1, "fused": 0, "far_split": 3 if prec == "mixed" else 0,
                                  "sym_split": 2})


def _batch_equals_separate(prec, tuning):
    # sizes with different Morton resolutions (4, 5, 5 and 6 bits per axis): the
    # far split's sort keys then differ in width alone and in the batch
    bunches = [wl.workload("gaussian_65536", n_override=n)[0] for n in (70, 700, 1300, 5000)]
    say(f"batch == separate {prec} {tuning}")
    with Sim(bunches, prec, tuning=tuning) as sim:
        sim.push(3)
        batched = [np.concatenate([sim.host(k)[sim.bunch_slice(i)] for k in ("x", "vx", "vz")])
                   for i in range(len(bunches))]
    for i, b in enumerate(bunches):
        with Sim([b], prec, tuning=tuning) as one:
            one.push(3)
            alone = np.concatenate([one.host(k) for k in ("x", "vx", "vz")])
        np.testing.assert_array_equal(batched[i], alone)


@pytest.mark.parametrize("prec", PRECS)
def test_run_to_run_and_split_run_bitwise(prec):
    b = wl.workload("cold_sphere_2048")[0]
    say(f"run-to-run and 10+10 == 20 {prec}")
    with Sim([b], prec) as s1, Sim([b], prec) as s2:
        f1, f2 = gpu_field(s1), gpu_field(s2)
        for k in f1:
            np.testing.assert_array_equal(f1[k], f2[k])
        s1.push(20)
        s2.push(10)
        s2.push(10)
        for k in ("x", "vy", "z"):
            np.testing.assert_array_equal(s1.host(k), s2.host(k))


def _energy(sim, b):
    """Total energy from the GPU's state and its softened potential (pp_field
    with phi); the sums are done here in FP64."""
    f = sim.field(want_phi=True)
    phi = f["phi"].cpu().numpy()
    v2 = sim.host("vx") ** 2 + sim.host("vy") ** 2 + sim.host("vz") ** 2
    ke = 0.5 * b.weight * np.sum(b.m * v2)
    pe = 0.5 * b.weight * np.sum(b.q * phi)
    return ke + pe


def test_mixed_energy_tracks_fp64(orc):
    """Total energy of the mixed path follows the FP64 path within 1e-6 of
    |E_tot(0)| over 100 steps; each path's own drift is reported."""
    b = wl.workload("gaussian_65536", n_override=4096)[0]
    say("energy mixed vs fp64, 100 steps, n=4096 (phi from pp_field)")
    traj = {}
    for prec in PRECS:
        with Sim([b], prec) as sim:
            es = [_energy(sim, b)]
            for _ in range(10):
                sim.push(10)
                es.append(_energy(sim, b))
            traj[prec] = np.array(es)
    e0 = abs(traj["fp64"][0])
    gap = np.abs(traj["mixed"] - traj["fp64"]).max() / e0
    drift = {p: np.abs(traj[p] - traj[p][0]).max() / e0 for p in PRECS}
    print(f"    max|E_mixed-E_fp64|/|E0|={gap:.3e} drift fp64={drift['fp64']:.3e} mixed={drift['mixed']:.3e}",
          flush=True)
    assert gap <= 1e-6


def test_nonfinite_is_detected_and_context_survives():
    b = wl.workload("cold_sphere_2048", n_override=300)[0]
    b.softening = 0.0
    b.x[7], b.y[7], b.z[7] = b.x[3], b.y[3], b.z[3]    # coincident pair, no softening
    say("PP_CHECK non-finite")
    with Sim([b], "mixed") as sim:
        with pytest.raises(pp.PPError) as e:
            sim.step_batched(2, graph=False, check=True)
        assert e.value.status == pp.PP_ERR_NOT_FINITE
        sim.sync()   # still usable
        assert not np.all(np.isfinite(sim.host("vx")))


COINCIDENT_TILINGS = {
    "ordered": ORDERED_TUNING,
    "fused": {"symmetric": 0, "far_split": 0, "sym_split": 1, "fused": 8, "i_per_lane": 2},
    "symmetric": {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 1},
    "symmetric_far": {"symmetric": 1, "fused": 0, "i_per_lane": 2, "far_split": 3, "sym_split": 2},
}


@pytest.mark.parametrize("prec,sched", [(p, s) for p in PRECS for s in COINCIDENT_TILINGS
                                         if not (s == "symmetric_far" and p == "fp64")])
def test_coincident_particles(orc, prec, sched):
    """Two pairs of particles at the same position, one pair inside a block
    and one across blocks.  Softened, Eq. (B) is well defined there (the pair
    term is zero): every field and potential equals the oracle's.  Without
    softening the pair term is 0/0: exactly the four coincident particles get
    a non-finite field and potential, and every other particle equals the
    oracle's."""
    b = wl.workload("cold_sphere_2048", n_override=3000)[0]
    for i, j in ((3, 7), (10, 2500)):
        b.x[j], b.y[j], b.z[j] = b.x[i], b.y[i], b.z[i]
    bad = np.zeros(b.n, bool)
    bad[[3, 7, 10, 2500]] = True
    t = COINCIDENT_TILINGS[sched]
    say(f"coincident particles {prec} {sched} n={b.n} eps={b.softening:.3e} and 0")
    with Sim([b], prec, tuning=t) as sim:
        got = gpu_field(sim)
    check_field(got, oracle_field(orc, b), TOL[prec], f"coincident softened {sched}")
    b.softening = 0.0
    with Sim([b], prec, tuning=t) as sim:
        got = gpu_field(sim)
    ref = oracle_field(orc, b)
    for key in ("ex", "ey", "ez", "phi"):
        assert not np.any(np.isfinite(got[key][bad])), key
        assert np.all(np.isfinite(got[key][~bad])), key
    sub = lambda d: {key: v[~bad] for key, v in d.items()}
    check_field(sub(got), sub(ref), TOL[prec], f"coincident unsoftened {sched}, the other particles")


@pytest.mark.parametrize("prec,sched", [(p, s) for p in PRECS for s in COINCIDENT_TILINGS
                                         if not (s == "symmetric_far" and p == "fp64")])
def test_zero_extent_bunches(orc, prec, sched):
    """Bunches with no extent: one particle with and without softening, and
    three particles at one point with softening, in one batch beside an
    ordinary bunch.  Their fields are exactly zero and so are the lone
    particles' potentials (a zero extent must not blow up the mixed frame's
    scale); the three coincident ones each see the potential 2 q / eps of the
    other two, equal to the oracle's; the ordinary bunch's values are finite."""
    lone = wl.workload("cold_sphere_2048", n_override=1)[0]
    bare = wl.workload("cold_sphere_2048", n_override=1)[0]
    bare.softening = 0.0
    trio = wl.workload("cold_sphere_2048", n_override=3)[0]
    for k in (1, 2):
        trio.x[k], trio.y[k], trio.z[k] = trio.x[0], trio.y[0], trio.z[0]
    other = wl.workload("cold_sphere_2048", n_override=700)[0]
    bunches = [lone, bare, trio, other]
    say(f"zero-extent bunches {prec} {sched}")
    with Sim(bunches, prec, tuning=COINCIDENT_TILINGS[sched]) as sim:
        got = gpu_field(sim)
        slices = [sim.bunch_slice(i) for i in range(len(bunches))]
    for i in range(3):
        for key in ("ex", "ey", "ez") + (("phi",) if i < 2 else ()):
            assert np.all(got[key][slices[i]] == 0.0), (i, key, got[key][slices[i]])
    ref = oracle_field(orc, trio)["phi"]
    np.testing.assert_allclose(got["phi"][slices[2]], ref, rtol=TOL[prec], atol=0)
    for key in ("ex", "ey", "ez", "phi"):
        assert np.all(np.isfinite(got[key][slices[3]]))


@pytest.mark.parametrize("prec,sched", [(p, s) for p in PRECS for s in COINCIDENT_TILINGS
                                         if not (s == "symmetric_far" and p == "fp64")])
def test_neutral_bunches(orc, prec, sched):
    """Bunches whose particles carry no charge: alone, and in a batch beside a
    bunch of equal charges (where the uniform-charge kernels would otherwise
    apply).  Their fields and potentials are exactly zero; the charged
    bunch's equal the oracle's."""
    neutral = wl.workload("cold_sphere_2048", n_override=900)[0]
    neutral.q[:] = 0.0
    charged = wl.workload("cold_sphere_2048", n_override=1300)[0]
    t = COINCIDENT_TILINGS[sched]
    say(f"neutral bunches {prec} {sched}")
    with Sim([neutral], prec, tuning=t) as sim:
        alone = gpu_field(sim)
    with Sim([neutral, charged], prec, tuning=t) as sim:
        both = gpu_field(sim)
        s0, s1 = sim.bunch_slice(0), sim.bunch_slice(1)
    for key in ("ex", "ey", "ez", "phi"):
        assert np.all(alone[key] == 0.0), key
        assert np.all(both[key][s0] == 0.0), key
    check_field({key: v[s1] for key, v in both.items()}, oracle_field(orc, charged), TOL[prec],
                f"beside a neutral bunch {sched}")


def test_device_side_validation():
    b = wl.workload("cold_sphere_2048", n_override=64)[0]
    say("create validates q and m on the device")
    b.m[5] = -1.0
    with pytest.raises(pp.PPError) as e:
        Sim([b], "mixed")
    assert e.value.status == pp.PP_ERR_INVALID_ARG and "mass" in e.value.message
    b = wl.workload("cold_sphere_2048", n_override=64)[0]
    b.q[9] = np.nan
    with pytest.raises(pp.PPError) as e:
        Sim([b], "fp64")
    assert e.value.status == pp.PP_ERR_INVALID_ARG


def test_invalid_tuning_rejected():
    b = wl.workload("cold_sphere_2048", n_override=64)[0]
    say("invalid tuning")
    with Sim([b], "fp64") as sim:
        for bad in ({"i_per_lane": 3}, {"i_per_lane": 8}, {"sum_tile": 48}, {"grid_per_cu": 0},
                    {"chunk_pairs_log2": 40}, {"graph_steps": 0}, {"symmetric": 1, "fused": 0, "i_per_lane": 8}):
            with pytest.raises(pp.PPError) as e:
                sim.set_tuning(**bad)
            assert e.value.status == pp.PP_ERR_INVALID_ARG
        sim.push(1)


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_sampled_parity_cold_sphere_1m(orc, prec):
    """The 1 048 576-particle cold sphere in the benchmark's configuration
    (default tiling of each precision): the GPU field at 384 sampled receivers
    against the oracle."""
    b = wl.workload("cold_sphere_1m")[0]
    rng = np.random.default_rng(99)
    recv = np.sort(rng.choice(b.n, 384, replace=False))
    say(f"full size sampled parity cold_sphere_1m {prec} n={b.n}")
    with Sim([b], prec) as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        got = gpu_field(sim, sl=recv)
    ref = oracle_field(orc, b, recv=recv)
    check_field(got, ref, TOL[prec], f"cold_sphere_1m/{prec} sampled")


@pytest.mark.parametrize("prec", PRECS)
def test_split_with_many_slot_bands_sampled_parity_1m(orc, prec):
    """Block pairs split in 2 at 1 048 576 particles: the sub-rounds' slots
    exceed one 12 GiB band (3 bands mixed, 6 FP64), so the fold carries the
    accumulators across bands and the diagonal items sit in the first one."""
    b = wl.workload("cold_sphere_1m")[0]
    rng = np.random.default_rng(98)
    recv = np.sort(rng.choice(b.n, 256, replace=False))
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 4, "sym_split": 2, "far_split": 3 if prec == "mixed" else 0}
    say(f"split 2 with slot bands, cold_sphere_1m {prec}")
    with Sim([b], prec, tuning=tun) as sim:
        got = gpu_field(sim, sl=recv)
    check_field(got, oracle_field(orc, b, recv=recv), TOL[prec], f"cold_sphere_1m/{prec} split 2 sampled")


# ---------------------------------------------------------------------------
# symmetric (one rsq per unordered pair) schedule
# ---------------------------------------------------------------------------

def _sym_bunches():
    return [wl.workload("gaussian_65536", n_override=3000)[0], wl.workload("cold_sphere_2048")[0],
            mixed_charge_bunch(1500, seed=5), wl.workload("cold_sphere_2048", n_override=5)[0]]


@pytest.mark.parametrize("prec,K,split", [("mixed", 1, 1), ("mixed", 2, 1), ("mixed", 4, 1), ("fp64", 1, 1),
                                          ("fp64", 2, 1), ("fp64", 4, 1), ("mixed", 1, 4), ("mixed", 4, 2),
                                          ("fp64", 1, 4), ("fp64", 4, 2)])
def test_symmetric_field_parity(orc, prec, K, split):
    # split > 1: each block pair (diagonal ones too) is swept as `split` items
    # over parts of the source block, folded in a fixed order
    bunches = _sym_bunches()
    say(f"symmetric field {prec} K={K} split={split} sizes={[b.n for b in bunches]}")
    with Sim(bunches, prec, tuning={"symmetric": 1, "fused": 0, "i_per_lane": K, "far_split": 0, "sym_split": split}) as sim:
        assert sim.tuning()["symmetric"] == 1 and sim.tuning()["sym_split"] == split
        full = gpu_field(sim)
        for k, b in enumerate(bunches):
            sl = sim.bunch_slice(k)
            got = {key: v[sl] for key, v in full.items()}
            check_field(got, oracle_field(orc, b), TOL[prec], f"sym {prec} K={K} n={b.n}")


@pytest.mark.parametrize("K,split", [(1, 1), (4, 1), (1, 4)])
@pytest.mark.parametrize("prec", PRECS)
def test_symmetric_push_graph_and_trajectory(orc, prec, K, split):
    b = wl.workload("gaussian_65536", n_override=2500)[0]
    say(f"symmetric push == step_batched(graph) and trajectory vs oracle, 8 steps, {prec}, K={K} split={split}")
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": K, "graph_steps": 3, "sym_split": split}
    res = []
    for mode in ("push", "graph"):
        with Sim([b], prec, tuning=tun) as sim:
            if mode == "push":
                sim.push(8)
            else:
                sim.step_batched(8, graph=True)
            res.append({k: sim.host(k) for k in ("x", "y", "z", "vx", "vy", "vz")})
    for k in res[0]:
        np.testing.assert_array_equal(res[0][k], res[1][k])
    s = _state(b)
    orc.vv(s, 8)
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    ev = max(np.abs(res[0][k] - getattr(s, k)).max() for k in ("vx", "vy", "vz")) / v_rms
    print(f"    symmetric trajectory: max|dv|/v_rms={ev:.3e}", flush=True)
    assert ev <= (1e-11 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("prec", PRECS)
def test_default_tiling_splits_mid_size_bunches(orc, prec):
    """A 32768-particle bunch has too few block pairs to fill the last wave of
    items unsplit (16-32 blocks): the cost model splits them; at 12288 the
    ordered kernel stays cheaper.  The split default reproduces the field."""
    say(f"default tiling at 12288 and 32768 particles, {prec}")
    with Sim(wl.workload("cold_sphere_1m", n_override=12288), prec) as sim:
        assert sim.tuning()["symmetric"] == 0
    b = wl.workload("cold_sphere_1m", n_override=32768)[0]
    with Sim([b], prec) as sim:
        t = sim.tuning()
        assert t["symmetric"] == 1 and t["sym_split"] > 1, t
        got = gpu_field(sim)
    rng = np.random.default_rng(11)
    recv = np.sort(rng.choice(b.n, 256, replace=False))
    ref = orc.field(b.x, b.y, b.z, b.q, b.weight, b.softening, recv=recv, want_phi=True, want_amag=True,
                    want_pmag=True)
    check_field({k: v[recv] for k, v in got.items()}, ref, TOL[prec], f"default split {prec} n={b.n}")


@pytest.mark.parametrize("prec", PRECS)
def test_symmetric_equals_itself_run_to_run(prec):
    b = wl.workload("cold_sphere_2048")[0]
    say(f"symmetric run-to-run bitwise {prec}")
    outs = []
    for _ in range(2):
        with Sim([b], prec, tuning={"symmetric": 1, "fused": 0, "i_per_lane": 2}) as sim:
            outs.append(gpu_field(sim))
    for k in outs[0]:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])


# ---------------------------------------------------------------------------
# near/far split of the symmetric schedule (spatial sort every evaluation)
# ---------------------------------------------------------------------------

def _far_bunches():
    return [wl.workload("gaussian_65536", n_override=20000)[0],
            wl.workload("cold_sphere_2048", n_override=12289)[0],
            mixed_charge_bunch(6000, seed=8), wl.workload("cold_sphere_2048", n_override=5)[0]]


def _far_bound(f):
    # plain FP32 separations of the high parts change a term by at most this
    # fraction of its magnitude when the boxes are farther apart than U 2^-f
    return 2.0 * math.sqrt(3.0) * 2.0 ** -23 * 2.0 ** f


@pytest.mark.parametrize("K,far,split", [(1, 1, 1), (2, 3, 1), (4, 2, 1), (2, 3, 4)])
def test_far_split_field_parity(orc, K, far, split):
    bunches = _far_bunches()
    say(f"far split field K={K} far={far} split={split} sizes={[b.n for b in bunches]} gap=3")
    base = {"symmetric": 1, "fused": 0, "i_per_lane": K, "sym_split": split}
    with Sim(bunches, "mixed", tuning={**base, "far_split": far}, gap=3) as sim:
        assert sim.tuning()["far_split"] == far
        got_far = gpu_field(sim)
        sim.set_tuning(**base, far_split=0)
        got_near = gpu_field(sim)
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
        mask = np.ones(sim.n_total, bool)
        for sl in slices:
            mask[sl] = False
    assert np.all(got_far["ex"][mask] == 0) and np.all(got_far["phi"][mask] == 0)
    changed = 0
    for k, b in enumerate(bunches):
        sl = slices[k]
        gf = {key: v[sl] for key, v in got_far.items()}
        gn = {key: v[sl] for key, v in got_near.items()}
        ref = oracle_field(orc, b)
        check_field(gf, ref, TOL["mixed"], f"far={far} K={K} n={b.n}")
        # the far path differs from hi/lo by no more than the per-term bound
        d = np.linalg.norm(vec(gf) - vec(gn), axis=1)
        lim = (_far_bound(far) * 1.01 + 1e-7) * ref["amag"]
        assert np.all(d <= lim), (b.n, float((d / ref["amag"]).max()))
        changed += int(np.any(d > 0))
    assert changed >= 1  # the far path ran


@pytest.mark.parametrize("split", [1, 2])
def test_far_split_push_graph_run_to_run_and_trajectory(orc, split):
    b = wl.workload("gaussian_65536", n_override=9000)[0]
    say(f"far split push == step_batched(graph), run-to-run, trajectory vs oracle, 6 steps, split={split}")
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3, "graph_steps": 2, "sym_split": split}
    res = []
    for mode in ("push", "graph", "push"):
        with Sim([b], "mixed", tuning=tun) as sim:
            if mode == "push":
                sim.push(6)
            else:
                sim.step_batched(6, graph=True)
            res.append({k: sim.host(k) for k in ("x", "y", "z", "vx", "vy", "vz")})
    for r in res[1:]:
        for k in res[0]:
            np.testing.assert_array_equal(res[0][k], r[k])
    s = _state(b)
    orc.vv(s, 6)
    v_rms = math.sqrt(np.mean(s.vx ** 2 + s.vy ** 2 + s.vz ** 2))
    ev = max(np.abs(res[0][k] - getattr(s, k)).max() for k in ("vx", "vy", "vz")) / v_rms
    print(f"    far trajectory: max|dv|/v_rms={ev:.3e}", flush=True)
    assert ev <= 1e-6


def test_far_split_tuning_rules():
    b = wl.workload("cold_sphere_2048", n_override=64)[0]
    say("far split tuning validation")
    with Sim([b], "mixed") as sim:
        for bad in ({"symmetric": 0, "fused": 0, "far_split": 2}, {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 5},
                    {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": -1},
                    {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 3},
                    {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 0},
                    {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 0, "sym_split": 8}):
            with pytest.raises(pp.PPError) as e:
                sim.set_tuning(**bad)
            assert e.value.status == pp.PP_ERR_INVALID_ARG
    with Sim([b], "fp64") as sim:
        with pytest.raises(pp.PPError):
            sim.set_tuning(symmetric=1, fused=0, i_per_lane=1, far_split=1)
        sim.set_tuning(symmetric=1, fused=0, i_per_lane=2, far_split=0)   # symmetric FP64 has no far split


def test_autotune_keeps_a_passing_tiling_and_caches_it(orc, tmp_path, monkeypatch):
    """PP_AUTOTUNE times candidate tilings (ordered and symmetric, with and
    without the far split), keeps the fastest one that reproduces the field,
    and stores it; a second context of the same shape reuses the stored one."""
    b = wl.workload("gaussian_65536", n_override=20000)[0]
    cache = tmp_path / "it's a" / "new dir" / "tune.txt"  # created without a shell, quotes and all
    monkeypatch.setenv("PP_TUNE_CACHE", str(cache))
    junk = "not a record\ngfx950:old:format 1 64 22 4 16 0 3 1\n"  # skipped, and must not shift later records
    say(f"autotune mixed n={b.n}, cache {cache}")
    with Sim([b], "mixed") as sim:
        cache.parent.mkdir(parents=True)
        cache.write_text(junk)
        sim.step_batched(2, graph=False, autotune=True)
        tuned = sim.tuning()
        got = gpu_field(sim)
        st = {k: sim.host(k) for k in ("x", "y", "z")}
    print(f"    tuning chosen: {tuned}", flush=True)
    ref = orc.field(st["x"], st["y"], st["z"], b.q, b.weight, b.softening, want_phi=True, want_amag=True,
                    want_pmag=True)
    check_field(got, ref, TOL["mixed"], "autotuned tiling")
    lines = cache.read_text().splitlines()
    assert lines[:2] == junk.splitlines() and len(lines) == 3
    line = lines[2].split()
    assert len(line) == 11 and line[0].startswith("gfx950:")
    assert [int(v) for v in line[1:]] == [tuned[k] for k in ("i_per_lane", "sum_tile", "chunk_pairs_log2",
                                                               "grid_per_cu", "graph_steps", "symmetric",
                                                               "far_split", "sym_split", "fused", "sym_rounds")]
    with Sim([b], "mixed") as sim:
        sim.step_batched(1, graph=False, autotune=True)
        assert sim.tuning() == tuned
    assert len(cache.read_text().splitlines()) == 3  # found in the cache: no second search


def test_autotune_fp64_searches_both_schedules(orc, tmp_path, monkeypatch):
    """On the FP64 path the search covers the ordered kernel and the FP64
    symmetric schedule (1, 2 or 4 receivers per lane, never the far split);
    whatever it keeps reproduces the field within the FP64 tolerance."""
    b = wl.workload("gaussian_65536", n_override=24000)[0]
    monkeypatch.setenv("PP_TUNE_CACHE", str(tmp_path / "tune64.txt"))
    say(f"autotune fp64 n={b.n}")
    with Sim([b], "fp64") as sim:
        sim.step_batched(1, graph=False, autotune=True)
        tuned = sim.tuning()
        got = gpu_field(sim)
        st = {k: sim.host(k) for k in ("x", "y", "z")}
    print(f"    tuning chosen: {tuned}", flush=True)
    assert tuned["far_split"] == 0 and tuned["i_per_lane"] in (1, 2, 4) and tuned["sym_split"] in (1, 2, 4)
    ref = orc.field(st["x"], st["y"], st["z"], b.q, b.weight, b.softening, want_phi=True, want_amag=True,
                    want_pmag=True)
    check_field(got, ref, TOL["fp64"], "autotuned fp64 tiling")
    assert len((tmp_path / "tune64.txt").read_text().splitlines()) == 1


# ---------------------------------------------------------------------------
# the other benchmark workloads at full size, default tilings (as bench.py runs them)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", PRECS)
def test_full_size_parity_gaussian_65536(orc, prec):
    b = wl.workload("gaussian_65536")[0]
    say(f"full size parity gaussian_65536 {prec} n={b.n} (every receiver)")
    with Sim([b], prec) as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        got = gpu_field(sim)
    check_field(got, oracle_field(orc, b), TOL[prec], f"gaussian_65536/{prec}")


def test_full_size_energy_drift_cold_sphere_1m_200_steps():
    """The benchmark's 1 048 576-particle cold sphere in mixed precision with
    its default tiling: over 200 Velocity Verlet steps (hipGraph replay) the
    total energy (the library's own FP64 diagnostics) drifts by at most 1e-6
    of its initial value."""
    b = wl.workload("cold_sphere_1m")[0]
    say(f"energy drift cold_sphere_1m mixed, 200 steps, n={b.n}")
    with Sim([b], "mixed") as sim:
        e0 = sim.diagnostics()[0]["total"]
        sim.step_batched(200, graph=True)
        d = sim.diagnostics()[0]
    drift = abs(d["total"] - e0) / abs(e0)
    print(f"    step {d['step']}: relative energy drift {drift:.3e}", flush=True)
    assert d["step"] == 200
    assert drift <= 1e-6


def test_full_size_sampled_parity_ellipsoid_4m(orc):
    b = wl.workload("ellipsoid_4m")[0]
    rng = np.random.default_rng(98)
    recv = np.sort(rng.choice(b.n, 384, replace=False))
    say(f"full size sampled parity ellipsoid_4m mixed n={b.n}")
    with Sim([b], "mixed") as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        got = gpu_field(sim, sl=recv)
    check_field(got, oracle_field(orc, b, recv=recv), TOL["mixed"], "ellipsoid_4m/mixed sampled")


def test_full_size_sampled_parity_sweep_64(orc):
    bunches = wl.workload("sweep_64")
    rng = np.random.default_rng(97)
    say(f"full size sampled parity sweep_64 mixed: {len(bunches)} bunches, {sum(b.n for b in bunches)} particles")
    with Sim(bunches, "mixed") as sim:
        print(f"    tuning {sim.tuning()}", flush=True)
        full = gpu_field(sim)
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
    worst = (0.0, 0.0)
    for k, b in enumerate(bunches):
        recv = np.sort(rng.choice(b.n, 16, replace=False))
        got = {key: v[slices[k]][recv] for key, v in full.items()}
        ref = oracle_field(orc, b, recv=recv)
        G, R = vec(got), vec(ref)
        e = (l2_rel(G, R), cond_max(G, R, ref["amag"]))
        worst = (max(worst[0], e[0]), max(worst[1], e[1]))
        assert e[0] <= TOL["mixed"] and e[1] <= TOL["mixed"], (k, b.n, e)
        assert l2_rel(got["phi"], ref["phi"]) <= TOL["mixed"], k
        assert phi_cond_max(got["phi"], ref["phi"], ref["pmag"]) <= TOL["mixed"], k
    print(f"    sweep_64 worst over bunches: l2={worst[0]:.3e} cond_max={worst[1]:.3e}", flush=True)


@pytest.mark.parametrize("variant", ["ordered", "symmetric_far"])
def test_graph_replays_match_eager_steps_one_by_one(variant):
    """Several replays of one captured step graph, with eager work (field
    evaluations, host copies, synchronisations) between them: after every
    replay the state equals that of a twin context stepped without graphs."""
    tun = {"graph_steps": 4}
    if variant == "symmetric_far":
        tun.update({"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3})
    b = wl.workload("gaussian_65536", n_override=5000)[0]
    say(f"graph replays one by one ({variant})")
    with Sim([b], "mixed", tuning=tun) as g, Sim([b], "mixed", tuning=tun) as e:
        for rep in range(4):
            g.step_batched(4, graph=True)
            e.push(4)
            g.field(want_phi=True)  # eager work on the graph's context between replays
            g.sync()
            for k in ("x", "vx", "z", "vz"):
                np.testing.assert_array_equal(g.host(k), e.host(k), err_msg=f"replay {rep} {k}")


def test_far_split_order_reuse_matches_one_step_pushes():
    """The far split's Morton order is recomputed at steps that are multiples
    of 8 and reused in between.  Graph replays of 3 steps (every phase of the
    rule), diagnostics and field evaluations between calls, and an
    invalidation at a step that is not a multiple of 8 must give the bits of a
    twin context advanced by one-step pushes with the same invalidation."""
    tun = {"graph_steps": 3, "symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3}
    b = wl.workload("gaussian_65536", n_override=6000)[0]
    say("far split order reuse vs one-step pushes (graphs of 3, diagnostics, invalidation at step 5)")
    with Sim([b], "mixed", tuning=tun) as g, Sim([b], "mixed", tuning=tun) as e:
        g.step_batched(5, graph=True)
        g.diagnostics()
        g.field(want_phi=True)
        for _ in range(5):
            e.push(1)
        g.invalidate()
        e.invalidate()
        g.step_batched(13, graph=True)  # eager to step 8, graphs from phases 0, 3, 6, then eager
        g.diagnostics()
        g.step_batched(7, graph=False)
        for _ in range(20):
            e.push(1)
        for k in ("x", "y", "vx", "vz"):
            np.testing.assert_array_equal(g.host(k), e.host(k), err_msg=k)


TWO_BODY_TOL = {"fp64": 2e-15, "mixed": 1e-6}


@pytest.mark.parametrize("prec,sched", [("fp64", "ordered"), ("fp64", "symmetric"), ("mixed", "ordered"),
                                        ("mixed", "symmetric")])
def test_two_body_closed_form_over_eleven_decades(prec, sched):
    """Independent of the oracle: 32 two-particle bunches with separations from
    1e-9 m to 100 m along a skew direction, no softening.  Each particle's
    field must be k w q (r_i - r_j) / |r_i - r_j|^3 (Eq. (A)/(B) for one pair),
    evaluated here in 40-digit decimal arithmetic from the same doubles: FP64
    to within 2e-15 relative (v_rsq_f64 alone is good to ~2^-24 and one Newton
    step to ~4e-15, so either shortcut would fail), mixed to within 1e-6 (FP32
    pair arithmetic on hi/lo separations)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 40
    pi = Decimal("3.141592653589793238462643383279502884197")
    k = 1 / (4 * pi * Decimal(repr(wl.EPS0)))
    bunches, expect = [], []
    for i in range(32):
        d = 10.0 ** (-9 + 11 * i / 31)
        x = np.array([0.0, d / 3]); y = np.array([0.0, 2 * d / 3]); z = np.array([0.0, -2 * d / 3])
        q = np.full(2, -wl.E_CHARGE); m = np.full(2, wl.M_ELECTRON); zero = np.zeros(2)
        w = 7.0
        bunches.append(wl.Bunch(x, y, z, zero, zero.copy(), zero.copy(), q, m, w, 0.0, 1e-15, 0, {}))
        dx, dy, dz = (Decimal(repr(float(a[0]))) - Decimal(repr(float(a[1]))) for a in (x, y, z))
        r = (dx * dx + dy * dy + dz * dz).sqrt()
        f = k * Decimal(repr(w)) * Decimal(repr(-wl.E_CHARGE)) / (r * r * r)
        expect.append([float(f * dx), float(f * dy), float(f * dz)])  # on particle 0; particle 1 opposite
    tun = ORDERED_TUNING if sched == "ordered" else {"symmetric": 1, "fused": 0, "i_per_lane": 1}
    say(f"{prec} two-body closed form, 32 separations 1e-9..1e2 m ({sched})")
    with Sim(bunches, prec, tuning=tun) as sim:
        f = gpu_field(sim)
        worst = 0.0
        for i in range(len(bunches)):
            sl = sim.bunch_slice(i)
            g = np.stack([f["ex"][sl], f["ey"][sl], f["ez"][sl]], 1)
            e = np.array(expect[i])
            for row, sign in ((0, 1.0), (1, -1.0)):
                rel = np.abs(g[row] - sign * e).max() / np.abs(e).max()
                worst = max(worst, rel)
                assert rel <= TWO_BODY_TOL[prec], (i, row, g[row], sign * e, rel)
    print(f"    worst relative error {worst:.3e}", flush=True)


def test_time_field_and_profile_leave_the_run_unchanged():
    """pp_time_field returns a positive time and the ordered pair count, and
    neither it nor the event profiling changes a run's bits: 3 steps, a timed
    field, 3 more steps with profiling on equal 6 plain steps (far split on,
    so the order-reuse rule is exercised too)."""
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "far_split": 3}
    b = wl.workload("gaussian_65536", n_override=5000)[0]
    say("pp_time_field and profiling leave the trajectory unchanged")
    with Sim([b], "mixed", tuning=tun) as t, Sim([b], "mixed", tuning=tun) as e:
        t.push(3)
        with t._on():
            ms, pairs = pp.pp_time_field(t.ctx, 2)
            pp.pp_set_profiling(t.ctx, True)
        assert ms > 0.0 and pairs == float(b.n) * (b.n - 1)
        t.push(3)
        with t._on():
            prof = pp.pp_get_profile(t.ctx)
            pp.pp_set_profiling(t.ctx, False)
        assert prof["evaluations"] == 3 and prof["launches"] >= 3 and prof["total_ms"] > 0.0
        assert prof["pairs"] == pairs
        e.push(6)
        for k in ("x", "vx", "vz"):
            np.testing.assert_array_equal(t.host(k), e.host(k), err_msg=k)


def test_simulation_calls_under_another_current_stream(orc, gpu):
    """The wrapper runs every call on its context's stream: a caller whose
    current torch stream is another one still gets the right field (the output
    tensors are zero-filled on the context's stream, ahead of the kernels)."""
    torch = gpu
    b = wl.workload("cold_sphere_2048")[0]
    say("field with another torch stream current")
    with Sim([b], "mixed") as sim:
        other = torch.cuda.Stream()
        with torch.cuda.stream(other):
            f = sim.field(want_phi=True)
            sim.push(2)
            sim.sync()
            got = {k: v.cpu().numpy() for k, v in f.items()}
    check_field(got, oracle_field(orc, b), TOL["mixed"], "under another stream")


# ---------------------------------------------------------------------------
# several rounds per symmetric item (tuning field sym_rounds)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec,M,n", [("mixed", 2, 70000), ("mixed", 4, 140000), ("fp64", 4, 140000),
                                      ("fp64", 8, 270000)])
def test_sym_rounds_field_parity(orc, prec, M, n):
    """Items sweeping M consecutive rounds (one receiver-side partial per
    group of rounds): a large bunch with at least 128 M blocks at one receiver
    per lane, so groups of M rounds apply (70000 particles: 274 blocks;
    140000: 547; 270000: 1055), a small one that keeps one round per item,
    and a 5-particle one in one batch; sampled receivers of the large bunch
    and every receiver of the others against the oracle."""
    big = wl.workload("gaussian_65536", n_override=n)[0]
    bunches = [big, wl.workload("cold_sphere_2048", n_override=3000)[0],
               wl.workload("cold_sphere_2048", n_override=5)[0]]
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "sym_split": 1, "sym_rounds": M,
           "far_split": 3 if prec == "mixed" else 0}
    say(f"sym_rounds={M} field {prec} sizes={[b.n for b in bunches]}")
    rng = np.random.default_rng(31)
    recv = np.sort(rng.choice(big.n, 256, replace=False))
    with Sim(bunches, prec, tuning=tun) as sim:
        assert sim.tuning()["sym_rounds"] == M
        full = gpu_field(sim)
        slices = [sim.bunch_slice(k) for k in range(len(bunches))]
    got = {key: v[slices[0]][recv] for key, v in full.items()}
    check_field(got, oracle_field(orc, big, recv=recv), TOL[prec], f"sym_rounds={M} n={big.n} sampled")
    for k, b in enumerate(bunches[1:], start=1):
        check_field({key: v[slices[k]] for key, v in full.items()}, oracle_field(orc, b), TOL[prec],
                    f"sym_rounds={M} n={b.n}")


@pytest.mark.parametrize("prec", PRECS)
def test_sym_rounds_bitwise_equivalences(prec):
    """With up to 4 rounds per item (2 for the 274-block bunch): push ==
    step_batched with graphs, and a batch (one bunch with the groups, one
    without) equals the bunches alone."""
    bunches = [wl.workload("gaussian_65536", n_override=70000)[0], wl.workload("gaussian_65536", n_override=2500)[0]]
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 1, "sym_split": 1, "sym_rounds": 4, "graph_steps": 2,
           "far_split": 3 if prec == "mixed" else 0}
    say(f"sym_rounds=4 push == graph, batch == alone, {prec}")
    res = []
    for mode in ("push", "graph"):
        with Sim(bunches, prec, tuning=tun) as sim:
            if mode == "push":
                sim.push(4)
            else:
                sim.step_batched(4, graph=True)
            res.append([np.concatenate([sim.host(k)[sim.bunch_slice(i)] for k in ("x", "vx", "vz")])
                        for i in range(len(bunches))])
    for i in range(len(bunches)):
        np.testing.assert_array_equal(res[0][i], res[1][i])
        with Sim([bunches[i]], prec, tuning=tun) as one:
            one.push(4)
            alone = np.concatenate([one.host(k) for k in ("x", "vx", "vz")])
        np.testing.assert_array_equal(res[0][i], alone)


@pytest.mark.parametrize("prec", PRECS)
def test_sym_rounds_with_split_and_bands_sampled_parity_1m(orc, prec):
    """8 rounds per item at 1 048 576 particles with block pairs split in 2:
    the groups of rounds line up with the slot bands (3 mixed, 6 FP64)."""
    b = wl.workload("cold_sphere_1m")[0]
    rng = np.random.default_rng(97)
    recv = np.sort(rng.choice(b.n, 256, replace=False))
    tun = {"symmetric": 1, "fused": 0, "i_per_lane": 4, "sym_split": 2, "sym_rounds": 8,
           "far_split": 3 if prec == "mixed" else 0}
    say(f"sym_rounds=8 split 2 with slot bands, cold_sphere_1m {prec}")
    with Sim([b], prec, tuning=tun) as sim:
        got = gpu_field(sim, sl=recv)
    check_field(got, oracle_field(orc, b, recv=recv), TOL[prec], f"cold_sphere_1m/{prec} sym_rounds 8 split 2")
