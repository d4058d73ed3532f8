"""Benchmark of the PP hot path on one MI355X.

One step = one Velocity Verlet step of the whole path (drift + pack, the
persistent pair-sum kernel over every pair, chunk combine + kick) through
pp_step_batched.  Default workload: the 1 048 576-particle cold uniform sphere
(R = 200 um, 1e10 electrons, eps = 5e-4 spacing, dt = 0.005/omega_p) in mixed
precision (FP32 pair arithmetic on hi/lo positions with two-sum tile
accumulation, FP64 push).  Inputs are resident in HBM before timing starts.

Prints one JSON line:
  value      ordered pair interactions per second over the timed steps
  roofline   the pair-sum kernel's achieved FP32 rate in algorithmic flops (20
             per ordered pair, the usual count for a softened inverse-square
             interaction) over its average duration, measured with HIP events
             on the stream it runs on, against the 157.3 TFLOP/s FP32 vector
             peak of the MI355X (the FP64 path: its FP64 rate against the 78.6
             TFLOP/s FP64 peak).  The symmetric kernel evaluates each unordered
             pair once for two ordered interactions (Newton's third law), so
             its algorithmic rate counts work it did not have to issue; for it
             the fraction of the FP32 vector peak the hardware actually
             delivered is counted_frac: the FP32 flops rocprofv3 counted for
             the same kernel, workload, tiling and sources
             (SQ_INSTS_VALU_FLOPS_FP32, stored beside the profile under
             profiles/), over the same measured duration.  counted_frac and
             counted_tflops are null when no stored count matches.
  cpu_baseline  the CPU oracle on a bounded sample of the same field evaluation
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 20
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
COUNTERS = os.path.join(ROOT, "profiles", "pair_sym_cold_sphere_1m_counters.json")


TUNING_KEYS = ("symmetric", "i_per_lane", "far_split", "sym_split", "fused", "sym_rounds")


def stored_counters(workload, kernel, tuning):
    """Hardware-counter figures measured for this kernel, workload and tiling
    (see profiles/), used only while the kernel sources still hash to the
    value recorded with them."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    rec = json.load(open(COUNTERS))
    if rec.get("workload") != workload or not rec.get("kernel", "").startswith(kernel):
        return None
    want = rec.get("tuning")
    if not want or any(want.get(k) != tuning.get(k) for k in TUNING_KEYS):
        return None
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in rec["sources"])).hexdigest()[:16]
    return rec if h == rec.get("source_sha256_16") else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="cold_sphere_1m")
    p.add_argument("--n", type=int, default=0, help="override the particle count")
    p.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    p.add_argument("--graph", action="store_true", help="replay steps from hipGraphs (no per-kernel timing)")
    p.add_argument("--autotune", action="store_true")
    p.add_argument("--tuning", default="", help="k=v,... tiling override (i_per_lane, sum_tile, ...)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU time of the oracle sample")
    p.add_argument("--cpu-threads", type=int, default=0,
                   help="oracle threads for --mode oracle (0: every host core)")
    p.add_argument("--sizes", default="12288,16384,24576,32768,49152,65536,98304,131072",
                   help="particle counts for --mode tilings")
    p.add_argument("--mode", default="throughput",
                   choices=["throughput", "drift", "paper", "oracle", "tilings", "steps", "ubench"],
                   help="drift: run --steps steps in mixed and FP64 precision and report the total-energy drift "
                        "and the mixed-vs-FP64 energy gap every --every steps (no timing line); paper: the "
                        "paper's own cube-lattice runs to 10 ns with the emittance series (--paper-cases); "
                        "oracle: time only the CPU oracle on --cpu-threads threads (no GPU); tilings: pair-stage time of "
                        "the default tiling against the ordered kernel and the unsplit symmetric ones at --sizes; "
                        "steps: per-step time (graph replay) of the default, the ordered and the fused tilings at "
                        "--sizes; ubench: vector-ALU issue rates per clock per CU (micro-benchmarks)")
    p.add_argument("--paper-cases", default="main,dt,np,pic,long",
                   help="subset of main,dt,np,pic,long for --mode paper")
    p.add_argument("--every", type=int, default=20)
    p.add_argument("--precisions", default="mixed,fp64")
    p.add_argument("--calibrate-copy-mib", type=int, default=0,
                   help="only run a plain device-to-device copy of this many MiB (3 times) and exit: the "
                        "reference for scaling the FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def calibrate_copy(mib):
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4,
                      "copies": 3}))


def cpu_baseline(bunches, target_s, threads=0):
    """Time the CPU oracle's field evaluation on a bounded sample of receivers
    of the first bunch (every source), scaled to pairs/s; on every host core
    unless ``threads`` names a count."""
    import numpy as np
    from oracle.oracle import default
    orc = default()
    if threads:
        orc.set_num_threads(threads)
    b = bunches[0]
    rng = np.random.default_rng(7)
    nrecv = 256
    while True:
        recv = np.sort(rng.choice(b.n, min(nrecv, b.n), replace=False))
        t0 = time.perf_counter()
        orc.field(b.x, b.y, b.z, b.q, b.weight, b.softening, recv=recv)
        dt = time.perf_counter() - t0
        if dt >= target_s or nrecv >= b.n:
            break
        nrecv = min(b.n, int(nrecv * max(2.0, 1.2 * target_s / max(dt, 1e-3))))
    pairs = recv.size * (b.n - 1)
    return {"value": pairs / dt, "unit": "pair interactions/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{recv.size} receivers x {b.n} sources of {b.meta.get('name', 'bunch')}, one FP64 field "
                      f"evaluation with compensated sums ({pairs:.3e} pairs in {dt:.2f} s)"}


def oracle_only(a):
    """The CPU oracle alone on the workload's first bunch (no GPU is touched):
    the host-side reference rate, serial with --cpu-threads 1."""
    from paper_2502_10640_amd import workloads as wl
    bunches = wl.workload(a.workload, n_override=a.n or None)
    base = cpu_baseline(bunches, a.cpu_seconds, a.cpu_threads)
    print(json.dumps({"metric": "pair interactions/s (CPU oracle)", "value": base["value"],
                      "unit": base["unit"], "cpu_baseline": base,
                      "config": {"workload": a.workload, "n": bunches[0].n}}))


def tilings(a):
    """Pair-stage time per field evaluation (pp_time_field: sort, pair kernel
    and fold, HIP events) of the default tiling and of the ordered kernel and
    the unsplit symmetric tilings, for --workload at each of --sizes.  Each
    context is warmed first; every case is timed twice, the minimum kept."""
    from paper_2502_10640_amd import pp
    from paper_2502_10640_amd import workloads as wl
    from paper_2502_10640_amd.sim import Simulation
    for prec in a.precisions.split(","):
        for n in (int(x) for x in a.sizes.split(",")):
            bunches = wl.workload(a.workload, n_override=n)
            with Simulation(bunches, prec) as sim:
                d = sim.tuning()
                reps = max(3, min(50, int(4e10 / n ** 2)))
                pp.pp_time_field(sim.ctx, 3 * reps)
                cands = [("default", d),
                         ("ordered", {**d, "symmetric": 0, "fused": 0, "far_split": 0, "sym_split": 1,
                                      "i_per_lane": 2 if (prec == "mixed" and n >= 16384) else 1})]
                for k in (2, 4):
                    cands.append((f"symmetric K={k} split 1", {**d, "symmetric": 1, "fused": 0, "i_per_lane": k, "sym_split": 1,
                                                                "far_split": 3 if prec == "mixed" else 0}))
                best = {}
                for _ in range(2):
                    for name, t in cands:
                        sim.set_tuning(**t)
                        pp.pp_time_field(sim.ctx, 2)
                        ms, _ = pp.pp_time_field(sim.ctx, reps)
                        best[name] = min(best.get(name, float("inf")), ms)
            print(json.dumps({"mode": "tilings", "workload": a.workload, "precision": prec, "n": n,
                              "default_tuning": {k: d[k] for k in ("symmetric", "i_per_lane", "sym_split", "far_split")},
                              "pair_stage_ms": best}), flush=True)


UBENCH_OPS = {  # name: (op code, lane operations per chain-iteration, iterations)
    "fma_f32": (0, 1, 400000), "add_f32": (1, 1, 400000), "mul_f32": (2, 1, 400000),
    "rsq_f32": (3, 1, 100000), "fma8_rsq_f32": (4, 9, 40000), "fma_f64": (5, 1, 200000),
    "add_f64": (6, 1, 200000), "mul_f64": (7, 1, 200000), "rsq_f64": (8, 1, 50000)}


def ubench(a):
    """Vector-ALU issue rates of gfx950 (libpp_ubench.so): lane operations per
    shader clock per compute unit for FP32 FMA, add, mul, v_rsq_f32, 8 FMA
    interleaved with one rsq, and FP64 FMA, add, mul and v_rsq_f64.  8 workgroups of 256 threads per
    CU, 8 independent chains per thread; the clock is measured inside the
    kernel (shader-clock counter against the wall clock)."""
    import ctypes
    import torch
    from paper_2502_10640_amd.build import UBENCH_PATH
    L = ctypes.CDLL(UBENCH_PATH)
    L.pp_ubench_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    L.pp_ubench_valu.restype = ctypes.c_int
    L.pp_ubench_wall_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int)]
    L.pp_ubench_wall_clock_khz.restype = ctypes.c_int
    khz = ctypes.c_int(0)
    assert L.pp_ubench_wall_clock_khz(ctypes.byref(khz)) == 0
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 8 * cus
    inp = torch.rand(1024, device="cuda")
    out = torch.empty(blocks * 256, device="cuda")
    clk = torch.zeros(2 * blocks, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    res = {"mode": "ubench", "cus": cus, "wall_clock_khz": khz.value, "blocks": blocks, "threads_per_block": 256,
           "chains_per_thread": 8, "ops": {}}
    for name, (op, per, iters) in UBENCH_OPS.items():
        ms = ctypes.c_double(0.0)
        for it in (max(1, iters // 50), iters):  # warm-up, then the measured run
            rc = L.pp_ubench_valu(op, blocks, it, inp.data_ptr(), out.data_ptr(), clk.data_ptr(), ctypes.byref(ms))
            assert rc == 0, (name, rc)
        c = clk.cpu().numpy()
        cycles, ticks = float(c[0::2].mean()), float(c[1::2].mean())
        clock_hz = cycles / ticks * khz.value * 1e3
        lane_ops = blocks * 256 * 8 * iters * per
        res["ops"][name] = {"ms": ms.value, "lane_ops": lane_ops, "clock_ghz": clock_hz / 1e9,
                            "lane_ops_per_clock_per_cu": lane_ops / (cus * ms.value * 1e-3 * clock_hz),
                            "lane_ops_per_block_span_per_cu": lane_ops / (cus * cycles)}
        print(f"[ubench] {name}: {res['ops'][name]['lane_ops_per_clock_per_cu']:.1f} lane-ops/clock/CU "
              f"at {clock_hz / 1e9:.2f} GHz", file=sys.stderr, flush=True)
    print(json.dumps(res))


def step_times(a):
    """Per-step time (hipGraph replay) of the default tiling and of the
    schedules that compete for small bunches -- the two-kernel ordered step,
    and the fused step at 4..32 receivers per workgroup of 512 threads --
    for --workload at each of --sizes.  Best of two timed runs; prints one
    JSON line per precision and size."""
    import torch
    from paper_2502_10640_amd import workloads as wl
    from paper_2502_10640_amd.sim import Simulation
    cands = [("default", {}), ("ordered", {"symmetric": 0, "fused": 0, "far_split": 0, "sym_split": 1, "i_per_lane": 1})]
    for r in (4, 8, 16, 32):
        cands.append((f"fused R={r}", {"symmetric": 0, "fused": r, "far_split": 0, "sym_split": 1, "i_per_lane": 2}))
    for prec in a.precisions.split(","):
        for n in (int(x) for x in a.sizes.split(",")):
            bunches = wl.workload(a.workload, n_override=n)
            total = sum(b.n for b in bunches)
            steps = max(50, min(2000, int(2e10 / total ** 2)))
            res, default = {}, None
            for name, tun in cands:
                with Simulation(bunches, prec, tuning={**tun, "graph_steps": 50}) as sim:
                    if default is None:
                        default = {k: v for k, v in sim.tuning().items() if k != "graph_steps"}
                    sim.step_batched(50, graph=True)
                    torch.cuda.synchronize()
                    best = float("inf")
                    for _ in range(2):
                        t0 = time.perf_counter()
                        sim.step_batched(steps, graph=True)
                        torch.cuda.synchronize()
                        best = min(best, (time.perf_counter() - t0) / steps * 1e6)
                res[name] = round(best, 2)
            print(json.dumps({"mode": "steps", "workload": a.workload, "precision": prec, "n": total,
                              "steps": steps, "default_tuning": default, "us_per_step": res}), flush=True)


def total_energy(sim):
    """Total energy per bunch (kinetic + softened potential, Sec. 2.2) from
    pp_diagnostics: the library's FP64 reductions on the device."""
    return [d["total"] for d in sim.diagnostics()]


def drift(a):
    import numpy as np
    import torch
    from paper_2502_10640_amd import workloads as wl
    from paper_2502_10640_amd.sim import Simulation
    bunches = wl.workload(a.workload, n_override=a.n or None)
    traj = {}
    wall = {}
    for prec in a.precisions.split(","):
        print(f"[drift] {a.workload} {prec} {a.steps} steps", file=sys.stderr, flush=True)
        with Simulation(bunches, prec) as sim:
            es = [total_energy(sim)]
            t_run = 0.0
            done = 0
            while done < a.steps:
                k = min(a.every, a.steps - done)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step_batched(k, graph=False)
                torch.cuda.synchronize()
                t_run += time.perf_counter() - t0
                done += k
                es.append(total_energy(sim))
                print(f"[drift] {prec} step {done}", file=sys.stderr, flush=True)
            traj[prec] = np.array(es)
            wall[prec] = t_run
    pairs = float(sum(b.n * (b.n - 1) for b in bunches))
    out = {"mode": "drift", "workload": a.workload, "n_particles": sum(b.n for b in bunches), "steps": a.steps,
           "every": a.every, "dt_omega": [b.meta.get("dt_omega") for b in bunches][:4]}
    for prec, e in traj.items():
        e0 = np.abs(e[0])
        out[f"max_rel_drift_{prec}"] = float(np.max(np.abs(e - e[0]) / e0))
        out[f"final_rel_drift_{prec}"] = float(np.max(np.abs(e[-1] - e[0]) / e0))
        out[f"pairs_per_s_{prec}"] = a.steps * pairs / wall[prec]
    if "mixed" in traj and "fp64" in traj:
        gap = np.abs(traj["mixed"] - traj["fp64"]) / np.abs(traj["fp64"][0])
        out["max_rel_gap_mixed_vs_fp64"] = float(np.max(gap))
    print(json.dumps(out))


PAPER_T_END = 1e-8  # every case of the paper's PP study runs to 10 ns (Sec. 2.2)
PAPER_WALL_S = 532.0  # the paper's time for its 16^3 case, 100 000 steps, 64 EPYC 9174F threads


def run_series(sim, n_steps, every):
    """Step n_steps (hipGraph replay) with diagnostics every `every` steps;
    returns the wall time of the stepping alone and the per-bunch series.
    The context's graphs should be long (paper_tuning): each replay costs
    ~10 us of launch gap, 3% of a step of the 4096-particle cube at 16 steps
    per graph."""
    import torch
    series = [[] for _ in sim.bunches]

    def record():
        for k, d in enumerate(sim.diagnostics()):
            series[k].append((d["time"], d["emittance"][0], d["x_rms"][0], d["total"], d["x_max"][0],
                              d["v_rms"][0], d["v_max"][0]))

    record()
    t_run, done = 0.0, 0
    while done < n_steps:
        k = min(every, n_steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step_batched(k, graph=True)
        torch.cuda.synchronize()
        t_run += time.perf_counter() - t0
        done += k
        record()
    return t_run, series


def paper_tuning(every):
    """hipGraphs of up to 200 steps (a multiple of the far split's 8-step
    resort cadence), or one diagnostics interval if that is shorter: longer
    graphs save little more and cost more to instantiate."""
    return {"graph_steps": max(1, min(200, every))}


# The PP runs of the paper's PIC comparison: the 8^3 = 512-particle cube at
# dt = 1e-12 s, 100 steps (Sec. 3.2) and to 3200 ps (Sec. 3.3), with the
# paper's serial wall times (other hardware; context, not a target).
PAPER_512 = {"pic": {"steps": 100, "every": 10, "paper_serial_s": 0.28},
             "long": {"steps": 3200, "every": 100, "paper_serial_s": 23.0}}


def cpu_baseline_vv(b, n_steps):
    """The CPU oracle's Velocity Verlet run of one bunch (trajectory only, no
    diagnostics), timed on one thread and on every host core."""
    from oracle.oracle import OracleState, default
    orc = default()
    every_core = orc.num_threads()
    out = {"kind": "oracle", "steps": n_steps, "n": b.n,
           "pairs": float(b.n) * (b.n - 1) * (n_steps + 1)}
    try:
        for label, nt in (("serial", 1), ("all_cores", every_core)):
            orc.set_num_threads(nt)
            s = OracleState(b.x, b.y, b.z, b.vx, b.vy, b.vz, b.q, b.m, b.weight, b.softening, b.dt)
            t0 = time.perf_counter()
            orc.vv(s, n_steps)
            out[f"{label}_s"] = time.perf_counter() - t0
            out[f"{label}_cores"] = nt
    finally:
        orc.set_num_threads(every_core)
    return out


def paper(a):
    """The paper's own PP runs: the 16^3 cube lattice to 10 ns at dt = 1e-13 s,
    the time-step sweep {1e-13 .. 1e-10} s and the macro-particle sweep
    {4^3 .. 32^3} (one batch) of Sec. 2.2, with the emittance of Eq. (I)
    sampled every 0.1 ns; the 512-particle PP runs of the PIC comparison
    (Sec. 3.2: 100 steps of 1 ps; Sec. 3.3: to 3200 ps) with the observables
    Sec. 3.2 plots, in both precisions, beside the serial CPU oracle on the
    same runs.  Prints one JSON line."""
    import numpy as np
    from paper_2502_10640_amd import workloads as wl
    from paper_2502_10640_amd.sim import Simulation
    out = {"mode": "paper", "t_end_s": PAPER_T_END, "sample_every_s": 1e-10, "cases": {}}

    def summary(bunches, prec, dt, series, t_run, n_steps):
        pairs = float(sum(b.n * (b.n - 1) for b in bunches)) * n_steps
        res = {"precision": prec, "dt_s": dt, "steps": n_steps, "n_particles": [b.n for b in bunches],
               "wall_s": t_run, "pairs_per_s": pairs / t_run, "emittance_x": [], "x_rms": [], "x_max": [],
               "v_rms": [], "v_max": []}
        for k in range(len(bunches)):
            ser = np.array(series[k])
            e0 = ser[0, 3]
            for col, key in ((1, "emittance_x"), (2, "x_rms"), (4, "x_max"), (5, "v_rms"), (6, "v_max")):
                res[key].append([float(v) for v in ser[:, col]])
            res.setdefault("max_rel_energy_drift", []).append(float(np.max(np.abs(ser[:, 3] - e0)) / abs(e0)))
        return res

    cases = a.paper_cases.split(",")
    if "main" in cases:
        for prec in ("mixed", "fp64"):
            b = wl.paper_cube(16)
            n_steps = int(round(PAPER_T_END / b.dt))
            print(f"[paper] 16^3 {prec}: {n_steps} steps", file=sys.stderr, flush=True)
            every = int(round(1e-10 / b.dt))
            with Simulation([b], prec, tuning=paper_tuning(every)) as sim:
                t_run, ser = run_series(sim, n_steps, every)
            out["cases"][f"main_{prec}"] = summary([b], prec, b.dt, ser, t_run, n_steps)
        m, f = out["cases"]["main_mixed"], out["cases"]["main_fp64"]
        em, ef = np.array(m["emittance_x"][0]), np.array(f["emittance_x"][0])
        out["main_emittance_mixed_vs_fp64_max_rel"] = float(np.max(np.abs(em - ef)[1:] / np.abs(ef[1:])))
        out["main_speedup_vs_paper_wall"] = PAPER_WALL_S / m["wall_s"]
    if "dt" in cases:
        for dt in (1e-12, 1e-11, 1e-10):
            b = wl.paper_cube(16, dt=dt)
            n_steps = int(round(PAPER_T_END / dt))
            print(f"[paper] dt sweep dt={dt:g}: {n_steps} steps", file=sys.stderr, flush=True)
            every = max(1, int(round(1e-10 / dt)))
            with Simulation([b], "mixed", tuning=paper_tuning(every)) as sim:
                t_run, ser = run_series(sim, n_steps, every)
            out["cases"][f"dt_{dt:g}"] = summary([b], "mixed", dt, ser, t_run, n_steps)
    if "np" in cases:
        bunches = wl.workload("paper_np_batch")
        n_steps = int(round(PAPER_T_END / bunches[0].dt))
        print(f"[paper] N_p sweep as one batch: {n_steps} steps", file=sys.stderr, flush=True)
        every = int(round(1e-10 / bunches[0].dt))
        with Simulation(bunches, "mixed", tuning=paper_tuning(every)) as sim:
            t_run, ser = run_series(sim, n_steps, every)
        out["cases"]["np_batch"] = summary(bunches, "mixed", bunches[0].dt, ser, t_run, n_steps)
    for case, spec in PAPER_512.items():
        if case not in cases:
            continue
        b = wl.paper_cube(8, dt=1e-12)
        for prec in ("mixed", "fp64"):
            print(f"[paper] 8^3 at dt = 1e-12 s, {spec['steps']} steps, {prec}", file=sys.stderr, flush=True)
            with Simulation([b], prec, tuning=paper_tuning(spec["every"])) as sim:
                t_run, ser = run_series(sim, spec["steps"], spec["every"])
            res = summary([b], prec, b.dt, ser, t_run, spec["steps"])
            res["paper_serial_wall_s"] = spec["paper_serial_s"]
            out["cases"][f"{case}_{prec}"] = res
        print(f"[paper] 8^3, {spec['steps']} steps: CPU oracle", file=sys.stderr, flush=True)
        out["cases"][f"{case}_oracle"] = cpu_baseline_vv(b, spec["steps"])
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}): the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    if a.mode == "drift":
        drift(a)
        return
    if a.mode == "paper":
        paper(a)
        return
    if a.mode == "oracle":
        oracle_only(a)
        return
    if a.mode == "tilings":
        tilings(a)
        return
    if a.mode == "ubench":
        ubench(a)
        return
    if a.mode == "steps":
        step_times(a)
        return
    if a.calibrate_copy_mib:
        calibrate_copy(a.calibrate_copy_mib)
        return
    import torch
    from paper_2502_10640_amd import pp
    from paper_2502_10640_amd import workloads as wl
    from paper_2502_10640_amd.sim import Simulation

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    bunches = wl.workload(a.workload, n_override=a.n or None)
    pairs = float(sum(b.n * (b.n - 1) for b in bunches))
    tuning = {}
    if a.tuning:
        for kv in a.tuning.split(","):
            k, v = kv.split("=")
            tuning[k] = int(v)
    print(f"[bench] workload={a.workload} n={sum(b.n for b in bunches)} bunches={len(bunches)} "
          f"precision={a.precision}", file=sys.stderr, flush=True)
    sim = Simulation(bunches, a.precision, tuning=tuning or None)
    sim.step_batched(a.warmup, graph=a.graph, autotune=a.autotune)
    torch.cuda.synchronize()
    print(f"[bench] warmup done, tuning={sim.tuning()}", file=sys.stderr, flush=True)
    pp.pp_set_profiling(sim.ctx, True)
    pp.pp_get_profile(sim.ctx)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_batched(a.steps, graph=a.graph)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pp.pp_get_profile(sim.ctx)
    pp.pp_set_profiling(sim.ctx, False)
    wall = t1 - t0
    value = a.steps * pairs / wall
    print(f"[bench] {a.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    used_tuning = sim.tuning()
    sym = used_tuning.get("symmetric", 0) == 1
    if sym:
        kernel = "pair_sym_kernel" if a.precision == "mixed" else "pair_sym64_kernel"
    elif used_tuning.get("fused", 0):
        kernel = "fused_kernel"  # the whole evaluation and its update in one kernel
    else:
        kernel = f"pair_{a.precision}_kernel"
    peak = PEAK_FP32_TFLOPS if a.precision == "mixed" else PEAK_FP64_TFLOPS
    roofline = None
    if prof["launches"] > 0 and prof["evaluations"] > 0:
        # pair-kernel time per field evaluation: the sum of its dispatches (one
        # persistent dispatch, or one per band of rounds of the symmetric
        # schedule), timed with HIP events on the stream they run on
        eval_s = prof["total_ms"] / prof["evaluations"] * 1e-3
        achieved = FLOPS_PER_PAIR * pairs / eval_s / 1e12
        roofline = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": None,
                    "frac_kind": ("algorithmic: 20 flops per ordered pair; the symmetric kernel evaluates each "
                                  "unordered pair once for two ordered interactions" if sym else
                                  "algorithmic: 20 flops per ordered pair"),
                    "counted_frac": None, "counted_tflops": None, "counted_source": None,
                    "kernel": kernel, "kernel_ms_per_evaluation": eval_s * 1e3,
                    "launches_per_evaluation": prof["launches"] / prof["evaluations"],
                    "avg_launch_ms": prof["total_ms"] / prof["launches"],
                    "flops_per_pair": FLOPS_PER_PAIR}
        rec = stored_counters(a.workload, kernel, used_tuning) if not a.n else None
        if rec:
            roofline["traffic"] = rec["traffic_bytes_per_evaluation"]
            counted = rec["counted_fp32_flops_per_evaluation"] / eval_s / 1e12
            roofline["counted_tflops"] = counted
            roofline["counted_frac"] = counted / PEAK_FP32_TFLOPS
            roofline["counted_source"] = os.path.relpath(COUNTERS, ROOT)
    sim.close()
    base = None
    if not a.no_cpu_baseline:
        base = cpu_baseline(bunches, a.cpu_seconds)
    out = {
        "metric": "pair interactions/s & % FP32 VALU peak",
        "value": value,
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if a.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "n_particles": sum(b.n for b in bunches), "bunches": len(bunches),
                   "pairs_per_step": pairs, "precision": a.precision,
                   "pair_math": "f32 hi/lo separations, two-sum tile accumulation" if a.precision == "mixed"
                   else "f64", "push": "f64 velocity Verlet", "graph": a.graph,
                   "parallelism": "single GPU",
                   "tuning": ",".join(f"{k}={v}" for k, v in used_tuning.items())},
        "roofline": roofline,
        "cpu_baseline": base,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
