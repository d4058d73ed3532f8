"""bench.py's one-line JSON record on the GPU: the fields the benchmark
driver reads, their types, and their internal consistency (value = ordered
pairs per step over the time per step; roofline frac = achieved / peak; the
pair kernel's rate at least the whole step's).  A reduced workload keeps each
run to a few seconds; with a particle-count override no stored counter
record applies, so traffic and the counted fraction are null.
"""
import json
import math
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAK = {"mixed": 157.3, "fp64": 78.6}


def run_bench(*args):
    print(f"[case] bench.py {' '.join(args)}", flush=True)
    r = subprocess.run([sys.executable, "bench.py", *args], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [ln for ln in r.stdout.strip().splitlines() if ln.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0])


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_bench_json_record(prec):
    n, steps, warmup = 16384, 3, 1
    d = run_bench("--workload", "gaussian_65536", "--n", str(n), "--steps", str(steps), "--warmup", str(warmup),
                  "--precision", prec, "--cpu-seconds", "0.5")
    for key, typ in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                     ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                     ("dtype", str), ("data", str), ("config", dict), ("roofline", dict),
                     ("cpu_baseline", dict)):
        assert isinstance(d[key], typ), (key, d[key])
    assert d["n_gpus"] == 1 and d["steps"] == steps and d["warmup"] == warmup
    assert d["higher_is_better"] is True and d["scaling"] == "weak" and d["vs_baseline"] is None
    assert d["dtype"] == ("f32" if prec == "mixed" else "f64") and d["data"] == "synthetic"
    cfg = d["config"]
    assert cfg["workload"] == "gaussian_65536" and cfg["n_particles"] == n and cfg["precision"] == prec
    assert "model" not in cfg
    assert cfg["pairs_per_step"] == float(n * (n - 1))
    # value: ordered pair interactions per second of the whole timed step loop
    assert math.isclose(d["value"], cfg["pairs_per_step"] / (d["ms_per_step"] * 1e-3), rel_tol=1e-9)

    rf = d["roofline"]
    assert rf["bound"] == "alu" and rf["unit"] == "TFLOP/s" and rf["peak"] == PEAK[prec]
    assert rf["achieved"] > 0 and math.isclose(rf["frac"], rf["achieved"] / rf["peak"], rel_tol=1e-12)
    assert math.isclose(rf["achieved"], rf["flops_per_pair"] * cfg["pairs_per_step"]
                        / (rf["kernel_ms_per_evaluation"] * 1e-3) / 1e12, rel_tol=1e-9)
    # the pair kernel takes part of each step: its rate is at least the step's
    assert rf["achieved"] >= 0.99 * rf["flops_per_pair"] * d["value"] / 1e12
    assert rf["launches_per_evaluation"] >= 1
    assert rf["traffic"] is None and rf["counted_frac"] is None

    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "pair interactions/s"
    assert cb["value"] > 0 and isinstance(cb["cores"], int) and cb["cores"] >= 1
    assert isinstance(cb["sample"], str) and cb["sample"]
