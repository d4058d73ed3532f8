"""bench.py's command line without a GPU: it refuses GPU counts other than one
in every mode, before touching a device, and its oracle-only mode runs on the
CPU alone."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("mode", ["throughput", "drift", "paper", "oracle", "tilings", "steps", "ubench"])
def test_bench_refuses_more_than_one_gpu(mode):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--mode", mode],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_bench_oracle_mode_serial():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "oracle", "--n", "3000",
                        "--cpu-threads", "1", "--cpu-seconds", "0.2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    base = line["cpu_baseline"]
    assert base["cores"] == 1 and base["kind"] == "oracle"
    assert line["value"] == base["value"] > 0
    assert line["config"]["n"] == 3000


def test_paper_512_oracle_timing_leaves_the_thread_count():
    """The serial and all-core oracle timing of the 512-particle PP run of the
    paper's PIC comparison (Sec. 3.2) restores the oracle's thread count and
    reports both times."""
    sys.path.insert(0, ROOT)
    import bench
    from oracle.oracle import default
    from paper_2502_10640_amd import workloads as wl
    before = default().num_threads()
    b = wl.paper_cube(8, dt=1e-12)
    res = bench.cpu_baseline_vv(b, 20)
    assert default().num_threads() == before
    assert res["serial_cores"] == 1 and res["all_cores_cores"] == before
    assert res["serial_s"] > 0 and res["all_cores_s"] > 0
    assert res["pairs"] == 512 * 511 * 21
    assert bench.PAPER_512["pic"]["steps"] == 100 and bench.PAPER_512["long"]["steps"] == 3200
