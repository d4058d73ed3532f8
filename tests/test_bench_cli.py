"""bench.py's command line without a GPU: it refuses GPU counts other than one
in every mode, before touching a device, and its oracle-only mode runs on the
CPU alone."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("mode", ["throughput", "drift", "paper", "oracle", "tilings"])
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
