"""Host logic of the benchmark script and the workload listing (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_overrides_parse_and_reject():
    sys.path.insert(0, ROOT)
    import bench
    cfg = {"n": 1 << 20, "k": 64, "sigma_m": 10.0}
    ov = bench._apply_overrides(cfg, ["n=4096", "sigma_m=2.5", "k=16", "dt=5e-4"])
    assert ov == {"n": 4096, "sigma_m": 2.5, "k": 16, "dt": 5e-4}
    assert cfg["n"] == 4096 and isinstance(cfg["n"], int) and cfg["dt"] == 5e-4
    for bad in ("foo=1", "n", "k=x"):
        with pytest.raises((SystemExit, ValueError)):
            bench._apply_overrides(dict(cfg), [bad])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workload_listing():
    r = subprocess.run([sys.executable, "-m", "workloads", "all"], capture_output=True, text=True,
                       cwd=ROOT, timeout=120, check=True)
    rows = [json.loads(line) for line in r.stdout.splitlines()]
    assert [x["name"] for x in rows] == ["C1", "C2", "C3", "C4", "C5", "BLK"]
    c2 = rows[1]
    assert c2["n"] == 1 << 20 and c2["k"] == 64 and c2["sigma_m"] == 10.0 and c2["host"]
    assert len(rows[3]["halos"]) == 64
    assert rows[4]["n"] == 1 << 24 and rows[4]["eps"] == 0.002
