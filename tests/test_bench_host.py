"""Host-side checks of the benchmark's command line (no GPU needed)."""
import json
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.parametrize("workload", [None, "batch_uneven_256", "bp_sizes_a180"])
def test_more_than_one_gpu_is_refused(workload):
    cmd = [sys.executable, str(ROOT / "bench.py"), "--gpus", "2"]
    if workload:
        cmd += ["--workload", workload]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_elems_key():
    sys.path.insert(0, str(ROOT))
    import bench

    assert bench.elems_key(8, 8) == "8"
    assert bench.elems_key(4, 8) == "4,8"
