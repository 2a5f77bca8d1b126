"""Host-side behaviour of bench.py: it refuses more than one GPU with a message, and with no GPU
it stops with an error instead of reporting a number from any other path."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, cwd=ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = _run("--gpus", str(n))
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == n and "one GPU" in line["error"]


def test_no_gpu_no_number():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("--steps", "1", "--warmup", "0", "--no-extras", "--no-cpu-baseline")
    assert r.returncode != 0
    assert "needs a GPU" in r.stderr
    assert '"value"' not in r.stdout


def test_cpu_legs_report_threads_and_host():
    """Both CPU legs time the oracle on a power-of-two sample and name the threads they used
    and the host's CPU."""
    import numpy as np

    sys.path.insert(0, ROOT)
    import bench
    from paper_2508_11443_amd import workloads
    keys = workloads.unique_u64(1 << 12, 5)
    vals = np.arange(keys.size, dtype=np.uint32)
    q, _ = workloads.u64_queries(keys, keys.size, 0.5, 6)
    for omp in (False, True):
        r = bench.cpu_leg(keys, vals, q, keys.size, 0.01, omp)
        assert r["kind"] == "oracle" and r["value"] > 0 and r["nproc"] >= 1
        assert r["cores"] == (1 if not omp else r["cores"]) and r["cores"] >= 1
        assert str(keys.size) in r["sample"]
