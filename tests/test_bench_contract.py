"""CPU checks of the benchmark's contract and bookkeeping (no GPU).

* The stored HBM-traffic counters (profiles/traffic_counters.json) were taken
  on the current kernel code, so `bench.py` reports them; a change of the
  kernels without new counters fails here.
* --gpus above 1 is refused with a message and exit status 2.
* Algorithmic bytes per launch: 8 B per slab value (16 B in FP64), chunk
  shifts x 2^N values (2^(N-1) in the Hermitian-pair forms).
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_stored_counters_match_the_kernel_code():
    with open(os.path.join(ROOT, "profiles", "traffic_counters.json")) as f:
        rec = json.load(f)
    sha = bench.kernel_source_sha()
    assert rec["entries"] and all(e["source_sha"] == sha for e in rec["entries"])
    t = bench.stored_traffic("k_pass1", 20, "fp32")
    assert t is not None and abs(t / 2 ** 35 - 1) < 0.05  # the 32 GiB slab of a chunk


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("form,eb,ns", [("fp32", 8, 20), ("fp32h", 8, 19), ("fp64", 16, 20)])
def test_algorithmic_bytes_per_launch(form, eb, ns):
    pytest.importorskip("torch")
    by, ops = bench.alg_units(20, form, "pass1", 4096)
    assert by == eb * 4096 * (1 << ns)
    assert ops > 0
