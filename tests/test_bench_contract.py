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
    assert t is not None and abs(t / 2 ** 34 - 1) < 0.05  # the 16 GiB half slab of a row-pair chunk
    t = bench.stored_traffic("k_pass1", 20, "split16")
    assert t is not None and abs(t / 2 ** 34 - 1) < 0.05  # the split form's row pairs too


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("form,eb,L,half", [("fp32", 8, 12, True), ("fp32h", 8, 12, True),
                                             ("fp64", 16, 11, True), ("fp64h", 16, 11, True),
                                             ("split16", 8, 12, True)])
def test_algorithmic_bytes_per_evaluation(form, eb, L, half):
    """Slab bytes of a whole N = 20 evaluation: shifts below 2^L take the
    full slab of 2^20 values, the others (Hermitian pair, row pairs) half
    slabs (also the split forms, with row pairs on by default)."""
    pytest.importorskip("torch")
    by, ops = bench.alg_totals(20, form, "pass1", 0, 1 << 20)
    vals = (1 << L) * (1 << 20) + ((1 << 20) - (1 << L)) * (1 << 19) if half else 1 << 40
    assert by == eb * vals
    assert ops > 0
    # a range inside the half-slab shifts: 2^(N-1) values per shift
    by, _ = bench.alg_totals(20, form, "pass1", 1 << 19, 4096)
    assert by == eb * 4096 * (1 << (19 if half else 20))
