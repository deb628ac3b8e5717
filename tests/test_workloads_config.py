"""The benchmark configurations file (workloads/configs.json) is the source of
the workloads' seeds: the inputs it describes are the ones the stored oracle
values (tests/golden) were computed for."""
import hashlib
import json
import os

import numpy as np

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")


def _sha(psi):
    return hashlib.sha256(np.ascontiguousarray(psi).tobytes()).hexdigest()


def test_configs_file_lists_the_five_configurations():
    names = [c["name"] for c in W.CONFIGS["configs"]]
    assert names == ["n10_small", "n16_batch", "n20_single", "serving", "n22_n24_large"]
    assert [c["id"] for c in W.CONFIGS["configs"]] == [1, 2, 3, 4, 5]
    offsets = [c["seed_offset"] for c in W.CONFIGS["configs"]]
    assert len(set(offsets)) == 5  # one independent seed per configuration
    assert W.SEED_N20 == W.CONFIGS["base_seed"] + 3


def test_inputs_follow_the_file():
    cfg = {c["name"]: c for c in W.CONFIGS["configs"]}
    n10 = W.workload_inputs("n10_small")
    assert len(n10) == 3 and all(p.size == 1 << cfg["n10_small"]["N"] for _, p, _ in n10)
    assert all(p.dtype == np.complex128 for _, p, _ in n10)
    b = W.workload_inputs("n16_batch")
    assert len(b) == cfg["n16_batch"]["haar"] + cfg["n16_batch"]["graph_t"]
    assert all(p.size == 1 << 16 and p.dtype == np.complex64 for _, p, _ in b)
    reqs = W.serving_requests(cfg["serving"]["requests"])
    Ns = [r["N"] for r in reqs]
    assert len(reqs) == 4096 and min(Ns) == cfg["serving"]["N_min"] and max(Ns) == cfg["serving"]["N_max"]


def test_stored_oracle_values_belong_to_these_inputs():
    with open(GOLDEN) as f:
        g = json.load(f)
    psi20 = W.haar(20, W.SEED_N20, np.complex64)
    assert g["haar20"]["sha256"] == _sha(psi20)
    batch = dict((name, p) for name, p, _ in W.workload_inputs("n16_batch"))
    assert g["haar16_batch_0"]["sha256"] == _sha(batch["haar16_0"])
