"""GPU checks on the benchmark workloads beyond the N=20 single state.

* N=10 small states (complex128): Haar, |T>^10 and a graph state in every
  form against the oracle and the closed forms.
* N=16 batch: 32 Haar states against stored oracle M2 values (each stored
  value keeps the SHA-256 of its input bytes) and 8 graph+T states against
  m log2(4/3), through the packed batched path.
* N=20 Ising snapshot sequence psi_t = diag(exp(i pi t/64 h)) H^N |0>: M2 = 0
  at the Clifford angles t = 0, 16, 32, 48; M2(t) = M2(t + 32) = M2(32 - t);
  stored oracle values at t = 5 and 21 when present.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2512_24685_amd as sre2  # noqa: E402

LOG43 = np.log2(4.0 / 3.0)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sre2.lib()


def golden():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as f:
        return json.load(f)


def sha(psi):
    return hashlib.sha256(np.ascontiguousarray(psi).tobytes()).hexdigest()


def dev(psi):
    return torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")


@pytest.mark.parametrize("form", ["fp32", "fp64", "fp32h", "fp64h", "split16", "splitbf16"])
def test_n10_small(oracle_mod, form):
    """The N = 10 complex128 workload (Haar, |T>^10, graph state) in every
    form against the oracle on the same bytes and the closed forms."""
    print("CASE n10-small", form, flush=True)
    tol = 1e-9 if form.startswith("fp64") else 1e-5
    for name, psi, closed in W.workload_inputs("n10_small"):
        r = sre2.m2(dev(psi), form=form)
        assert r.status == 0, name
        assert abs(r.m2 - oracle_mod.m2(psi)) <= tol, (name, r.m2)
        if closed is not None:
            ctol = 1e-12 if form.startswith("fp64") else tol
            assert abs(r.m2 - closed) <= ctol, (name, r.m2, closed)


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16"])
def test_n16_batch(form):
    print("CASE n16-batch", form, flush=True)
    inputs = W.workload_inputs("n16_batch")
    g = golden()
    res = sre2.m2_batched([dev(p) for _, p, _ in inputs], form=form)
    checked = 0
    for i, ((name, psi, closed), r) in enumerate(zip(inputs, res)):
        assert r.status == 0
        if closed is not None:
            tol = 1e-5 if form.startswith("split") else 1e-6
            assert abs(r.m2 - closed) <= tol, name
            checked += 1
        else:
            rec = g.get(f"haar16_batch_{i}")
            assert rec and rec["sha256"] == sha(psi), f"stored oracle value missing for {name}"
            assert abs(r.m2 - rec["m2"]) <= 1e-5, name
            checked += 1
    assert checked == len(inputs) == 40


@pytest.mark.parametrize("form", ["fp32h", "fp32", "split16"])
def test_n20_snapshot_sequence(form):
    """Each result within the form's 1e-5 bar of the truth, so two results
    that must be equal differ by at most twice the bar in the split forms
    (their error is not the same function of the two states)."""
    print("CASE snapshots", form, flush=True)
    tol = 1e-5
    pair_tol = 2e-5 if form.startswith("split") else 1e-5
    zero_tol = 1e-5 if form.startswith("split") else 1e-6
    N = 20
    J = W.snapshot_couplings(N)
    h = W.ising_energy(N, J)
    g = golden()
    ts = [0, 5, 16, 21, 27, 32, 37, 48, 53]
    m = {}
    for t in ts:
        psi = W.ising_snapshot(N, t, J, dtype=np.complex64, energy=h)
        r = sre2.m2(dev(psi), form=form)
        assert r.status == 0
        m[t] = r.m2
        rec = g.get(f"ising20_t{t}")
        if t in (5, 21):  # stored oracle values (tests/golden)
            assert rec and rec["sha256"] == sha(psi), t
        if rec and rec["sha256"] == sha(psi):
            assert abs(r.m2 - rec["m2"]) <= tol, t
    for t in (0, 16, 32, 48):
        assert abs(m[t]) <= zero_tol, (t, m[t])
    for a, b in ((5, 37), (5, 27), (21, 53), (27, 37)):
        assert abs(m[a] - m[b]) <= pair_tol, (a, b, m[a], m[b])
    assert m[5] > 1.0 and m[21] > 1.0  # non-trivial between Clifford angles
