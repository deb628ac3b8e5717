"""GPU checks of the quench-dynamics simulator and its snapshot pipeline.

* Product states, two-qubit gates (brickwork Haar U(4) circuits, distant and
  reversed pairs) and TFIM steps match the CPU dynamics oracle (Kronecker
  products, tensor contraction, expm_multiply) to 1e-11.
* The pipeline (evolve -> snapshot -> serving loop, overlapped) returns for
  every step the same M2, bit for bit, as evaluating the same snapshot alone,
  and matches the oracle's M2 of the oracle-evolved state; M2 of the initial
  product state matches its Bloch-vector closed form.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2512_24685_amd as sre2  # noqa: E402
from oracle import dynamics as D  # noqa: E402

P = W.TFIM_PARAMS


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sre2.lib()


def host(t):
    return t.cpu().numpy()


def test_initial_and_product_states():
    print("CASE sim product", flush=True)
    for N in (2, 7, 12):
        sim = sre2.Simulator(N)
        ref = np.zeros(1 << N, np.complex128)
        ref[0] = 1.0
        assert np.array_equal(host(sim.state()), ref)
        th, ph = W.product_angles(N, 40 + N)
        sim.product_state(th, ph)
        assert np.abs(host(sim.state()) - D.product_state(th, ph)).max() < 1e-15
        sim.close()


def test_gates_match_oracle():
    print("CASE sim gates", flush=True)
    N, steps = 10, 4
    gates, pairs = W.brickwork_gates(N, steps, 5)
    sim = sre2.Simulator(N)
    th, ph = W.product_angles(N, 3)
    sim.product_state(th, ph)
    ref = D.product_state(th, ph)
    for t in range(steps):
        sim.apply_gates(gates[t], pairs)
        for U, (a, b) in zip(gates[t], pairs):
            ref = D.apply_2q(ref, U, a, b)
    assert np.abs(host(sim.state()) - ref).max() < 1e-13
    # distant and reversed pairs
    rng = np.random.default_rng(9)
    extra = [(0, 9), (7, 2), (5, 4)]
    Us = [W.haar_u4(rng) for _ in extra]
    sim.apply_gates(Us, extra)
    for U, (a, b) in zip(Us, extra):
        ref = D.apply_2q(ref, U, a, b)
    assert np.abs(host(sim.state()) - ref).max() < 1e-13
    sim.close()


@pytest.mark.parametrize("N", [6, 10, 14])
def test_tfim_steps_match_oracle(N):
    print("CASE sim tfim", N, flush=True)
    sim = sre2.Simulator(N)
    th, ph = W.product_angles(N, 70 + N)
    sim.product_state(th, ph)
    H = D.tfim_hamiltonian(N, P["J"], P["hx"], P["hz"])
    ref = D.product_state(th, ph)
    for _ in range(5):
        sim.tfim_step(P["J"], P["hx"], P["hz"], P["dt"])
    ref = D.tfim_evolve(ref, H, P["dt"], steps=5)
    assert np.abs(host(sim.state()) - ref).max() < 1e-11
    for _ in range(5):  # back in time
        sim.tfim_step(P["J"], P["hx"], P["hz"], -P["dt"])
    assert np.abs(host(sim.state()) - D.product_state(th, ph)).max() < 1e-11
    sim.close()


@pytest.mark.parametrize("form,dtype", [("fp32", "complex64"), ("fp32h", "complex64"),
                                        ("fp64", "complex128")])
def test_tfim_pipeline(oracle_mod, form, dtype):
    print("CASE pipeline tfim", form, flush=True)
    N, steps = 12, 10
    th, ph = W.product_angles(N, 123)
    sim = sre2.Simulator(N)
    sim.product_state(th, ph)
    srv = sre2.Server(form=form, hbm_budget=256 << 20, max_slots=16)
    res = sim.run_tfim(srv, P["J"], P["hx"], P["hz"], P["dt"], steps, dtype=dtype)
    srv.close()
    sim.close()
    assert len(res) == steps + 1 and all(r.status == 0 for r in res)
    # alone: the same snapshots evaluated one by one
    alone = sre2.Simulator(N)
    alone.product_state(th, ph)
    tdt = torch.complex64 if dtype == "complex64" else torch.complex128
    H = D.tfim_hamiltonian(N, P["J"], P["hx"], P["hz"])
    ref = D.product_state(th, ph)
    tol = 1e-9 if form == "fp64" else 1e-5
    for t in range(steps + 1):
        if t:
            alone.tfim_step(P["J"], P["hx"], P["hz"], P["dt"])
            ref = D.tfim_evolve(ref, H, P["dt"])
        a = sre2.m2(alone.state(tdt), form=form)
        assert a.m2 == res[t].m2 and a.S == res[t].S, t
        if t in (0, 1, 5, steps):
            assert abs(res[t].m2 - oracle_mod.m2(ref)) <= tol, t
    alone.close()
    assert abs(res[0].m2 - D.product_m2(th, ph)) <= tol


def test_circuit_pipeline(oracle_mod):
    print("CASE pipeline circuit", flush=True)
    N, steps = 11, 6
    gates, pairs = W.brickwork_gates(N, steps, 77)
    sim = sre2.Simulator(N)  # starts in |0...0> (all spins up)
    srv = sre2.Server(form="fp32h", hbm_budget=256 << 20, max_slots=16)
    res = sim.run_circuit(srv, gates, pairs)
    srv.close()
    sim.close()
    ref = np.zeros(1 << N, np.complex128)
    ref[0] = 1.0
    assert abs(res[0].m2) <= 1e-6  # a computational basis state is a stabilizer state
    for t in range(steps):
        for U, (a, b) in zip(gates[t], pairs):
            ref = D.apply_2q(ref, U, a, b)
        assert abs(res[t + 1].m2 - oracle_mod.m2(ref.astype(np.complex64))) <= 1e-5, t
    # M2 grows towards the Haar value log2(2^N + 3) - 2
    assert res[-1].m2 > res[1].m2 and res[-1].m2 < np.log2(2 ** N + 3) - 2 + 0.5
