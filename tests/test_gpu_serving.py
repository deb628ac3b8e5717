"""GPU tests of the batched path and the continuous-batching server.

* Packed batches (several states of one N in shared launches) give results
  bitwise identical to single calls, for every form, including packs larger
  than one launch holds.
* The server's results for a mixed stream of requests are bitwise identical
  to each state evaluated alone, and within the form's tolerance of the
  oracle on sampled requests.
* Admission by memory budget (backpressure), cancellation of queued
  requests, rejection of invalid inputs, device-resident inputs.
"""
import time

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2512_24685_amd as sre2  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sre2.lib()


def dev(psi):
    return torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")


def mixed_states(count, seed, n_lo, n_hi, dtype=np.complex64):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.integers(n_lo, n_hi + 1))
        if rng.random() < 0.5:
            out.append(W.haar(N, seed * 7919 + i, dtype))
        else:
            psi, _ = W.graph_t(N, min(N, int(rng.integers(1, 9))), seed * 7919 + i, dtype=dtype)
            out.append(psi)
    return out


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16", "fp64", "fp64h"])
def test_packed_batch_bitwise_equals_single(form):
    states = mixed_states(60, 11, 1, 16)
    states += [W.haar(9, 500 + i, np.complex64) for i in range(70)]  # > one pack of N=9
    d = [dev(p) for p in states]
    print("CASE batch", form, flush=True)
    batch = sre2.m2_batched(d, form=form)
    for p, b in zip(d, batch):
        a = sre2.m2(p, form=form)
        assert a.m2 == b.m2 and a.S == b.S and a.n == b.n and a.status == b.status


def wait_all(srv, tickets, timeout=300.0):
    res = {}
    t_end = time.time() + timeout
    while len(res) < len(tickets):
        assert time.time() < t_end, "server did not finish in time"
        for t in tickets:
            if t in res:
                continue
            st, r, lat = srv.poll(t)
            if st >= sre2.REQ_DONE:
                res[t] = (st, r, lat)
        time.sleep(0.001)
    return res


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16"])
def test_server_mix_equals_alone(oracle_mod, form):
    states = mixed_states(160, 23, 3, 18)
    print("CASE server-mix", form, flush=True)
    srv = sre2.Server(form=form, hbm_budget=1 << 30, max_slots=64)
    tickets = []
    for i, p in enumerate(states):
        tickets.append(srv.submit(p))
        if i % 16 == 0:
            time.sleep(0.002)  # arrivals spread over time: later ones join running work
    res = wait_all(srv, tickets)
    stats = srv.stats()
    srv.close()
    assert stats["completed"] == len(states) and stats["packs"] > 0 and stats["singles"] > 0
    assert stats["packed_states"] > stats["packs"]  # some launches really were shared
    for k, (p, t) in enumerate(zip(states, tickets)):
        st, r, lat = res[t]
        assert st == sre2.REQ_DONE and r.status == 0 and lat > 0
        alone = sre2.m2(dev(p), form=form)
        assert r.m2 == alone.m2 and r.S == alone.S, k
        if p.size <= 1 << 12:
            assert abs(r.m2 - oracle_mod.m2(p)) <= 1e-5


def test_server_backpressure_cancel_and_bad_inputs():
    print("CASE server-backpressure", flush=True)
    budget = 3 << 20  # three N=18 states at most
    srv = sre2.Server(form="fp32", hbm_budget=budget, max_slots=8)
    states = [W.haar(18, 900 + i, np.complex64) for i in range(8)]
    tickets = [srv.submit(p) for p in states]
    srv.cancel(tickets[-1])  # still queued behind the budget
    res = wait_all(srv, tickets)
    stats = srv.stats()
    assert res[tickets[-1]][0] == sre2.REQ_CANCELLED
    for t in tickets[:-1]:
        assert res[t][0] == sre2.REQ_DONE
    assert stats["peak_bytes"] <= budget
    assert stats["peak_inflight"] <= 3
    # invalid inputs fail alone, at submit
    bad = W.haar(8, 1, np.complex64)
    bad[7] = np.nan
    with pytest.raises(sre2.SRE2Error) as e:
        srv.submit(bad)
    assert e.value.code == sre2.ENORM
    with pytest.raises(sre2.SRE2Error) as e:
        srv.submit(np.zeros(1 << 22, np.complex64))  # can never fit 3 MiB
    assert e.value.code == sre2.ENOMEM
    good = W.haar(10, 3, np.complex64)
    t = srv.submit(good)
    (st, r, _), = wait_all(srv, [t]).values()
    assert st == sre2.REQ_DONE and r.m2 == sre2.m2(dev(good)).m2
    with pytest.raises(sre2.SRE2Error) as e:
        srv.poll(t)  # released after its final poll
    assert e.value.code == sre2.ENOTFOUND
    srv.close()


def test_server_launch_failure_fails_requests_without_hanging(monkeypatch):
    """Transform launches that report an error (forced from the host; no
    kernel fails): every request of the small and the large lane still
    completes, as failed, and drain and destroy report the HIP error."""
    print("CASE server-launch-fault", flush=True)
    srv = sre2.Server(form="fp32", hbm_budget=64 << 20, max_slots=16)
    monkeypatch.setenv("SRE2_FAULT", "launch")
    states = [W.haar(N, 950 + N, np.complex64) for N in (8, 12, 16, 17)]
    tickets = [srv.submit(p) for p in states]
    res = wait_all(srv, tickets)
    assert all(res[t][0] == sre2.REQ_FAILED for t in tickets)
    with pytest.raises(sre2.SRE2Error) as e:
        srv.drain(60.0)
    assert e.value.code == sre2.EHIP
    monkeypatch.delenv("SRE2_FAULT")
    with pytest.raises(sre2.SRE2Error) as e:
        srv.close()
    assert e.value.code == sre2.EHIP


def test_server_device_inputs_and_zero_state():
    print("CASE server-device", flush=True)
    srv = sre2.Server(form="fp32h", hbm_budget=256 << 20, max_slots=16)
    d = [dev(W.haar(N, 40 + N, np.complex64)) for N in (6, 12, 15, 17)]
    z = dev(np.zeros(1 << 9, np.complex64))
    torch.cuda.synchronize()  # device inputs must be complete before submit
    tickets = [srv.submit(p) for p in d] + [srv.submit(z)]
    res = wait_all(srv, tickets)
    srv.drain(60.0)
    srv.close()
    for p, t in zip(d, tickets):
        assert res[t][1].m2 == sre2.m2(p, form="fp32h").m2
    zr = res[tickets[-1]][1]
    assert zr.status == 1 and np.isnan(zr.m2)
