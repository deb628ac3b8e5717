"""sre2_m2 under HIP graph capture: after one eager call has sized the
context's workspace, a call enqueues only kernel launches on the caller's
stream (zeroing is done by kernels, not memset nodes), so it can be captured
once and replayed.  Every replay is checked against the eager result, with
other eager work on the GPU between replays."""
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


@pytest.mark.parametrize("N,form", [(12, "fp32"), (13, "fp64"), (16, "fp32"), (16, "split16"),
                                    (17, "fp32h")])
def test_m2_replays_from_a_hip_graph(N, form):
    print("CASE graph", N, form, flush=True)
    psi = dev(W.haar(N, 300 + N, np.complex64))
    other = dev(W.haar(N, 400 + N, np.complex64))
    ctx = sre2.Context(0)
    side = sre2.Context(0)
    eager, _ = sre2.m2_async(psi, form=form, ctx=ctx)  # sizes the workspace
    torch.cuda.synchronize()
    eager = eager.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out, _ = sre2.m2_async(psi, form=form, ctx=ctx)
    ref_other = sre2.m2(other, form=form, ctx=side)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), (out, eager)
        r = sre2.m2(other, form=form, ctx=side)  # eager work between replays
        assert r.m2 == ref_other.m2 and r.S == ref_other.S
    ctx.close()
    side.close()
