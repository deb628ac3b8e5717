"""GPU test of sre2_m2_noalloc, the allocation-free variant of sre2_m2.

Called through the C ABI and checked against sre2_m2 on the same inputs,
two calls in a row on one device with the second input smaller than the
first, so that the second call runs over what the first left in the shared
fixed array: results must be bitwise equal to sre2_m2's (the same kernels
and reduction order; chunking never changes a result bit), and within the
method's bar of the FP64 oracle where that is cheap.
"""
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


def noalloc(d, form, partials=False):
    out = torch.empty(sre2.OUT_LEN, dtype=torch.float64, device=d.device)
    part = torch.empty(d.numel(), dtype=torch.float64, device=d.device) if partials else None
    sre2.m2_noalloc_async(d, out, form=form, partials=part)
    return out.cpu().tolist(), (part.cpu().numpy() if partials else None)


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "fp64", "fp64h"])
def test_noalloc_equals_m2_two_calls(oracle_mod, form):
    big = W.haar(18 if not form.startswith("fp64") else 17, 515, np.complex64)
    small = W.haar(13, 516, np.complex64)
    for psi in (big, small):  # the second call is smaller than the first
        N = psi.size.bit_length() - 1
        print("CASE noalloc", form, N, flush=True)
        d = dev(psi)
        got, _ = noalloc(d, form)
        ref = sre2.m2(d, form=form)
        assert got[3] == 0.0 and ref.status == 0
        assert got[0] == ref.m2 and got[1] == ref.S and got[2] == ref.n, (got, ref)
        if N <= 13:
            tol = 1e-9 if form.startswith("fp64") else 1e-5
            assert abs(got[0] - oracle_mod.m2(psi)) <= tol


def test_noalloc_partials_and_input_conversion():
    psi = W.haar(16, 517, np.complex128)
    d = dev(psi)
    print("CASE noalloc partials", flush=True)
    got, part = noalloc(d, "fp32", partials=True)
    ref = sre2.m2(d, form="fp32", partials=True)
    assert got[0] == ref.m2 and got[1] == ref.S
    assert np.array_equal(part, ref.partials.cpu().numpy())
    small = dev(W.haar(9, 518, np.complex128))
    got2, _ = noalloc(small, "fp64")
    assert got2[0] == sre2.m2(small, form="fp64").m2


def test_noalloc_rejects_beyond_limit_without_work():
    d = dev(np.zeros(1 << 21, np.complex64))
    out = torch.empty(sre2.OUT_LEN, dtype=torch.float64, device="cuda")
    with pytest.raises(sre2.SRE2Error) as e:
        sre2.m2_noalloc_async(d, out, form="fp32")
    assert e.value.code == sre2.ESCRATCH
