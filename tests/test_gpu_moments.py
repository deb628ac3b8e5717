"""GPU moments of the input (n = sum |psi|^2, sum |psi|^4, non-finite count)
through the C ABI against the FP64 oracle on the same bytes."""
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


@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
@pytest.mark.parametrize("N", [1, 3, 9, 14, 15, 20])
def test_moments_match_oracle(oracle_mod, N, dtype):
    psi = W.haar(N, 300 + N, dtype) * 1.25  # unnormalised on purpose
    print("CASE moments", N, np.dtype(dtype).name, flush=True)
    n, ipr, bad = sre2.moments(dev(psi))
    assert bad == 0
    # the same FP64 terms summed in another order: a few ulps apart
    assert abs(n - oracle_mod.norm2(psi)) <= 1e-13 * n
    assert abs(ipr - oracle_mod.ipr(psi)) <= 1e-13 * ipr
    again = sre2.moments(dev(psi))
    assert again == (n, ipr, bad)  # fixed summation order


def test_moments_special_inputs():
    print("CASE moments special", flush=True)
    assert sre2.moments(dev(np.zeros(1 << 10, np.complex64))) == (0.0, 0.0, 0)
    e = np.zeros(1 << 12, np.complex128)
    e[1234] = 1.0
    assert sre2.moments(dev(e)) == (1.0, 1.0, 0)
    bad = W.haar(16, 4, np.complex64)
    bad[[3, 40000, 65535]] = [np.nan, np.inf, complex(1.0, -np.inf)]
    assert sre2.moments(dev(bad))[2] == 3
