"""GPU checks of the general Renyi index (Eq. 1) and the Pauli spectrum.

* M_alpha for alpha in {0.5, 1, 1.5, 3} in every non-split form, at sizes that
  take the tiny, fused and two-pass kernels, against the FP64 oracle
  (|dM| <= 1e-5 for FP32 forms, 1e-9 for FP64 forms).
* alpha = 2 gives results bitwise equal to sre2_m2, in every form.
* Closed forms: |T>^N gives N (1/(1-alpha)) log2((1 + 2^(1-alpha))/2)
  (N/2 at alpha = 1); stabilizer states give 0.
* Spectrum: exact counts for stabilizer and |T>-product states (their values
  sit at bin centres), total 4^N always, and Haar states within the number
  of oracle values near a bin edge.
* N = 22 (FP32): the general kernels' half-LDS column tiles of pass 2 (ten
  slab-row bits, 2^14-value tiles) on |T>^22 against both closed forms.
"""
import functools

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2512_24685_amd as sre2  # noqa: E402

ALPHAS = [0.5, 1.0, 1.5, 3.0]
FORMS = ["fp32", "fp32h", "fp64", "fp64h"]
TOL = {"fp32": 1e-5, "fp32h": 1e-5, "fp64": 1e-9, "fp64h": 1e-9}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sre2.lib()


def dev(psi):
    return torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")


def t_single(alpha):
    if alpha == 1:
        return 0.5
    return np.log2((1.0 + 2.0 ** (1.0 - alpha)) / 2.0) / (1.0 - alpha)


@functools.lru_cache(maxsize=None)
def haar_case(N, c128):
    return W.haar(N, 4242 + N, np.complex128 if c128 else np.complex64)


@functools.lru_cache(maxsize=None)
def oracle_sre(N, c128, alpha):
    import oracle
    return oracle.sre(haar_case(N, c128), alpha)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N", [3, 6, 9, 13, 15])
def test_alpha_matches_oracle(form, N):
    c128 = form.startswith("fp64")
    psi = haar_case(N, c128)
    d = dev(psi)
    for alpha in ALPHAS:
        print("CASE alpha", form, N, alpha, flush=True)
        r = sre2.sre(d, alpha, form=form)
        assert r.status == 0
        err = abs(r.m2 - oracle_sre(N, c128, alpha))
        assert err <= TOL[form], (alpha, err)


@pytest.mark.parametrize("form", FORMS + ["split16", "splitbf16"])
def test_alpha2_is_m2_bitwise(form):
    for N in (4, 11, 16):
        psi = W.haar(N, 77 + N, np.complex64)
        d = dev(psi)
        print("CASE alpha2", form, N, flush=True)
        a, b = sre2.sre(d, 2.0, form=form), sre2.m2(d, form=form)
        assert a.m2 == b.m2 and a.S == b.S and a.n == b.n


@pytest.mark.parametrize("form", FORMS)
def test_alpha_closed_forms(form):
    dt = np.complex128 if form.startswith("fp64") else np.complex64
    for N in (4, 10, 16):
        t = dev(W.t_product(N, dt))
        g = dev(W.graph(N, 55 + N, dtype=dt))
        for alpha in ALPHAS:
            print("CASE closed", form, N, alpha, flush=True)
            assert abs(sre2.sre(t, alpha, form=form).m2 - N * t_single(alpha)) <= 2 * TOL[form]
            assert abs(sre2.sre(g, alpha, form=form).m2) <= 2 * TOL[form]


@pytest.mark.parametrize("form", FORMS)
def test_spectrum_closed_forms(form):
    from math import comb
    dt = np.complex128 if form.startswith("fp64") else np.complex64
    for N in (4, 10, 15):
        d = 1 << N
        print("CASE spectrum closed", form, N, flush=True)
        counts, r = sre2.pauli_spectrum(dev(W.graph(N, 21 + N, dtype=dt)), 24, form=form)
        assert r.status == 0
        assert counts[0] == d and counts[-1] == d * d - d and counts[1:-1].sum() == 0
        counts, _ = sre2.pauli_spectrum(dev(W.t_product(N, dt)), N + 3, form=form)
        for k in range(N + 1):
            assert counts[k] == comb(N, k) * 2 ** k, (k, counts[k])
        assert counts[-1] == 4 ** N - 3 ** N


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N", [5, 12, 15])
def test_spectrum_haar_matches_oracle(oracle_mod, form, N):
    c128 = form.startswith("fp64")
    psi = haar_case(N, c128)
    nbins = N + 6
    print("CASE spectrum haar", form, N, flush=True)
    counts, r = sre2.pauli_spectrum(dev(psi), nbins, form=form)
    assert r.status == 0 and counts.sum() == 4 ** N
    ref, near = oracle_mod.spectrum(psi, nbins, eps=2e-3 if not c128 else 1e-7)
    diff = int(np.abs(counts - ref).sum())
    assert diff <= 2 * near, (diff, near)



def test_general_kernels_half_lds_tiles_n22():
    """At N = 22 the FP32 pass 2 holds ten row bits in 2^14-value tiles that
    transpose through half the LDS; the general reductions take those tiles
    too.  |T>^22: M_3 = 22 log2((1 + 2^-2)/2) / (1 - 3) and the spectrum
    C(22, k) 2^k strings at q = 2^-k, 4^22 - 3^22 zeros (last bin)."""
    from math import comb
    N = 22
    t = dev(W.t_product(N, np.complex64))
    print("CASE alpha n22", flush=True)
    r = sre2.sre(t, 3.0, form="fp32")
    assert r.status == 0
    assert abs(r.m2 - N * t_single(3.0)) <= TOL["fp32"], r.m2
    print("CASE spectrum n22", flush=True)
    counts, r = sre2.pauli_spectrum(t, N + 2, form="fp32")
    assert r.status == 0
    for k in range(N + 1):
        assert counts[k] == comb(N, k) * 2 ** k, (k, counts[k])
    assert counts[-1] == 4 ** N - 3 ** N
