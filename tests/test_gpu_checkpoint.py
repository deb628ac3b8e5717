"""Checkpointed evaluation on the GPU: M2 from per-shift sums gathered over
shift ranges (sre2_partials, then sre2_m2_from_partials; the shifts are
independent units, main text) equals one sre2_m2 call bitwise, also after a
planned stop and a resume with ranges that do not align with the library's
chunks."""
import numpy as np
import pytest
import torch

import paper_2512_24685_amd as sre2
import workloads as W
from paper_2512_24685_amd.checkpoint import m2_checkpointed

pytestmark = pytest.mark.gpu

# fused, two-pass, Hermitian pair across the plain / pair boundary, split MFMA, FP64
CASES = [(12, "fp32", np.complex64), (16, "fp32", np.complex64), (17, "fp32h", np.complex64),
         (15, "split16", np.complex64), (14, "fp64", np.complex128)]


def _dev(N, dt):
    return torch.from_numpy(W.haar(N, 300 + N, dt)).to("cuda:0")


@pytest.mark.parametrize("N,form,dt", CASES)
def test_from_partials_equals_m2(N, form, dt):
    print(f"case from_partials N={N} form={form}", flush=True)
    psi = _dev(N, dt)
    r = sre2.m2(psi, form=form, partials=True)
    f = sre2.m2_from_partials(psi, r.partials, form=form)
    assert f.status == 0
    assert (f.m2, f.S, f.n) == (r.m2, r.S, r.n)


@pytest.mark.parametrize("N,form,dt", CASES)
def test_checkpointed_resume_equals_m2(tmp_path, N, form, dt):
    print(f"case checkpoint N={N} form={form}", flush=True)
    psi = _dev(N, dt)
    ref = sre2.m2(psi, form=form)
    seg = (1 << N) // 10 + 7
    path = str(tmp_path / "ck")
    assert m2_checkpointed(psi, path, form=form, segment=seg, stop_after=4) is None
    r = m2_checkpointed(psi, path, form=form, segment=seg, remove=True)
    assert r.status == 0
    assert (r.m2, r.S, r.n) == (ref.m2, ref.S, ref.n)


def test_from_partials_rejects_a_wrong_buffer():
    psi = _dev(10, np.complex64)
    with pytest.raises(ValueError):
        sre2.m2_from_partials(psi, torch.zeros(10, dtype=torch.float64, device="cuda:0"))
