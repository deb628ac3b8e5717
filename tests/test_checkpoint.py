"""Checkpointed evaluation (paper_2512_24685_amd.checkpoint): stop, resume and
refusal logic on the CPU, with the FP64 oracle's per-shift sums standing in
for the library calls (Algorithm 1's loop body over shift ranges; the shifts
are independent units, main text).  The GPU counterpart is in
tests/test_gpu_checkpoint.py."""
import json
import os

import numpy as np
import pytest

import workloads as W
from paper_2512_24685_amd.checkpoint import checkpoint_files, m2_checkpointed

N = 8


@pytest.fixture(scope="module")
def psi():
    return W.haar(N, 123, np.complex128)


def _fns(oracle_mod, psi, calls):
    def partials_fn(x0, xc):
        calls.append((x0, xc))
        return oracle_mod.partials(psi, list(range(x0, x0 + xc)))

    def finish_fn(sx):
        return oracle_mod.m2_from_total(oracle_mod.sum_ascending(sx), oracle_mod.norm2(psi), N)

    return partials_fn, finish_fn


def test_straight_run_matches_oracle(tmp_path, oracle_mod, psi):
    calls = []
    pf, ff = _fns(oracle_mod, psi, calls)
    m = m2_checkpointed(psi, str(tmp_path / "a"), segment=40, partials_fn=pf, finish_fn=ff)
    assert m == pytest.approx(oracle_mod.m2(psi), abs=1e-12)
    # ranges cover [0, 2^N) in order, the last one short
    assert calls[0] == (0, 40) and calls[-1] == (240, 16)
    assert sum(c for _, c in calls) == 1 << N
    sx = np.load(checkpoint_files(str(tmp_path / "a"))[0])
    assert np.array_equal(sx, oracle_mod.partials(psi))


def test_stop_and_resume_gives_the_same_result(tmp_path, oracle_mod, psi):
    path = str(tmp_path / "b")
    calls = []
    pf, ff = _fns(oracle_mod, psi, calls)
    assert m2_checkpointed(psi, path, segment=32, stop_after=3, partials_fn=pf,
                           finish_fn=ff) is None
    with open(checkpoint_files(path)[1]) as f:
        assert json.load(f)["done"] == 96
    calls.clear()
    seen = []
    m = m2_checkpointed(psi, path, segment=32, partials_fn=pf, finish_fn=ff,
                        progress=lambda done, total: seen.append((done, total)))
    assert calls[0] == (96, 32)  # resumed at the first range not stored
    assert seen == [(128, 256), (160, 256), (192, 256), (224, 256), (256, 256)]
    ref = m2_checkpointed(psi, str(tmp_path / "ref"), segment=256, partials_fn=pf,
                          finish_fn=ff)
    assert m == ref


def test_failure_mid_run_keeps_the_finished_ranges(tmp_path, oracle_mod, psi):
    path = str(tmp_path / "c")
    calls = []
    pf, ff = _fns(oracle_mod, psi, calls)

    def failing(x0, xc):
        if x0 >= 64:
            raise RuntimeError("device lost")
        return pf(x0, xc)

    with pytest.raises(RuntimeError):
        m2_checkpointed(psi, path, segment=32, partials_fn=failing, finish_fn=ff)
    with open(checkpoint_files(path)[1]) as f:
        assert json.load(f)["done"] == 64
    calls.clear()
    m = m2_checkpointed(psi, path, segment=50, partials_fn=pf, finish_fn=ff, remove=True)
    assert calls[0] == (64, 50)
    assert m == pytest.approx(oracle_mod.m2(psi), abs=1e-12)
    assert not any(os.path.exists(p) for p in checkpoint_files(path))


def test_checkpoint_of_another_state_or_form_is_refused(tmp_path, oracle_mod, psi):
    path = str(tmp_path / "d")
    pf, ff = _fns(oracle_mod, psi, [])
    assert m2_checkpointed(psi, path, segment=64, stop_after=1, partials_fn=pf,
                           finish_fn=ff) is None
    other = W.haar(N, 124, np.complex128)
    pf2, ff2 = _fns(oracle_mod, other, [])
    with pytest.raises(ValueError, match="another state or form"):
        m2_checkpointed(other, path, segment=64, partials_fn=pf2, finish_fn=ff2)
    with pytest.raises(ValueError, match="another state or form"):
        m2_checkpointed(psi, path, form="fp64", segment=64, partials_fn=pf, finish_fn=ff)
