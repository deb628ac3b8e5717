"""Checkpointed M2 evaluation: stop and resume a long run.

The shifts x of Algorithm 1 are independent units (main text), so one
evaluation can be cut into shift ranges: each range's per-shift sums S_x
(`sre2_partials`) are stored on the host as soon as they are done, and a run
that stops - a killed job, a lost node - resumes at the first range not yet
stored.  The end is `sre2_m2_from_partials`: the norm, the fixed-order sum
over x and the logarithm of `sre2_m2`, so the result is bitwise that of one
uninterrupted call (S_x of a shift do not depend on the range it was computed
in).  A whole N = 24 FP32 evaluation takes about 13 minutes on one MI355X.

Files: `<path>.sx.npy` (float64, 2^N S_x, written in place as ranges finish)
and `<path>.json` (N, form, input dtype, SHA-256 of the state's bytes and the
count of shifts done, replaced atomically after the S_x of a range are
flushed).  A checkpoint of another state or form is refused.

This module only orders library calls and stores their results; every step
of the evaluation runs in the library's kernels.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

__all__ = ["m2_checkpointed", "checkpoint_files"]


def checkpoint_files(path: str) -> tuple[str, str]:
    """(S_x array file, metadata file) of a checkpoint."""
    return path + ".sx.npy", path + ".json"


def _state_bytes(psi) -> bytes:
    if isinstance(psi, np.ndarray):
        return np.ascontiguousarray(psi).tobytes()
    return psi.detach().reshape(-1).cpu().numpy().tobytes()


def _write_meta(meta_path: str, meta: dict) -> None:
    tmp = meta_path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(meta, f)
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, meta_path)


def m2_checkpointed(psi, path: str, form: str = "fp32", segment: int | None = None,
                    ctx=None, stop_after: int | None = None, remove: bool = False,
                    partials_fn=None, finish_fn=None, progress=None):
    """M2 of `psi` (complex64/complex128 device tensor of 2^N values) with
    its S_x checkpointed under `path` after every `segment` shifts.

    Returns the library's Result, or None when `stop_after` ranges were done
    in this call and the evaluation is not finished (a planned stop; calling
    again with the same arguments resumes).  `remove` deletes the checkpoint
    files after a finished evaluation.  `partials_fn(x_begin, x_count)` (host
    float64 array of S_x) and `finish_fn(sx)` (Result from all S_x as a host
    array) replace the library calls; by default they are `shift_partials`
    and `m2_from_partials` on psi's device.  `progress(done, total)` is called
    after every stored range.
    """
    n_values = psi.size if isinstance(psi, np.ndarray) else psi.numel()
    N = int(n_values).bit_length() - 1
    if n_values < 2 or (1 << N) != n_values:
        raise ValueError("state length must be 2^N with N >= 1")
    d = 1 << N
    if partials_fn is None or finish_fn is None:
        import torch

        import paper_2512_24685_amd as sre2

        if partials_fn is None:
            def partials_fn(x0, xc):
                return sre2.shift_partials(psi, x0, xc, form=form, ctx=ctx).cpu().numpy()
        if finish_fn is None:
            def finish_fn(sx):
                return sre2.m2_from_partials(psi, torch.from_numpy(sx).to(psi.device),
                                             form=form, ctx=ctx)
        if segment is None:
            c = ctx or sre2.context(psi.device.index or 0,
                                    int(torch.cuda.current_stream(psi.device).cuda_stream))
            cs, _ = c.chunking(N, form)
            segment = max(int(cs), d // 64)
    if segment is None:
        segment = max(1, d // 64)
    if segment < 1:
        raise ValueError("segment must be at least one shift")

    sx_path, meta_path = checkpoint_files(path)
    digest = hashlib.sha256(_state_bytes(psi)).hexdigest()
    dtype = str(psi.dtype).replace("torch.", "")
    want = {"N": N, "form": form, "dtype": dtype, "sha256": digest}
    if os.path.exists(meta_path):
        with open(meta_path) as f:
            meta = json.load(f)
        if any(meta.get(k) != v for k, v in want.items()):
            raise ValueError(f"checkpoint {path} belongs to another state or form: "
                             f"{ {k: meta.get(k) for k in want} }")
        sx = np.load(sx_path, mmap_mode="r+")
        if sx.shape != (d,) or sx.dtype != np.float64:
            raise ValueError(f"checkpoint {path}: S_x file of the wrong shape")
    else:
        sx = np.lib.format.open_memmap(sx_path, mode="w+", dtype=np.float64, shape=(d,))
        meta = dict(want, done=0)
        _write_meta(meta_path, meta)

    x = int(meta["done"])
    ranges = 0
    while x < d:
        if stop_after is not None and ranges >= stop_after:
            sx.flush()
            return None
        xc = min(segment, d - x)
        part = np.asarray(partials_fn(x, xc), dtype=np.float64)
        if part.shape != (xc,):
            raise ValueError(f"partials of shifts [{x}, {x + xc}) have shape {part.shape}")
        sx[x:x + xc] = part
        sx.flush()
        x += xc
        meta["done"] = x
        _write_meta(meta_path, meta)
        ranges += 1
        if progress is not None:
            progress(x, d)

    res = finish_fn(np.array(sx))
    del sx
    if remove:
        for p in (sx_path, meta_path):
            os.remove(p)
    return res
