"""Write oracle-only expected values for the large parity cases.

Every value stored by this script comes from the FP64 CPU oracle in
``oracle/`` applied to the seeded inputs of ``workloads``; nothing here comes
from the GPU path.  Each record keeps the SHA-256 of the exact input bytes, so
a test can detect a drifted generator instead of comparing against a stale
value.

Usage:  python tests/golden/make_golden.py [--threads T] [--only NAME ...]
The N=20 full evaluation takes about an hour on 8 cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")


def sha(psi: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(psi).tobytes()).hexdigest()


def sample_shifts(N: int, count: int = 256, seed: int = 7) -> list[int]:
    """x = 0, a few structured shifts, then seeded random ones (sorted, unique)."""
    d = 1 << N
    rng = np.random.default_rng(seed + N)
    xs = {0, 1, d - 1, d >> 1, (d >> 1) - 1, 0x5555555555555555 & (d - 1),
          0x3333333333333333 & (d - 1)}
    while len(xs) < count:
        xs.add(int(rng.integers(0, d)))
    return sorted(xs)


def cases():
    """(name, builder) for every stored case; builders are cheap."""
    out = []
    s20, sl = W.SEED_N20, W.SEED_LARGE
    out.append(("haar20_sampled", lambda: W.haar(20, s20, np.complex64), "sampled"))
    out.append(("haar22_sampled", lambda: W.haar(22, sl, np.complex64), "sampled"))
    out.append(("haar24_sampled", lambda: W.haar(24, sl + 1, np.complex64), "sampled"))
    s16 = W.SEED_N16_BATCH
    for i in range(32):
        out.append((f"haar16_batch_{i}",
                    (lambda i=i: W.haar(16, s16 * 1000 + i, np.complex64)), "full"))
    out.append(("haar20", lambda: W.haar(20, s20, np.complex64), "full"))
    J = W.snapshot_couplings(20)
    for t in (5, 21):
        out.append((f"ising20_t{t}",
                    (lambda t=t: W.ising_snapshot(20, t, J, dtype=np.complex64)), "full"))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--only", nargs="*", default=None)
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name, build, kind in cases():
        if args.only and name not in args.only:
            continue
        psi = build()
        h = sha(psi)
        if name in data and data[name].get("sha256") == h:
            continue
        N = psi.size.bit_length() - 1
        t0 = time.time()
        rec = {"N": N, "dtype": str(psi.dtype), "sha256": h, "kind": kind}
        if kind == "full":
            S, n = oracle.total(psi, threads=args.threads)
            rec.update(total=S, norm2=n, m2=oracle.m2_from_total(S, n, N))
        else:
            xs = sample_shifts(N)
            rec.update(shifts=xs, partials=oracle.partials(psi, xs, threads=args.threads).tolist(),
                       norm2=oracle.norm2(psi))
        rec["oracle_seconds"] = time.time() - t0
        data[name] = rec
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(f"{name}: {rec.get('m2', '')} ({rec['oracle_seconds']:.1f} s)", flush=True)


if __name__ == "__main__":
    main()
