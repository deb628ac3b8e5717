"""Throughput benchmark: Pauli strings per second of one exact M2 evaluation.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp32|fp64] [--N 20]

One step = one full evaluation (every shift x, its FWHT, sum |W|^4, the final
reduction and logarithm) of an N=20 Haar-random complex64 state that is
already resident in device memory.  Pauli strings per step = 4^N.

Printed (one JSON line on stdout): throughput, ms per step, the dominant
kernel's roofline position (timed live with HIP events around every launch in
the timed region), and the FP64 CPU oracle timed on this host's cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("Pauli strings/s at N=20 (fp32 vs split-fp16 MFMA, |ΔM2|≤1e-5); "
          "p50/p99 latency")
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU issue rate: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
# Bytes of the slab round trip per Pauli string and pass (complex values).
SLAB_BYTES = {"fp32": 8, "fp64": 16}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_roofline(N: int, form: str, kind: str, ms: float, launches: int, cs: int, P: int):
    """Roofline entry of one kernel class from its measured average duration."""
    avg_s = ms / 1e3 / launches
    d = 1 << N
    if kind in ("pass1", "pass2"):
        pauli_per_launch = cs * d
        by = SLAB_BYTES[form] * pauli_per_launch
        tb = 14 if form == "fp32" else 13
        ops = (4 + 2 * tb) if kind == "pass1" else (2 * (N - tb) + 5)
        gbs = by / avg_s / 1e9
        alu = ops * pauli_per_launch / avg_s
        ent = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
               "kernel": "k_pass1" if kind == "pass1" else "k_pass2",
               "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
               "alu_ops_per_pauli": ops, "alu_frac": round(alu / VALU_PEAK_OPS, 4)}
        if alu / VALU_PEAK_OPS > gbs / HBM_PEAK_GBS:
            ent.update(bound="alu", achieved=round(alu / 1e12, 3), peak=round(VALU_PEAK_OPS / 1e12, 2),
                       unit="Tops/s", frac=round(alu / VALU_PEAK_OPS, 4),
                       hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        return ent
    ops = 4 + 2 * N + 5
    pauli_per_launch = d * d
    alu = ops * pauli_per_launch / avg_s
    return {"bound": "alu", "achieved": round(alu / 1e12, 3), "peak": round(VALU_PEAK_OPS / 1e12, 2),
            "unit": "Tops/s", "frac": round(alu / VALU_PEAK_OPS, 4), "traffic": None,
            "kernel": "k_fused", "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
            "alu_ops_per_pauli": ops}


def cpu_baseline(psi: np.ndarray, target_s: float):
    import oracle

    N = psi.size.bit_length() - 1
    cores = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(1)
    probe = rng.choice(1 << N, size=cores, replace=False)
    t0 = time.perf_counter()
    oracle.partials(psi, probe, threads=cores)
    t1 = time.perf_counter() - t0
    per_shift = t1 / len(probe)
    count = int(max(cores, min(1 << N, target_s / max(per_shift, 1e-9))))
    count = max(cores, (count // cores) * cores)
    xs = rng.choice(1 << N, size=count, replace=False)
    t0 = time.perf_counter()
    oracle.partials(psi, xs, threads=cores)
    dt = time.perf_counter() - t0
    return {"value": count * float(1 << N) / dt, "unit": "Pauli strings/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{count} random shifts of the N={N} state (2^{N} Pauli strings each), "
                      f"{dt:.1f} s on {cores} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--N", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the evaluation shards over shifts x with no "
              "communication, so multi-GPU throughput is N x the one-GPU value; "
              "--gpus above 1 is not measured here.", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_24685_amd as sre2
    import workloads as W

    N = args.N
    log(f"bench: N={N} form={args.form} steps={args.steps} warmup={args.warmup}")
    psi = W.haar(N, W.config_seed(3), np.complex64)
    d_psi = torch.from_numpy(psi).to("cuda:0")
    ctx = sre2.Context(0)
    stream = torch.cuda.current_stream()
    for i in range(args.warmup):
        out, _ = sre2.m2_async(d_psi, form=args.form, ctx=ctx)
        torch.cuda.synchronize()
        log(f"warmup {i}: M2={out[0].item():.10f}")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    outs = []
    for i in range(args.steps):
        out, _ = sre2.m2_async(d_psi, form=args.form, ctx=ctx)
        outs.append(out)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    kt = ctx.timing_read()
    ctx.set_timing(False)
    m2s = [o[0].item() for o in outs]
    log(f"timed {args.steps} steps: {elapsed_ms:.1f} ms; M2={m2s[0]:.12f}; kernels={kt}")
    assert len(set(m2s)) == 1, "results differ between steps"
    ms_per_step = elapsed_ms / args.steps
    value = float(4 ** N) / (ms_per_step / 1e3)
    cs, P = ctx.chunking(N, args.form)
    dom = max((k for k in kt if k != "aux" and kt[k][1] > 0), key=lambda k: kt[k][0])
    roof = kernel_roofline(N, args.form, dom, kt[dom][0], kt[dom][1], cs, P)
    roof["kernels_ms_per_step"] = {k: round(v[0] / args.steps, 3) for k, v in kt.items()}
    cpu = None
    if not args.no_cpu:
        log("cpu baseline: timing the FP64 oracle on a sample of shifts ...")
        cpu = cpu_baseline(psi, args.cpu_seconds)
        log(f"cpu baseline: {cpu}")
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "Pauli strings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.form == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"exact M2 of one N={N} Haar-random complex64 state "
                               f"(plain XOR-FWHT, {args.form} butterflies, FP64 sums)",
                   "N": N, "pauli_strings_per_step": 4 ** N, "form": args.form,
                   "shifts_per_chunk": cs, "column_groups": P, "M2": m2s[0]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
