"""Throughput benchmark: Pauli strings per second of one exact M2 evaluation.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp32]
                    [--also fp32h,fp64] [--N 20] [--no-cpu]
    python bench.py --copy-calibration MiB     (plain device copy, for counters)

One step = one full evaluation (every shift x, its FWHT, sum |W|^4, the final
reduction and logarithm) of an N=20 Haar-random complex64 state that is
already resident in device memory.  Pauli strings per step = 4^N.

Printed (one JSON line on stdout): throughput of the headline form (plain
FP32 XOR-FWHT), ms per step, the dominant kernel's roofline position (timed
live with HIP events around every launch in the timed region), the other
forms measured the same way, and the FP64 CPU oracle timed on this host's
cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
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
# Non-packed FP32/FP64 VALU issue rate: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz.
VALU_PEAK_OPS = 256 * 64 * 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCES = ["paper_2512_24685_amd/csrc/sre2_kernels.hip",
                  "paper_2512_24685_amd/csrc/sre2_geometry.h",
                  "paper_2512_24685_amd/csrc/sre2_plan.h"]



def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """SHA-256 of the kernel sources' code: comments and blank space are
    dropped, so that only a change of the code itself retires the stored
    counter figures."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def alg_units(N: int, form: str, kind: str, cs: int):
    """Algorithmic bytes and VALU ops per launch of one kernel class.

    Two-pass slab: every complex value of a shift's (half-)slab is written once
    by pass 1 and read once by pass 2: 8 B (FP32) / 16 B (FP64) per value,
    2^N values per shift (2^(N-1) in the Hermitian-pair forms).
    VALU ops per slab value: pass 1 = 4 (conj product) + 2 per butterfly stage
    over the L row bits; pass 2 = 2 per stage over the remaining bits + 5
    (|W|^2, square in FP64, FP64 add); Hermitian pass 2: + 1 (two squares).
    """
    import paper_2512_24685_amd as sre2

    base = "fp64" if form.startswith("fp64") else "fp32"
    herm = form.endswith("h")
    ns = N - (1 if herm else 0)
    vals = cs * (1 << ns)
    eb = 8 if base == "fp32" else 16
    L = sre2.row_bits(N, form)
    if kind == "pass1":
        return eb * vals, (4 + 2 * L) * vals
    if kind == "pass2":
        return eb * vals, (2 * (ns - L) + (6 if herm else 5)) * vals
    raise ValueError(kind)


def roofline(N, form, kind, ms, launches, cs, traffic, evals=1):
    avg_s = ms / 1e3 / launches
    if kind in ("pass1", "pass2"):
        by, ops = alg_units(N, form, kind, cs)
        gbs = by / avg_s / 1e9
        alu = ops / avg_s
        ent = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
               "kernel": "k_pass1" if kind == "pass1" else "k_pass2",
               "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
               "alg_bytes_per_launch": by, "alu_tops": round(alu / 1e12, 3),
               "alu_frac": round(alu / VALU_PEAK_OPS, 4)}
        return ent
    # fused kernel: every value stays on chip; VALU-bound.  The Hermitian
    # forms run x = 0 as a separate short plain launch, so the work and the
    # time are taken per evaluation (all launches of the class) rather than
    # per launch.
    herm = form.endswith("h")
    nt = N - (1 if herm else 0)
    ops = (4 + 2 * nt + (6 if herm else 5)) * (1 << N) * (1 << nt)
    per_eval_s = ms / 1e3 / evals
    alu = ops / per_eval_s
    return {"bound": "alu", "achieved": round(alu / 1e12, 3), "peak": round(VALU_PEAK_OPS / 1e12, 2),
            "unit": "Tops/s", "frac": round(alu / VALU_PEAK_OPS, 4), "traffic": traffic,
            "kernel": "k_fused", "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
            "class_us_per_evaluation": round(per_eval_s * 1e6, 2),
            "alg_ops_per_evaluation": ops}


def stored_traffic(kernel: str, N: int, form: str):
    """HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, scaled by a plain copy of known size), if they were taken on
    the current kernel sources; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    for r in rec.get("entries", []):
        if r["kernel"] == kernel and r["N"] == N and r["form"] == form:
            if r.get("source_sha") != kernel_source_sha():
                return None
            return r["hbm_bytes_per_launch"]
    return None


def cpu_baseline(psi: np.ndarray, target_s: float):
    import oracle

    N = psi.size.bit_length() - 1
    cores = len(os.sched_getaffinity(0))
    order = np.random.default_rng(1).permutation(1 << N)
    oracle.partials(psi, order[:cores], threads=cores)  # warm-up, not timed
    batch = 4 * cores
    count, dt, pos = 0, 0.0, cores
    while dt < target_s and pos < (1 << N):
        xs = order[pos:pos + batch]
        t0 = time.perf_counter()
        oracle.partials(psi, xs, threads=cores)
        dt += time.perf_counter() - t0
        count += len(xs)
        pos += len(xs)
    return {"value": count * float(1 << N) / dt, "unit": "Pauli strings/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{count} random shifts x of the N={N} state, each a full FP64 FWHT over "
                      f"2^{N} Pauli strings (Algorithm 1 loop body), {dt:.1f} s on {cores} threads"}


SCRATCH_LIMIT = 0  # bytes; 0 keeps the library default
LAST_STEPS = None  # per-step ms (min, median, max) of the last measure()


def new_context(sre2):
    ctx = sre2.Context(0)
    if SCRATCH_LIMIT:
        ctx.set_scratch_limit(SCRATCH_LIMIT)
    return ctx


def measure(sre2, torch, d_psi, form, steps, warmup):
    ctx = new_context(sre2)
    stream = torch.cuda.current_stream()
    for i in range(warmup):
        out, _ = sre2.m2_async(d_psi, form=form, ctx=ctx)
        torch.cuda.synchronize()
        log(f"[{form}] warmup {i}: M2={out[0].item():.10f}")
    ctx.set_timing(True)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    outs = []
    for i in range(steps):
        outs.append(sre2.m2_async(d_psi, form=form, ctx=ctx)[0])
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    elapsed_ms = evs[0].elapsed_time(evs[-1])
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(steps))
    kt = ctx.timing_read()
    ctx.set_timing(False)
    m2s = [o[0].item() for o in outs]
    if len(set(m2s)) != 1:
        raise RuntimeError(f"{form}: results differ between steps: {m2s}")
    cs, P = ctx.chunking(d_psi.numel().bit_length() - 1, form)
    ctx.close()
    log(f"[{form}] {steps} steps: {elapsed_ms:.1f} ms; M2={m2s[0]:.12f}; kernels={kt}")
    global LAST_STEPS
    LAST_STEPS = {"min": round(per_step[0], 3), "median": round(per_step[len(per_step) // 2], 3),
                  "max": round(per_step[-1], 3)}
    return elapsed_ms / steps, m2s[0], kt, cs, P


def copy_calibration(mib: int):
    import torch

    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {mib} MiB ten times ({n * 4} bytes read and written per copy)")


def serving_benchmark(sre2, torch, W, count: int, form: str, load: float = 0.7,
                      n_lo: int = 8, n_hi: int = 18):
    """Poisson stream of `count` requests (N ~ U{n_lo..n_hi}, Haar or graph+T,
    complex64 host states), replayed at the same arrival times against (a)
    one-at-a-time sre2_m2 calls and (b) the continuous-batching server.
    The arrival rate is `load` / (mean one-at-a-time service time)."""
    reqs = W.serving_requests(count, n_min=n_lo, n_max=n_hi)
    states = [W.build_request(r) for r in reqs]
    log(f"serving: {count} requests generated")
    # calibration of the one-at-a-time service time per N
    t_n = {}
    for N in sorted({r["N"] for r in reqs}):
        psi = next(p for p, r in zip(states, reqs) if r["N"] == N)
        best = 1e9
        for _ in range(3):
            t0 = time.perf_counter()
            sre2.m2(torch.from_numpy(psi).to("cuda:0"), form=form)
            best = min(best, time.perf_counter() - t0)
        t_n[N] = best
    mean_service = float(np.mean([t_n[r["N"]] for r in reqs]))
    lam = load / mean_service
    arrivals = np.cumsum(np.random.default_rng(W.SEED_SERVING + 1).exponential(1 / lam, count))
    work = float(sum(4.0 ** r["N"] for r in reqs))

    def wait_until(t):
        while True:
            dt = t - time.perf_counter()
            if dt <= 0:
                return
            time.sleep(min(dt, 0.0005))

    # (a) one request at a time, in arrival order
    base_res, base_lat = [], []
    t0 = time.perf_counter() + 0.05
    for i, psi in enumerate(states):
        wait_until(t0 + arrivals[i])
        r = sre2.m2(torch.from_numpy(psi).to("cuda:0"), form=form)
        base_lat.append(time.perf_counter() - (t0 + arrivals[i]))
        base_res.append(r)
        if (i + 1) % 512 == 0:
            log(f"serving: one-at-a-time {i + 1}/{count}")
    base_makespan = time.perf_counter() - t0
    log(f"serving: one-at-a-time done in {base_makespan:.1f} s")

    # (b) continuous batching
    srv = sre2.Server(form=form, hbm_budget=8 << 30, max_slots=2048)
    tickets, lag = [], []
    done = {}
    t0 = time.perf_counter() + 0.05

    def poll_some():
        for j in range(len(tickets)):
            if j in done:
                continue
            st, res, lat = srv.poll(tickets[j])
            if st >= sre2.REQ_DONE:
                done[j] = (st, res, lat + lag[j])

    for i, psi in enumerate(states):
        while time.perf_counter() < t0 + arrivals[i]:
            poll_some()
            time.sleep(0.0002)
        lag.append(time.perf_counter() - (t0 + arrivals[i]))
        tickets.append(srv.submit(psi))
        if (i + 1) % 512 == 0:
            log(f"serving: server {i + 1}/{count} submitted, {len(done)} done")
    while len(done) < count:
        poll_some()
        time.sleep(0.0002)
    srv_makespan = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    log(f"serving: server done in {srv_makespan:.1f} s; stats={stats}")
    mismatch = sum(1 for j in range(count)
                   if done[j][1].m2 != base_res[j].m2 or done[j][1].S != base_res[j].S)
    srv_lat = [done[j][2] for j in range(count)]

    def pct(v, q):
        return float(np.percentile(np.array(v) * 1e3, q))

    return {
        "requests": count, "N_range": [n_lo, n_hi], "form": form,
        "arrival_rate_per_s": lam, "load_vs_one_at_a_time": load,
        "pauli_strings": work,
        "server": {"throughput_pauli_per_s": work / srv_makespan,
                   "requests_per_s": count / srv_makespan, "makespan_s": srv_makespan,
                   "p50_ms": pct(srv_lat, 50), "p99_ms": pct(srv_lat, 99), "stats": stats},
        "one_at_a_time": {"throughput_pauli_per_s": work / base_makespan,
                          "requests_per_s": count / base_makespan,
                          "makespan_s": base_makespan,
                          "p50_ms": pct(base_lat, 50), "p99_ms": pct(base_lat, 99)},
        "results_bitwise_equal": mismatch == 0, "mismatches": mismatch,
    }


def large_n_benchmark(sre2, torch, W, Ns=(22, 24), forms=("fp32", "split16"),
                      work=2 ** 35):
    """Large slabs: whole two-pass chunks of the full-evaluation launch shape
    (shifts from x = 2^(N-1)) per (N, form), `work` slab values in total
    (about 0.14 s: a timed region of only a few launches reads low, because
    the clocks ramp up after the host's synchronisation), with each pass's
    algorithmic HBM rate and its fraction of the 8 TB/s peak, and the
    full-evaluation time this implies."""
    out = {}
    for N in Ns:
        psi = torch.from_numpy(W.haar(N, W.SEED_LARGE + (0 if N == 22 else 1), np.complex64))
        d = psi.to("cuda:0")
        for form in forms:
            ctx = new_context(sre2)
            cs, P = ctx.chunking(N, form)
            chunks = max(1, work // (cs << N))
            x0 = 1 << (N - 1)
            sre2.shift_partials(d, x0, cs, form=form, ctx=ctx)  # warm-up chunk
            torch.cuda.synchronize()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            sre2.shift_partials(d, x0 + cs, chunks * cs, form=form, ctx=ctx)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            kt = ctx.timing_read()
            ctx.close()
            by, _ = alg_units(N, form, "pass1", cs)
            rec = {"shifts_per_chunk": cs, "chunks_timed": chunks,
                   "row_bits": sre2.row_bits(N, form),
                   "s_per_evaluation": dt / (chunks * cs) * (1 << N)}
            for k in ("pass1", "pass2"):
                ms, n = kt[k]
                gbs = by / (ms / 1e3 / n) / 1e9
                rec[k] = {"avg_launch_us": round(ms / n * 1e3, 1), "achieved_GBs": round(gbs, 1),
                          "frac": round(gbs / HBM_PEAK_GBS, 4)}
            out[f"N{N}_{form}"] = rec
            log(f"large N={N} {form}: {rec}")
    return out


def dynamics_benchmark(sre2, torch, W, N: int, steps: int, form: str):
    """TFIM quench (the paper's first dynamics example) from a random product
    state: M2 after every step (a) through the snapshot pipeline, evolution
    overlapped with evaluation in the serving loop, and (b) step, snapshot,
    evaluate, one after another."""
    P = W.TFIM_PARAMS
    th, ph = W.product_angles(N, W.SEED_LARGE + 7)
    srv = sre2.Server(form=form, hbm_budget=1 << 30, max_slots=64)
    sim = sre2.Simulator(N)
    sim.product_state(th, ph)
    sim.run_tfim(srv, P["J"], P["hx"], P["hz"], P["dt"], 2)  # warm-up
    sim.product_state(th, ph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    piped = sim.run_tfim(srv, P["J"], P["hx"], P["hz"], P["dt"], steps)
    t_pipe = time.perf_counter() - t0
    srv.close()
    sim.product_state(th, ph)
    torch.cuda.synchronize()
    seq = []
    t0 = time.perf_counter()
    for t in range(steps + 1):
        if t:
            sim.tfim_step(P["J"], P["hx"], P["hz"], P["dt"])
        seq.append(sre2.m2(sim.state(torch.complex64), form=form))
    t_seq = time.perf_counter() - t0
    sim.close()
    same = all(a.m2 == b.m2 for a, b in zip(piped, seq))
    return {"model": "TFIM with longitudinal field, open chain", "N": N, "steps": steps,
            "params": P, "form": form, "snapshots": steps + 1,
            "pipelined": {"seconds": t_pipe, "snapshots_per_s": (steps + 1) / t_pipe},
            "sequential": {"seconds": t_seq, "snapshots_per_s": (steps + 1) / t_seq},
            "results_bitwise_equal": same, "M2_first_last": [piped[0].m2, piped[-1].m2]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", default="fp32")
    ap.add_argument("--also", default="fp32h,split16,splitbf16", help="other forms, comma separated")
    ap.add_argument("--N", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB")
    ap.add_argument("--serving", type=int, default=160, metavar="R",
                    help="requests of the serving measurement (0: skip)")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--dynamics", type=int, default=20, metavar="STEPS",
                    help="TFIM quench steps of the snapshot-pipeline measurement (0: skip)")
    ap.add_argument("--dynamics-N", type=int, default=16)
    ap.add_argument("--large", type=int, default=1, help="large-slab measurement (0: skip)")
    ap.add_argument("--scratch-gib", type=float, default=0.0,
                    help="two-pass scratch limit per context in GiB (0: library default)")
    ap.add_argument("--profile-chunks", type=int, default=0, metavar="C",
                    help="run only C two-pass chunks (the benchmark's launch shape) from "
                         "x = 2^(N-1), for counter collection")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the evaluation shards over shifts x with no "
              "communication, so multi-GPU throughput is N x the one-GPU value; "
              "--gpus above 1 is not measured here.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    global SCRATCH_LIMIT
    SCRATCH_LIMIT = int(args.scratch_gib * 2 ** 30)

    import torch

    import paper_2512_24685_amd as sre2
    import workloads as W

    if args.serving_only:
        rec = serving_benchmark(sre2, torch, W, args.serving, "fp32")
        print(json.dumps({"metric": "serving stream: Pauli strings/s and p50/p99 latency",
                          "serving": rec}), flush=True)
        return

    N = args.N
    log(f"bench: N={N} form={args.form} also={args.also} steps={args.steps} warmup={args.warmup}")
    psi = W.haar(N, W.SEED_N20, np.complex64)
    d_psi = torch.from_numpy(psi).to("cuda:0")
    if args.profile_chunks:
        ctx = new_context(sre2)
        cs, _ = ctx.chunking(N, args.form)
        x0 = 1 << (N - 1)
        for c in range(args.profile_chunks):
            sre2.shift_partials(d_psi, x0 + c * cs, cs, form=args.form, ctx=ctx)
            torch.cuda.synchronize()
            log(f"profile chunk {c}: shifts [{x0 + c * cs}, {x0 + (c + 1) * cs})")
        return

    ms_per_step, m2, kt, cs, P = measure(sre2, torch, d_psi, args.form, args.steps, args.warmup)
    step_ms = LAST_STEPS
    value = float(4 ** N) / (ms_per_step / 1e3)
    dom = max((k for k in kt if k != "aux" and kt[k][1] > 0), key=lambda k: kt[k][0])
    kname = {"pass1": "k_pass1", "pass2": "k_pass2", "shift": "k_fused"}[dom]
    roof = roofline(N, args.form, dom, kt[dom][0], kt[dom][1], cs,
                    stored_traffic(kname, N, args.form), evals=args.steps)
    roof["kernels_ms_per_step"] = {k: round(v[0] / args.steps, 3) for k, v in kt.items()}

    forms = {}
    for f in [x for x in args.also.split(",") if x and x != args.form]:
        fsteps_n = max(3, args.steps // 2)
        fms, fm2, fkt, fcs, _ = measure(sre2, torch, d_psi, f, fsteps_n, min(2, args.warmup))
        fsteps = LAST_STEPS
        fdom = max((k for k in fkt if k != "aux" and fkt[k][1] > 0), key=lambda k: fkt[k][0])
        fk = {"pass1": "k_pass1", "pass2": "k_pass2", "shift": "k_fused"}[fdom]
        forms[f] = {"value": float(4 ** N) / (fms / 1e3), "ms_per_step": fms, "step_ms": fsteps,
                    "M2": fm2,
                    "abs_dM2_vs_headline": abs(fm2 - m2),
                    "roofline": roofline(N, f, fdom, fkt[fdom][0], fkt[fdom][1], fcs,
                                         stored_traffic(fk, N, f),
                                         evals=fsteps_n),
                    "kernels_ms_per_step": {k: round(v[0] / fsteps_n, 3)
                                            for k, v in fkt.items()}}
    serving = None
    if args.serving:
        serving = serving_benchmark(sre2, torch, W, args.serving, "fp32")
    large = large_n_benchmark(sre2, torch, W) if args.large else None
    dynamics = None
    if args.dynamics:
        dynamics = dynamics_benchmark(sre2, torch, W, args.dynamics_N, args.dynamics, "fp32")
        log(f"dynamics: {dynamics}")
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
        "dtype": "f64" if args.form.startswith("fp64") else "f32",
        "data": "synthetic",
        "config": {"workload": f"exact M2 of one N={N} Haar-random complex64 state, "
                               f"XOR-FWHT in the {args.form} form (FP64 sums), "
                               + ("two-pass row/column transform through an HBM slab"
                                  if dom != "shift" else
                                  "whole transforms in one workgroup's LDS (fused kernel)"),
                   "N": N, "pauli_strings_per_step": 4 ** N, "form": args.form,
                   "shifts_per_chunk": cs, "column_groups": P, "M2": m2, "step_ms": step_ms},
        "roofline": roof,
        "forms": forms,
        "serving": serving,
        "large_n": large,
        "dynamics": dynamics,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
