"""Throughput benchmark: Pauli strings per second of one exact M2 evaluation,
and every benchmark configuration as its own leg with its measured error.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form fp32]
                    [--also fp32h,split16,splitbf16,fp64,fp64h] [--N 20] [--no-cpu]
    python bench.py --copy-calibration MiB     (plain device copy, for counters)
    python bench.py --form F --profile-chunks C (C two-pass chunks, for counters)

One step = one full evaluation (every shift x, its FWHT, sum |W|^4, the final
reduction and logarithm) of an N=20 Haar-random complex64 state that is
already resident in device memory.  Pauli strings per step = 4^N.

Printed (one JSON line on stdout): throughput of the headline form (plain
FP32 XOR-FWHT) with |dM2| against the stored FP64 oracle value, ms per step,
the dominant kernel's roofline position (timed live with HIP events around
every launch in the timed region; for pass 1 also against the rate a
store-only kernel with its row layout reaches on the same GPU), the other
forms measured the same way,
and one leg per benchmark configuration:
  * N = 10 complex128 states (Haar, |T>^10, graph state), every form, |dM2|
    against the oracle and the closed forms;
  * N = 16 batch (32 Haar + 8 graph+T, complex64) through the packed batched
    path, |dM2| against stored oracle values and the closed forms;
  * N = 20 Haar and graph+T (m = 10) in every form, |dM2| against the stored
    oracle value and the closed form;
  * the serving stream (N ~ U{8..18}) at saturating load (4096 requests) and
    at 0.7 load, server against one-at-a-time calls;
  * N = 22 / 24 two-pass chunks (HBM rates, partials checked against stored
    oracle values) and a timed sample of the N = 20 Ising snapshot sequence;
  * the FP64 CPU oracle timed on this host's cores on bounded samples.
"""
from __future__ import annotations

import argparse
import hashlib
import subprocess
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


def slab_ranges(N: int, form: str, x0: int, xc: int):
    """The two-pass ranges of the shifts [x0, x0 + xc) as the library runs
    them: (slab values per shift, pass-1 row bits, transformed values per
    shift in pass 2, shifts).  Shifts below 2^L take the full slab of 2^N
    values; above (from `sre2_half_slab_first_shift`), the Hermitian-pair
    forms and (row pairs, on by default) the plain and split forms take half
    slabs of 2^(N-1) values; the row pairs still transform 2^N values per
    shift in pass 2."""
    import paper_2512_24685_amd as sre2

    herm = form.endswith("h")
    half = herm or ROW_PAIRS
    Lf = sre2.row_bits(N, "fp64" if form.startswith("fp64") else "fp32")
    if not half:
        return [(1 << N, Lf, 1 << N, xc)]
    Lh = sre2.row_bits(N, form)
    first = sre2.half_slab_first_shift(N, form)
    lo = max(0, min(x0 + xc, first) - x0)
    out = [(1 << N, Lf, 1 << N, lo)] if lo else []
    if xc > lo:
        out.append((1 << (N - 1), Lh, 1 << (N - 1) if herm else 1 << N, xc - lo))
    return out


def alg_totals(N: int, form: str, kind: str, x0: int, xc: int):
    """Algorithmic bytes and VALU ops of one kernel class over the shifts
    [x0, x0 + xc).

    Bytes: every slab value is written once by pass 1 and read once by
    pass 2: 8 B (FP32) / 16 B (FP64) per value (slab_ranges).
    VALU ops per value: pass 1 = 4 (conj product) + 2 per butterfly stage
    over the L row bits, per slab value; pass 2 = 2 per stage over the
    remaining bits + 5 (|W|^2, square in FP64, FP64 add), per transformed
    value; Hermitian pass 2: + 1 (two squares).
    """
    eb = 16 if form.startswith("fp64") else 8
    herm = form.endswith("h")
    by = ops = 0
    for vals, L, tvals, n in slab_ranges(N, form, x0, xc):
        by += eb * vals * n
        if kind == "pass1":
            ops += (4 + 2 * L) * vals * n
        elif kind == "pass2":
            nt = tvals.bit_length() - 1
            ops += (2 * (nt - L) + (6 if herm and vals < 1 << N else 5)) * tvals * n
        else:
            raise ValueError(kind)
    return by, ops


def roofline(N, form, kind, ms, launches, traffic, evals=1, x0=0, xc=None):
    """Roofline entry of one kernel class from its summed time `ms` over
    `launches` launches covering `evals` times the shifts [x0, x0 + xc)
    (default: whole evaluations).  achieved = algorithmic bytes per launch /
    mean launch time (= total bytes / total time: the launches of an
    evaluation differ in size, a full-slab chunk first, then half slabs)."""
    avg_s = ms / 1e3 / launches
    if kind in ("pass1", "pass2"):
        by, ops = alg_totals(N, form, kind, x0, (1 << N) if xc is None else xc)
        by, ops = by * evals, ops * evals
        tot_s = ms / 1e3
        gbs = by / tot_s / 1e9
        alu = ops / tot_s
        ent = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
               "kernel": "k_pass1" if kind == "pass1" else "k_pass2",
               "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
               "alg_bytes_per_launch": round(by / launches), "alu_tops": round(alu / 1e12, 3),
               "alu_frac": round(alu / VALU_PEAK_OPS, 4)}
        if alu / VALU_PEAK_OPS > gbs / HBM_PEAK_GBS:
            # closer to its arithmetic roof than to HBM (the row-pair pass 2):
            # report it against the VALU issue rate, HBM figures beside
            ent.update(bound="alu", achieved=round(alu / 1e12, 3),
                       peak=round(VALU_PEAK_OPS / 1e12, 2), unit="Tops/s",
                       frac=round(alu / VALU_PEAK_OPS, 4), alg_ops_per_launch=round(ops / launches),
                       hbm_GBs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
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


def store_ceiling():
    """Rate of a store-only kernel with pass 1's exact row layout (32 KiB per
    256-thread workgroup, 8-byte non-temporal stores in pass 1's lane order:
    `probe_store` pattern A), measured now on this GPU in a child process;
    the median of three rounds in GB/s, or None if the probe is not built or
    fails."""
    exe = os.path.join(ROOT, "paper_2512_24685_amd", "probe_store")
    if not os.path.exists(exe):
        return None
    try:
        out = subprocess.run([exe, "A", "3"], capture_output=True, text=True, timeout=120)
    except (OSError, subprocess.TimeoutExpired):
        return None
    rates = [float(m) for m in re.findall(r"pattern A\s+\S+ ms per 4 GiB, ([0-9.]+) TB/s", out.stdout)]
    if out.returncode != 0 or not rates:
        return None
    return round(1000.0 * sorted(rates)[len(rates) // 2], 1)


def cpu_model() -> str:
    """The host CPU's model name, family / model numbers and logical CPU count
    (from /proc/cpuinfo, as lscpu reports them)."""
    fields = {}
    count = 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key == "processor":
                    count += 1
                elif key in ("model name", "cpu family", "model") and key not in fields:
                    fields[key] = val.strip()
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    return (f"{name} (family {fields.get('cpu family', '?')}, model {fields.get('model', '?')}; "
            f"{count} logical CPUs on the host)")


def cpu_baseline(psi: np.ndarray, target_s: float, n10=None, n16=None):
    """The FP64 CPU oracle, as it stands, on this host's cores.

    * Headline: random shifts x of the N = 20 state, one FP64 FWHT over 2^20
      Pauli strings each (Algorithm 1's loop body), for about target_s, scaled
      to Pauli strings per second.
    * N = 10 states: one full oracle evaluation each (also the reference M2
      of the N = 10 leg).
    * N = 16: a full oracle evaluation of `n16` (sample states of the batch).
    """
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
    rec = {"value": count * float(1 << N) / dt, "unit": "Pauli strings/s", "cores": cores,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{count} random shifts x of the N={N} state, each a full FP64 FWHT over "
                     f"2^{N} Pauli strings (Algorithm 1 loop body), {dt:.1f} s on {cores} threads"}
    refs = {}
    per = {}
    for name, p in (n10 or []):
        t0 = time.perf_counter()
        refs[name] = oracle.m2(p, threads=cores)
        per[name] = time.perf_counter() - t0
    if n10:
        rec["n10_seconds_per_state"] = {k: round(v, 4) for k, v in per.items()}
    if n16:
        ts = []
        for name, p in n16:
            t0 = time.perf_counter()
            S, n = oracle.total(p, threads=cores)
            ts.append(time.perf_counter() - t0)
            refs[name] = oracle.m2_from_total(S, n, p.size.bit_length() - 1)
        rec["n16_seconds_per_state"] = round(float(np.mean(ts)), 3)
        rec["n16_sample"] = f"{len(n16)} of the 40 batch states, full evaluation each"
        rec["n16_pauli_per_s"] = float(4 ** 16) / float(np.mean(ts))
    return rec, refs


def golden():
    """Stored FP64 oracle values (written by tests/golden/make_golden.py from
    the oracle alone), keyed by case with the SHA-256 of their input bytes."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def stored_m2(g, name, psi):
    rec = g.get(name)
    return rec["m2"] if rec and rec.get("sha256") == sha256(psi) else None


SCRATCH_LIMIT = 0  # bytes; 0 keeps the library default
ROW_PAIRS = True  # row-pair half slabs of the plain forms (library default)
LAST_STEPS = None  # per-step ms (min, median, max) of the last measure()


def new_context(sre2):
    ctx = sre2.Context(0)
    if SCRATCH_LIMIT:
        ctx.set_scratch_limit(SCRATCH_LIMIT)
    if not ROW_PAIRS:
        ctx.set_row_pairs(False)
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


def serving_benchmark(sre2, torch, W, reqs, states, form: str, load: float,
                      n_lo: int = 8, n_hi: int = 18, t_n=None):
    """Poisson stream of the given requests (N ~ U{n_lo..n_hi}, Haar or
    graph+T, complex64 host states), replayed at the same arrival times
    against (a) one-at-a-time sre2_m2 calls and (b) the continuous-batching
    server.  The arrival rate is `load` / (mean one-at-a-time service time):
    load > 1 saturates the GPU, so throughput is GPU-bound.  Latency is from
    the scheduled arrival to the result on the host."""
    count = len(reqs)
    if t_n is None:
        t_n = service_times(sre2, torch, reqs, states, form)
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
            log(f"serving load {load}: one-at-a-time {i + 1}/{count}")
    base_makespan = time.perf_counter() - t0
    log(f"serving load {load}: one-at-a-time done in {base_makespan:.1f} s")

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
            log(f"serving load {load}: server {i + 1}/{count} submitted, {len(done)} done")
    while len(done) < count:
        poll_some()
        time.sleep(0.0002)
    srv_makespan = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    log(f"serving load {load}: server done in {srv_makespan:.1f} s; stats={stats}")
    mismatch = sum(1 for j in range(count)
                   if done[j][1].m2 != base_res[j].m2 or done[j][1].S != base_res[j].S)
    srv_lat = [done[j][2] for j in range(count)]
    fmax = 14 if not form.startswith("fp64") else 13
    small = [j for j in range(count) if reqs[j]["N"] <= fmax]
    large = [j for j in range(count) if reqs[j]["N"] > fmax]

    def pct(v, q):
        return float(np.percentile(np.array(v) * 1e3, q)) if len(v) else None

    def lane(lat, idx):
        return {"p50_ms": pct([lat[j] for j in idx], 50), "p99_ms": pct([lat[j] for j in idx], 99)}

    return {
        "requests": count, "N_range": [n_lo, n_hi], "form": form,
        "arrival_rate_per_s": lam, "load_vs_one_at_a_time": load,
        "pauli_strings": work,
        "server": {"throughput_pauli_per_s": work / srv_makespan,
                   "requests_per_s": count / srv_makespan, "makespan_s": srv_makespan,
                   "p50_ms": pct(srv_lat, 50), "p99_ms": pct(srv_lat, 99),
                   "small_N": lane(srv_lat, small), "large_N": lane(srv_lat, large),
                   "stats": stats},
        "one_at_a_time": {"throughput_pauli_per_s": work / base_makespan,
                          "requests_per_s": count / base_makespan,
                          "makespan_s": base_makespan,
                          "p50_ms": pct(base_lat, 50), "p99_ms": pct(base_lat, 99),
                          "small_N": lane(base_lat, small), "large_N": lane(base_lat, large)},
        "results_bitwise_equal": mismatch == 0, "mismatches": mismatch,
    }


def service_times(sre2, torch, reqs, states, form):
    """Calibration: the best of three one-at-a-time service times per N."""
    t_n = {}
    for N in sorted({r["N"] for r in reqs}):
        psi = next(p for p, r in zip(states, reqs) if r["N"] == N)
        best = 1e9
        for _ in range(3):
            t0 = time.perf_counter()
            sre2.m2(torch.from_numpy(psi).to("cuda:0"), form=form)
            best = min(best, time.perf_counter() - t0)
        t_n[N] = best
    return t_n


def serving_legs(sre2, torch, W, count_sat: int, count_07: int, form: str):
    """The serving configuration: `count_sat` requests at 4x the one-at-a-time
    service rate (saturating) and the first `count_07` at 0.7 of it."""
    n = max(count_sat, count_07)
    reqs = W.serving_requests(n)
    states = [W.build_request(r) for r in reqs]
    log(f"serving: {n} requests generated")
    t_n = service_times(sre2, torch, reqs, states, form)
    out = {}
    if count_sat:
        out["saturating"] = serving_benchmark(sre2, torch, W, reqs[:count_sat],
                                              states[:count_sat], form, 4.0, t_n=t_n)
    if count_07:
        out["load_0.7"] = serving_benchmark(sre2, torch, W, reqs[:count_07],
                                            states[:count_07], form, 0.7, t_n=t_n)
    return out


def large_n_benchmark(sre2, torch, W, Ns=(22, 24), forms=("fp32", "split16"),
                      work=2 ** 35):
    """Large slabs: whole two-pass chunks of the full-evaluation launch shape
    per (N, form), `work` slab values in total (about 0.14 s: a timed region
    of only a few launches reads low, because the clocks ramp up after the
    host's synchronisation), with each pass's algorithmic HBM rate and its
    fraction of the 8 TB/s peak, and the full-evaluation time this implies.
    The timed range is placed over stored oracle shifts of the same state
    (tests/golden), and the partials computed there are checked against them
    (relative 1e-4, the FP32 per-shift bar)."""
    g = golden()
    out = {}
    for N in Ns:
        name = f"haar{N}_sampled"
        psi_np = W.haar(N, W.SEED_LARGE + (0 if N == 22 else 1), np.complex64)
        rec = g.get(name)
        ref = dict(zip(rec["shifts"], rec["partials"])) if rec and \
            rec.get("sha256") == sha256(psi_np) else {}
        d = torch.from_numpy(psi_np).to("cuda:0")
        for form in forms:
            ctx = new_context(sre2)
            cs, P = ctx.chunking(N, form)
            chunks = max(1, work // (cs * slab_ranges(N, form, 1 << (N - 1), 1)[0][0]))
            span = chunks * cs
            # the chunk-aligned range of `span` shifts holding the most stored shifts
            starts = sorted({(x // cs) * cs for x in ref if x >= 2 * cs})
            best, x0 = -1, 1 << (N - 1)
            for st in starts:
                st = min(st, (1 << N) - span)
                k = sum(1 for x in ref if st <= x < st + span)
                if k > best:
                    best, x0 = k, st
            sre2.shift_partials(d, x0 - cs, cs, form=form, ctx=ctx)  # warm-up chunk
            torch.cuda.synchronize()
            ctx.set_timing(True)
            t0 = time.perf_counter()
            part = sre2.shift_partials(d, x0, span, form=form, ctx=ctx)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            kt = ctx.timing_read()
            ctx.close()
            got = part.cpu().numpy()
            xs = [x for x in ref if x0 <= x < x0 + span]
            errs = [abs(got[x - x0] - ref[x]) / ref[x] for x in xs]
            if errs and max(errs) > 1e-4:
                raise RuntimeError(f"N={N} {form}: partials off the stored oracle values "
                                   f"(max rel {max(errs):.3g})")
            by, _ = alg_totals(N, form, "pass1", x0, span)
            r = {"shifts_per_chunk": cs, "chunks_timed": chunks, "x_begin": x0,
                 "row_bits": sre2.row_bits(N, form),
                 "s_per_evaluation": dt / span * (1 << N),
                 "oracle_checked_shifts": len(xs),
                 "max_rel_err_vs_oracle": max(errs) if errs else None}
            for k in ("pass1", "pass2"):
                ms, n = kt[k]
                gbs = by / (ms / 1e3) / 1e9
                r[k] = {"avg_launch_us": round(ms / n * 1e3, 1), "achieved_GBs": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
            out[f"N{N}_{form}"] = r
            log(f"large N={N} {form}: {r}")
    return out


def n10_leg(sre2, torch, W, forms, reps=50):
    """The N = 10 complex128 states (Haar, |T>^10, graph state) in every form:
    mean device time per evaluation over `reps` back-to-back evaluations and
    the M2 of each (compared with the oracle after the CPU leg)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    for name, psi, closed in W.workload_inputs("n10_small"):
        d = torch.from_numpy(psi).to("cuda:0")
        for form in forms:
            o, _ = sre2.m2_async(d, form=form)
            torch.cuda.synchronize()
            ev[0].record()
            for _ in range(reps):
                o, _ = sre2.m2_async(d, form=form)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            m2 = o[0].item()
            out.setdefault(name, {"closed_form": closed})[form] = {
                "M2": m2, "ms_per_eval": round(ms, 4),
                "pauli_per_s": float(4 ** 10) / (ms / 1e3),
                "abs_dM2_vs_closed_form": abs(m2 - closed) if closed is not None else None}
    return out


def n16_leg(sre2, torch, W, forms, reps=3):
    """The N = 16 batch (32 Haar + 8 graph+T, complex64) through the packed
    batched path, per form: device time of one batch and the largest |dM2|
    against the stored oracle values (Haar) and the closed forms (graph+T)."""
    g = golden()
    inputs = W.workload_inputs("n16_batch")
    ds = [torch.from_numpy(p).to("cuda:0") for _, p, _ in inputs]
    refs = [closed if closed is not None else stored_m2(g, f"haar16_batch_{i}", p)
            for i, (_, p, closed) in enumerate(inputs)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = {}
    for form in forms:
        sre2.m2_batched(ds, form=form)
        torch.cuda.synchronize()
        ev[0].record()
        for _ in range(reps):
            res = sre2.m2_batched(ds, form=form)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        errs = [abs(r.m2 - ref) for r, ref in zip(res, refs) if ref is not None]
        out[form] = {"states": len(ds), "ms_per_batch": round(ms, 3),
                     "pauli_per_s": len(ds) * float(4 ** 16) / (ms / 1e3),
                     "checked": len(errs), "max_abs_dM2": max(errs) if errs else None}
        log(f"n16 batch {form}: {out[form]}")
    return out


def n20_graph_t_leg(sre2, torch, W, forms):
    """The N = 20 graph + T state (m = 10), one evaluation per form, against
    its closed form 10 log2(4/3) (Clifford invariance and additivity)."""
    _, psi, closed = W.workload_inputs("n20_single")[1]
    d = torch.from_numpy(psi).to("cuda:0")
    out = {"closed_form": closed}
    for form in forms:
        t0 = time.perf_counter()
        r = sre2.m2(d, form=form)
        out[form] = {"M2": r.m2, "abs_dM2_vs_closed_form": abs(r.m2 - closed),
                     "seconds": round(time.perf_counter() - t0, 3)}
        log(f"graph+T N=20 {form}: {out[form]}")
    return out


def n20_snapshot_leg(sre2, torch, W, forms=("fp32", "fp32h"), ts=(5, 16, 21, 37)):
    """A timed sample of the 64-snapshot N = 20 Ising sequence
    psi_t = diag(exp(i pi t/64 h)) H^N |0>: seconds per snapshot, with
    |dM2| against the stored oracle values (t = 5, 21), the Clifford point
    (t = 16, M2 = 0) and the period (M2(37) = M2(5))."""
    g = golden()
    N = 20
    J = W.snapshot_couplings(N)
    h = W.ising_energy(N, J)
    out = {}
    for form in forms:
        m, secs = {}, []
        for t in ts:
            psi = W.ising_snapshot(N, t, J, dtype=np.complex64, energy=h)
            d = torch.from_numpy(psi).to("cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m[t] = sre2.m2(d, form=form).m2
            secs.append(time.perf_counter() - t0)
            ref = stored_m2(g, f"ising20_t{t}", psi)
            if ref is not None:
                m[f"abs_dM2_vs_oracle_t{t}"] = abs(m[t] - ref)
        out[form] = {"M2": {str(k): v for k, v in m.items()},
                     "seconds_per_snapshot": round(float(np.mean(secs)), 3),
                     "snapshots_timed": len(ts),
                     "abs_M2_clifford_t16": abs(m[16]) if 16 in m else None,
                     "abs_dM2_period_t37_t5": abs(m[37] - m[5]) if 37 in m and 5 in m else None,
                     "sequence_64_estimate_s": round(64 * float(np.mean(secs)), 1)}
        log(f"snapshots {form}: {out[form]}")
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
    ap.add_argument("--also", default="fp32h,split16,splitbf16,fp64,fp64h",
                    help="other forms at N = 20, comma separated")
    ap.add_argument("--form-steps", type=int, default=3, help="timed steps of each other form")
    ap.add_argument("--N", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB")
    ap.add_argument("--mall-probe", action="store_true",
                    help="run the memory-hierarchy probe (L2 / MALL / HBM ping-pong)")
    ap.add_argument("--serving", type=int, default=4096, metavar="R",
                    help="requests of the saturating serving leg (0: skip)")
    ap.add_argument("--serving-07", type=int, default=1024, metavar="R",
                    help="requests of the serving leg at 0.7 load (0: skip)")
    ap.add_argument("--serving-form", default="fp32h")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--configs", type=int, default=1,
                    help="N = 10, N = 16 batch, N = 20 graph+T and snapshot legs (0: skip)")
    ap.add_argument("--dynamics", type=int, default=20, metavar="STEPS",
                    help="TFIM quench steps of the snapshot-pipeline measurement (0: skip)")
    ap.add_argument("--dynamics-N", type=int, default=16)
    ap.add_argument("--large", type=int, default=1, help="large-slab measurement (0: skip)")
    ap.add_argument("--scratch-gib", type=float, default=0.0,
                    help="two-pass scratch limit per context in GiB (0: library default)")
    ap.add_argument("--no-row-pairs", action="store_true",
                    help="full slabs in the plain FP32 / FP64 forms (for comparison; results "
                         "are bitwise the same)")
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
    if args.mall_probe:
        exe = os.path.join(ROOT, "paper_2512_24685_amd", "probe_mall")
        if not os.path.exists(exe):
            sys.exit("probe_mall is not built: run python -m paper_2512_24685_amd.build")
        sys.exit(subprocess.run([exe]).returncode)
    global SCRATCH_LIMIT, ROW_PAIRS
    SCRATCH_LIMIT = int(args.scratch_gib * 2 ** 30)
    ROW_PAIRS = not args.no_row_pairs

    import torch

    import paper_2512_24685_amd as sre2
    import workloads as W

    t_start = time.perf_counter()
    if args.serving_only:
        rec = serving_legs(sre2, torch, W, args.serving, args.serving_07, args.serving_form)
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

    g = golden()
    ref20 = stored_m2(g, "haar20", psi) if N == 20 else None
    ms_per_step, m2, kt, cs, P = measure(sre2, torch, d_psi, args.form, args.steps, args.warmup)
    step_ms = LAST_STEPS
    value = float(4 ** N) / (ms_per_step / 1e3)
    dom = max((k for k in kt if k != "aux" and kt[k][1] > 0), key=lambda k: kt[k][0])
    kname = {"pass1": "k_pass1", "pass2": "k_pass2", "shift": "k_fused"}[dom]
    roof = roofline(N, args.form, dom, kt[dom][0], kt[dom][1],
                    stored_traffic(kname, N, args.form), evals=args.steps)
    roof["kernels_ms_per_step"] = {k: round(v[0] / args.steps, 3) for k, v in kt.items()}
    if args.form in ("fp32", "fp64"):
        # the whole evaluation in algorithmic VALU operations of the plain
        # transform: (2N + 7) per Pauli string (4 for the conjugate product,
        # 2 per butterfly stage, 3 for |W|^2 and its square; the FP64
        # accumulation not counted) against the non-packed issue rate
        roof["evaluation_alu_frac"] = round((2 * N + 7) * 4.0 ** N / (ms_per_step / 1e3)
                                            / VALU_PEAK_OPS, 4)
    if dom == "pass2" and kt["pass1"][1] > 0:
        # the other pass beside the dominant one
        p1 = roofline(N, args.form, "pass1", kt["pass1"][0], kt["pass1"][1],
                      stored_traffic("k_pass1", N, args.form), evals=args.steps)
        roof["pass1"] = {k: p1[k] for k in ("bound", "achieved", "unit", "frac", "avg_launch_us",
                                            "alu_frac", "traffic")}
    p1_gbs = roof["achieved"] if kname == "k_pass1" else roof.get("pass1", {}).get("achieved")
    if p1_gbs and args.form in ("fp32", "fp32h", "split16", "splitbf16"):
        ceil = store_ceiling()
        if ceil:
            roof["store_ceiling"] = {"what": "store-only kernel with pass 1's row layout "
                                             "(probe_store pattern A, this GPU, now); frac = "
                                             "k_pass1's algorithmic rate over it",
                                     "GBs": ceil, "frac": round(p1_gbs / ceil, 4)}

    forms = {}
    all_forms = [args.form] + [x for x in args.also.split(",") if x and x != args.form]
    for f in all_forms[1:]:
        fsteps_n = max(1, args.form_steps)
        fms, fm2, fkt, fcs, _ = measure(sre2, torch, d_psi, f, fsteps_n, 1)
        fsteps = LAST_STEPS
        fdom = max((k for k in fkt if k != "aux" and fkt[k][1] > 0), key=lambda k: fkt[k][0])
        fk = {"pass1": "k_pass1", "pass2": "k_pass2", "shift": "k_fused"}[fdom]
        forms[f] = {"value": float(4 ** N) / (fms / 1e3), "ms_per_step": fms, "step_ms": fsteps,
                    "M2": fm2,
                    "abs_dM2_vs_oracle": abs(fm2 - ref20) if ref20 is not None else None,
                    "abs_dM2_vs_headline": abs(fm2 - m2),
                    "roofline": roofline(N, f, fdom, fkt[fdom][0], fkt[fdom][1],
                                         stored_traffic(fk, N, f), evals=fsteps_n),
                    "kernels_ms_per_step": {k: round(v[0] / fsteps_n, 3)
                                            for k, v in fkt.items()}}
        log(f"[{f}] {forms[f]['ms_per_step']:.1f} ms per step")
    configs = {}
    n10_inputs = n16_sample = None
    if args.configs and N == 20:
        configs["n20_graph_t_m10"] = n20_graph_t_leg(sre2, torch, W, all_forms)
        configs["n10"] = n10_leg(sre2, torch, W, all_forms)
        configs["n16_batch"] = n16_leg(sre2, torch, W,
                                       ["fp32", "fp32h", "split16", "splitbf16", "fp64"])
        configs["n20_snapshots"] = n20_snapshot_leg(sre2, torch, W)
        # configuration ids and seeds (workloads/configs.json) of the legs
        for leg, name in (("n10", "n10_small"), ("n16_batch", "n16_batch"),
                          ("n20_graph_t_m10", "n20_single"), ("n20_snapshots", "n22_n24_large")):
            if isinstance(configs.get(leg), dict):
                c = next(c for c in W.CONFIGS["configs"] if c["name"] == name)
                configs[leg]["config_id"] = c["id"]
                configs[leg]["seed"] = W.CONFIGS["base_seed"] + c["seed_offset"]
        n10_inputs = [(name, p) for name, p, _ in W.workload_inputs("n10_small")]
        n16_sample = [(f"haar16_{i}", W.haar(16, W.SEED_N16_BATCH * 1000 + i, np.complex64))
                      for i in (0, 1)]
    large = large_n_benchmark(sre2, torch, W) if args.large else None
    if large is not None:
        large.update(config_id=5, seed=W.SEED_LARGE)
    serving = None
    if args.serving or args.serving_07:
        serving = serving_legs(sre2, torch, W, args.serving, args.serving_07, args.serving_form)
        serving.update(config_id=4, seed=W.SEED_SERVING)
    dynamics = None
    if args.dynamics:
        dynamics = dynamics_benchmark(sre2, torch, W, args.dynamics_N, args.dynamics, "fp32")
        log(f"dynamics: {dynamics}")
    cpu = None
    if not args.no_cpu:
        log("cpu baseline: timing the FP64 oracle on samples of the workloads ...")
        cpu, refs = cpu_baseline(psi, args.cpu_seconds, n10_inputs, n16_sample)
        log(f"cpu baseline: {cpu}")
        for name, rec in configs.get("n10", {}).items():
            if name in refs:
                rec["oracle_M2"] = refs[name]
                for f in all_forms:
                    rec[f]["abs_dM2_vs_oracle"] = abs(rec[f]["M2"] - refs[name])
        if n16_sample:
            cpu["n16_sample_matches_stored"] = all(
                abs(refs[nm] - (stored_m2(g, f"haar16_batch_{nm.split('_')[1]}", p) or np.nan))
                < 1e-12 for nm, p in n16_sample)
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
                   "config_id": 3, "seed": W.SEED_N20,
                   "N": N, "pauli_strings_per_step": 4 ** N, "form": args.form,
                   "shifts_per_chunk": cs, "column_groups": P, "M2": m2,
                   "abs_dM2_vs_oracle": abs(m2 - ref20) if ref20 is not None else None,
                   "step_ms": step_ms},
        "roofline": roof,
        "forms": forms,
        "configs": configs,
        "serving": serving,
        "large_n": large,
        "dynamics": dynamics,
        "cpu_baseline": cpu,
        "bench_seconds": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
