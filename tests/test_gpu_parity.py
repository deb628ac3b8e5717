"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (bars of the method's two precisions):
  * FP64 form:  |dM2| <= 1e-9, per-shift S_x relative <= 1e-11.
  * FP32 form:  |dM2| <= 1e-5, per-shift S_x relative <= 1e-4 (FP32 butterflies
    over up to 26 stages; S_x = sum |W|^4 is dominated by the largest |W|,
    whose relative error is a few FP32 ulps times sqrt(N)).
The oracle always receives the exact bytes the GPU receives, upcast to FP64.
Sizes: every N from 1 to 16 in full; N = 20 (the benchmark state) in full
against the stored oracle M2 and per-shift sums; N = 22 and 24 on stored
sampled shifts and on one full default chunk (the launch shape of a full
evaluation: shifts per chunk from the context's chunking, slab offsets over
the whole chunk); N = 26 (the largest FP32 slab) on one shift computed here.

A per-shift relative bar does not bound M2: |dM2| = |dS / S| / ln 2 to first
order, so the sum over a chunk is held to the M2 bar times ln 2 as well.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2512_24685_amd as sre2  # noqa: E402

LOG43 = np.log2(4.0 / 3.0)
TOL_M2 = {"fp32": 1e-5, "fp64": 1e-9, "fp32h": 1e-5, "fp64h": 1e-9, "split16": 1e-5,
          "splitbf16": 1e-5}
TOL_SX = {"fp32": 1e-4, "fp64": 1e-11, "fp32h": 1e-4, "fp64h": 1e-11, "split16": 1e-4,
          "splitbf16": 1e-4}
FORMS = ["fp32", "fp64", "fp32h", "fp64h", "split16", "splitbf16"]
# relative error of a sum of S_x that keeps its share of M2 within TOL_M2
TOL_SUM = {f: TOL_M2[f] * np.log(2.0) for f in TOL_M2}
# Closed forms on complex64 inputs: the amplitude rounding alone moves M2 by
# < 1e-6; the split forms' 22-bit (FP16) and 16-bit (BF16) hi/lo values add
# up to their 1e-5 bound.
CLOSED_TOL = {"split16": 1e-5, "splitbf16": 1e-5}


def closed_tol(form):
    return CLOSED_TOL.get(form, 1e-6)


def is64(form):
    return form.startswith("fp64")


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")


def dev(psi):
    return torch.from_numpy(np.ascontiguousarray(psi)).to("cuda")


def case_id(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sre2.lib()


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N", list(range(1, 17)))
def test_haar_m2_and_partials(oracle_mod, form, N):
    dtype = np.complex128 if is64(form) else np.complex64
    psi = W.haar(N, 1000 + N, dtype)
    case_id("haar", N, form)
    r = sre2.m2(dev(psi), form=form, partials=True)
    S_ref, n_ref = oracle_mod.total(psi)
    m_ref = oracle_mod.m2_from_total(S_ref, n_ref, N)
    assert r.status == 0
    assert abs(r.m2 - m_ref) <= TOL_M2[form], (r.m2, m_ref)
    assert abs(r.n - n_ref) <= 1e-12 * n_ref
    Sx = r.partials.cpu().numpy()
    ref = oracle_mod.partials(psi)
    rel = np.max(np.abs(Sx - ref) / ref)
    assert rel <= TOL_SX[form], rel


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dtype", [np.complex64, np.complex128])
def test_input_dtype_conversion(oracle_mod, form, dtype):
    for N in (9, 15):
        psi = W.haar(N, 77, dtype)
        case_id("dtype", N, form, np.dtype(dtype).name)
        r = sre2.m2(dev(psi), form=form)
        ref = oracle_mod.m2(psi)
        assert abs(r.m2 - ref) <= TOL_M2[form]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N", [2, 4, 5, 6, 10, 14, 16])
def test_closed_forms(form, N):
    case_id("closed", N, form)
    r = sre2.m2(dev(W.t_product(N, np.complex64)), form=form)
    assert abs(r.m2 - N * LOG43) <= closed_tol(form)
    r = sre2.m2(dev(W.t_product(N, np.complex128)), form=form)
    assert abs(r.m2 - N * LOG43) <= (1e-12 if is64(form) else closed_tol(form))
    g = sre2.m2(dev(W.graph(N, 900 + N, dtype=np.complex64)), form=form)
    if N % 2 == 0:
        assert g.m2 == 0.0  # every value is an exact dyadic in every form
    else:
        assert abs(g.m2) <= closed_tol(form)
    m = min(N, 5)
    psi, _ = W.graph_t(N, m, 50 + N, dtype=np.complex64)
    r = sre2.m2(dev(psi), form=form)
    assert abs(r.m2 - m * LOG43) <= closed_tol(form)


def test_scale_invariance_and_bad_inputs(oracle_mod):
    psi = W.haar(12, 5)
    case_id("scale")
    a = sre2.m2(dev(psi * (3.0 - 1.0j)), form="fp64")
    assert abs(a.m2 - oracle_mod.m2(psi)) <= 1e-9
    z = sre2.m2(dev(np.zeros(1 << 8, np.complex64)))
    assert z.status == 1 and np.isnan(z.m2)
    bad = W.haar(8, 1, np.complex64)
    bad[3] = np.nan
    b = sre2.m2(dev(bad))
    assert b.status == 1 and np.isnan(b.m2)
    inf = W.haar(16, 1, np.complex64)
    inf[5] = np.inf
    assert sre2.m2(dev(inf)).status == 1


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N,x0,xc", [(3, 1, 5), (9, 0, 301), (13, 4095, 3), (15, 100, 37),
                                     (15, 4000, 200), (17, 65530, 6), (16, 0, 5000)])
def test_shift_ranges_ragged(oracle_mod, form, N, x0, xc):
    psi = W.haar(N, 3 + N, np.complex64)
    case_id("range", N, x0, xc, form)
    got = sre2.shift_partials(dev(psi), x0, xc, form=form).cpu().numpy()
    ref = oracle_mod.partials(psi, np.arange(x0, x0 + xc))
    assert np.max(np.abs(got - ref) / ref) <= TOL_SX[form]


def test_shard_sum_equals_whole():
    """Per-GPU shift shards (design of the multi-GPU split) add up to S."""
    psi = dev(W.haar(16, 8, np.complex64))
    case_id("shards")
    r = sre2.m2(psi)
    parts = [sre2.shift_partials(psi, g << 13, 1 << 13).double().sum().item() for g in range(8)]
    assert abs(sum(parts) - r.S) <= 1e-12 * r.S


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16"])
def test_determinism_and_batched(form):
    # N = 12..14 with two N = 14 states: packed launches of the one-shift
    # fused tiles, whose workgroups loop over several tiles each
    psis = [dev(W.haar(N, 60 + N + 100 * j, np.complex64))
            for N, j in ((3, 0), (8, 0), (12, 0), (13, 0), (14, 0), (14, 1), (15, 0), (16, 0))]
    case_id("determinism", form)
    single = [sre2.m2(p, form=form) for p in psis]
    again = [sre2.m2(p, form=form) for p in psis]
    batch = sre2.m2_batched(psis, form=form)
    for a, b, c in zip(single, again, batch):
        assert a.m2 == b.m2 and a.S == b.S
        assert a.m2 == c.m2 and a.S == c.S


@pytest.mark.parametrize("N", [8, 13, 16, 18])
def test_hermitian_pair_agrees_with_plain(N):
    psi = dev(W.haar(N, 90 + N, np.complex128))
    case_id("herm-vs-plain", N)
    a = sre2.shift_partials(psi, form="fp64").cpu().numpy()
    b = sre2.shift_partials(psi, form="fp64h").cpu().numpy()
    assert np.max(np.abs(a - b) / a) <= 1e-12


def test_scratch_limit_does_not_change_result():
    psi = dev(W.haar(17, 4, np.complex64))
    case_id("scratch-limit")
    a = sre2.m2(psi)
    ctx = sre2.Context(0)
    ctx.set_scratch_limit(1 << 20)  # one slab at a time
    b = sre2.m2(psi, ctx=ctx)
    ctx.close()
    assert a.m2 == b.m2 and a.S == b.S  # chunking never changes the summation order


def test_scratch_fallback_when_allocation_fails(monkeypatch):
    """A device that cannot hold the default slab (allocations above 4 GiB
    fail here) gets smaller chunks, with bitwise the same result."""
    psi = dev(W.haar(18, 6, np.complex64))  # 2 MiB per shift: 8 GiB chunks by default
    case_id("scratch-fallback")
    a = sre2.m2(psi)
    ctx = sre2.Context(0)
    ctx.set_timing(True)
    monkeypatch.setenv("SRE2_FAULT", "alloc_4g")
    b = sre2.m2(psi, ctx=ctx)
    launches = ctx.timing_read()["pass1"][1]
    ctx.close()
    assert a.m2 == b.m2 and a.S == b.S
    # 4 GiB chunks: 2048 full slabs of 2 MiB below 2^12, then row-pair half
    # slabs of 1 MiB, 4096 shifts per chunk (at most 2^12)
    assert launches == 4096 // 2048 + ((1 << 18) - 4096) // 4096


@pytest.mark.parametrize("form,N", [("fp32", 15), ("fp32", 17), ("fp32", 20), ("fp64", 14),
                                    ("fp64", 16), ("fp64", 19)])
def test_row_pairs_bitwise_equal_full_slab(form, N):
    """The row-pair half slabs (default) against the full slab (row pairs
    off): every S_x, S and M2 bit for bit, over whole evaluations that span
    the full-slab shifts below 2^L and the half-slab shifts above."""
    c128 = is64(form)
    psi = dev(W.haar(N, 300 + N, np.complex128 if c128 else np.complex64))
    case_id("row-pairs", form, N)
    on, off = sre2.Context(0), sre2.Context(0)
    off.set_row_pairs(False)
    try:
        a = sre2.shift_partials(psi, form=form, ctx=on).cpu().numpy()
        b = sre2.shift_partials(psi, form=form, ctx=off).cpu().numpy()
        assert np.array_equal(a, b)
        ra, rb = sre2.m2(psi, form=form, ctx=on), sre2.m2(psi, form=form, ctx=off)
        assert ra.m2 == rb.m2 and ra.S == rb.S
    finally:
        on.close()
        off.close()


@pytest.mark.parametrize("form", ["fp32", "fp64"])
def test_row_pairs_ragged_ranges_and_small_chunks(oracle_mod, form):
    """Shift ranges that start inside a block of 2^L shifts and cross
    several of them, with a scratch limit that leaves chunks of a few
    shifts: the row-pair chunks split at every block edge, bit for bit the
    full slab's S_x and within the bar of the oracle."""
    N = 16
    c128 = is64(form)
    psi_np = W.haar(N, 611, np.complex128 if c128 else np.complex64)
    psi = dev(psi_np)
    L = sre2.row_bits(N, form)
    x0, xc = (1 << L) - 6, 2 * (1 << L) + 613
    case_id("row-pairs-ragged", form, x0, xc)
    on, off = sre2.Context(0), sre2.Context(0)
    off.set_row_pairs(False)
    on.set_scratch_limit(5 << 20)
    try:
        a = sre2.shift_partials(psi, x0, xc, form=form, ctx=on).cpu().numpy()
        b = sre2.shift_partials(psi, x0, xc, form=form, ctx=off).cpu().numpy()
        assert np.array_equal(a, b)
        pick = np.array([0, 5, 6, 7, (1 << L) + 5, (1 << L) + 6, xc - 1])
        ref = oracle_mod.partials(psi_np, x0 + pick)
        assert np.max(np.abs(a[pick] - ref) / ref) <= TOL_SX[form]
    finally:
        on.close()
        off.close()


@pytest.mark.parametrize("form,N", [("split16", 15), ("split16", 18), ("splitbf16", 17),
                                    ("split16", 20)])
def test_row_pairs_split_forms_within_rounding(oracle_mod, form, N):
    """Split forms with row pairs: the rebuilt rows are the exact images of
    the computed stored rows, so S_x differs from the full slab's by rounding
    only (the matrix cores sum the H_16 products in their own order): both
    within the FP32 per-shift bar of each other and of the oracle."""
    psi_np = W.haar(N, 500 + N, np.complex64)
    psi = dev(psi_np)
    case_id("row-pairs-split", form, N)
    on, off = sre2.Context(0), sre2.Context(0)
    off.set_row_pairs(False)
    try:
        a = sre2.shift_partials(psi, form=form, ctx=on).cpu().numpy()
        b = sre2.shift_partials(psi, form=form, ctx=off).cpu().numpy()
        assert np.max(np.abs(a - b) / b) <= TOL_SX[form]
        xs = [0, 1, (1 << 12) + 5, (1 << N) - 1, 3 << (N - 2)]
        ref = oracle_mod.partials(psi_np.astype(np.complex128), xs)
        assert np.max(np.abs(a[xs] - ref) / ref) <= TOL_SX[form]
        ra = sre2.m2(psi, form=form, ctx=on)
        rb = sre2.m2(psi, form=form, ctx=off)
        assert abs(ra.m2 - rb.m2) <= TOL_M2[form]
    finally:
        on.close()
        off.close()


@pytest.mark.parametrize("form,N", [("fp32", 22), ("fp32", 23), ("fp64", 21), ("fp64", 22)])
def test_row_pairs_start_of_large_tiles(oracle_mod, form, N):
    """Where the half-LDS pass-2 tiles take row pairs only from
    2^(L + 5) on (sre2_half_slab_first_shift): shifts on both sides of that
    boundary, bit for bit the full slab's S_x and within the oracle's bar."""
    c128 = is64(form)
    psi_np = W.haar(N, 700 + N, np.complex128 if c128 else np.complex64)
    psi = dev(psi_np)
    first = sre2.half_slab_first_shift(N, form)
    assert first > 1 << sre2.row_bits(N, form)
    x0, xc = first - 3, 7
    case_id("row-pairs-start", form, N, first)
    on, off = sre2.Context(0), sre2.Context(0)
    off.set_row_pairs(False)
    try:
        a = sre2.shift_partials(psi, x0, xc, form=form, ctx=on).cpu().numpy()
        b = sre2.shift_partials(psi, x0, xc, form=form, ctx=off).cpu().numpy()
        assert np.array_equal(a, b)
        ref = oracle_mod.partials(psi_np, np.arange(x0, x0 + xc)[[0, 3, 6]])
        assert np.max(np.abs(a[[0, 3, 6]] - ref) / ref) <= TOL_SX[form]
    finally:
        on.close()
        off.close()


@pytest.mark.parametrize("form", ["fp32", "fp64"])
@pytest.mark.parametrize("N", [22, 24])
def test_row_pairs_bitwise_large_chunk(form, N):
    """N = 22 / 24: one whole default row-pair chunk (the 2^14-value
    half-LDS rows at N = 24 in FP32) against the full slab, bit for bit."""
    c128 = is64(form)
    psi = dev(W.haar(N, 400 + N, np.complex128 if c128 else np.complex64))
    on, off = sre2.Context(0), sre2.Context(0)
    off.set_row_pairs(False)
    try:
        cs, _ = on.chunking(N, form)
        x0 = 3 << (N - 2)
        case_id("row-pairs-large", form, N, cs)
        a = sre2.shift_partials(psi, x0, cs, form=form, ctx=on).cpu().numpy()
        b = sre2.shift_partials(psi, x0, cs, form=form, ctx=off).cpu().numpy()
        assert np.array_equal(a, b)
    finally:
        on.close()
        off.close()


@pytest.mark.parametrize("N", [12, 16])
def test_launch_failure_leaves_the_context_usable(monkeypatch, N):
    """A transform launch that reports an error (forced from the host, after
    the staging and norm kernels were enqueued; no kernel fails) fails the
    call with SRE2_EHIP, and the next call on the same context is exact."""
    psi = dev(W.haar(N, 7, np.complex64))
    case_id("launch-fault", N)
    ref = sre2.m2(psi)
    ctx = sre2.Context(0)
    monkeypatch.setenv("SRE2_FAULT", "launch")
    with pytest.raises(sre2.SRE2Error) as err:
        sre2.m2(psi, ctx=ctx)
    assert err.value.code == sre2.EHIP
    monkeypatch.delenv("SRE2_FAULT")
    b = sre2.m2(psi, ctx=ctx)
    ctx.close()
    assert b.status == 0 and b.m2 == ref.m2 and b.S == ref.S


def _golden():
    if not os.path.exists(GOLDEN):
        return {}
    with open(GOLDEN) as f:
        return json.load(f)


def _sha(psi):
    return hashlib.sha256(np.ascontiguousarray(psi).tobytes()).hexdigest()


@pytest.mark.parametrize("form", FORMS)
def test_n20_full_size(oracle_mod, form):
    """Benchmark shape (N=20, complex64, default launch configuration)."""
    g = _golden()
    psi = W.haar(20, W.SEED_N20, np.complex64)
    d = dev(psi)
    case_id("n20", form)
    r = sre2.m2(d, form=form, partials=True)
    assert r.status == 0
    rec = g.get("haar20_sampled")
    assert rec and rec["sha256"] == _sha(psi), "stored N=20 sampled shifts missing or stale"
    xs, ref = rec["shifts"], np.array(rec["partials"])
    got = r.partials.cpu().numpy()[xs]
    assert np.max(np.abs(got - ref) / ref) <= TOL_SX[form]
    full = g.get("haar20")
    assert full and full["sha256"] == _sha(psi), "stored N=20 oracle value missing or stale"
    assert abs(r.m2 - full["m2"]) <= TOL_M2[form], (r.m2, full["m2"])
    psi_t, _ = W.graph_t(20, 10, W.SEED_N20 + 1, dtype=np.complex64)
    rt = sre2.m2(dev(psi_t), form=form)
    assert abs(rt.m2 - 10 * LOG43) <= closed_tol(form)


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16", "fp64", "fp64h"])
@pytest.mark.parametrize("N", [22, 24])
def test_large_n_sampled_shifts(N, form):
    g = _golden()
    name = f"haar{N}_sampled"
    seed = W.SEED_LARGE + (0 if N == 22 else 1)
    psi = W.haar(N, seed, np.complex64)
    rec = g.get(name)
    if not rec or rec["sha256"] != _sha(psi):
        pytest.skip("no stored oracle values for this input")
    d = dev(psi)
    case_id("large", N)
    xs = rec["shifts"][:: max(1, len(rec["shifts"]) // 12)]
    ref = dict(zip(rec["shifts"], rec["partials"]))
    for x in xs:
        got = sre2.shift_partials(d, x, 1, form=form).item()
        assert abs(got - ref[x]) <= TOL_SX[form] * ref[x], x


@pytest.mark.parametrize("form", ["fp32", "fp32h", "split16", "splitbf16"])
def test_max_n_sampled_shift(oracle_mod, form):
    """The largest N of the FP32 forms (2^26 amplitudes, 512 MiB): one
    shift's S_x against the oracle, computed here."""
    N = sre2.MAX_N
    psi = _max_n_state()
    x = (1 << (N - 1)) + 0x2345
    case_id("max-n", N, form)
    got = sre2.shift_partials(dev(psi), x, 1, form=form).item()
    ref = _max_n_ref(x)
    assert abs(got - ref) <= TOL_SX[form] * ref


_MAXN = {}


def _max_n_state():
    if "psi" not in _MAXN:
        _MAXN["psi"] = W.haar(sre2.MAX_N, W.SEED_LARGE + 9, np.complex64)
    return _MAXN["psi"]


def _max_n_ref(x):
    import oracle
    if x not in _MAXN:
        _MAXN[x] = float(oracle.partials(_max_n_state(), [x], threads=1)[0])
    return _MAXN[x]


def _popcount(v):
    v = np.asarray(v, dtype=np.uint64)
    c = np.zeros(v.shape, dtype=np.int64)
    for b in range(64):
        c += ((v >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


_LARGE = {}


def _large_state(kind, N, c128):
    key = (kind, N, c128)
    if key not in _LARGE:
        dt = np.complex128 if c128 else np.complex64
        _LARGE.clear()  # keep one large state resident on the host
        _LARGE[key] = W.t_product(N, dt) if kind == "t" else W.haar(N, W.SEED_LARGE + 40 + N, dt)
    return _LARGE[key]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("N", [22, 24])
def test_large_n_full_default_chunk(oracle_mod, N, form):
    """One whole default chunk at x0 = 2^(N-1), exactly as a full evaluation
    launches it (shifts per chunk from the context, one pass-1 and one pass-2
    launch over the chunk, the 2^14-value half-LDS rows at N = 24).
    |T>^N: by Eq. 1 per qubit, sum_z |<X^a Z^b>|^4 is 1 for a = 0 and
    (1/2)^2 + (1/2)^2 = 1/2 for a = 1, so S_x = 2^-popcount(x) for every
    shift.  Haar: in-chunk shifts against the oracle."""
    c128 = is64(form)
    ctx = sre2.Context(0)
    try:
        cs, _ = ctx.chunking(N, form)
        # half slabs in every form: Hermitian pair, row pairs
        assert cs == (1024 if N == 22 else 256) // (2 if c128 else 1) * 2
        x0 = 1 << (N - 1)
        xs = x0 + np.arange(cs, dtype=np.int64)
        case_id("large-chunk-t", N, form, cs)
        psi = _large_state("t", N, c128)
        got = sre2.shift_partials(dev(psi), x0, cs, form=form, ctx=ctx).cpu().numpy()
        ref = 2.0 ** (-_popcount(xs).astype(np.float64))
        assert np.max(np.abs(got - ref) / ref) <= TOL_SX[form]
        assert abs(got.sum() - ref.sum()) <= TOL_SUM[form] * ref.sum()
        case_id("large-chunk-haar", N, form, cs)
        psi = _large_state("haar", N, c128)
        got = sre2.shift_partials(dev(psi), x0, cs, form=form, ctx=ctx).cpu().numpy()
        pick = [0, 1, cs // 2 + 3, cs - 1]
        ref = oracle_mod.partials(psi, xs[pick])
        assert np.max(np.abs(got[pick] - ref) / ref) <= TOL_SX[form]
        assert abs(got[pick].sum() - ref.sum()) <= TOL_SUM[form] * ref.sum()
    finally:
        ctx.close()
