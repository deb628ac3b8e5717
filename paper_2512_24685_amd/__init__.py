"""MI355X-native XOR-FWHT evaluation of the second-order stabilizer Renyi
entropy M2 (arXiv:2512.24685).

This module is the Python binding of libsre2 (C ABI in include/sre2.h).  It
only marshals arguments: device memory and streams come from PyTorch, every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if the library is not built, loading fails with an error.

    import torch, paper_2512_24685_amd as sre2
    psi = torch.randn(1 << 16, dtype=torch.complex64, device="cuda")
    r = sre2.m2(psi)            # r.m2, r.S, r.n

Calls without an explicit ``ctx`` use a default context per (device, stream):
a context's workspace serves one stream at a time.
    r3 = sre2.sre(psi, 3.0)     # any Renyi index: r3.m2 holds M_3
    counts, r = sre2.pauli_spectrum(psi, 32)
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsre2.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sre2.h")

OK, EINVAL, EDTYPE, EFORM, ENORM, ENOMEM, EHIP, EBUSY, ECANCELLED, ENOTFOUND, ESCRATCH = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10)
NOALLOC_SCRATCH_BYTES = 32 << 20
C64, C128 = 0, 1
FORMS = {"fp32": 0, "split16": 1, "splitbf16": 2, "fp64": 3, "fp32h": 4, "fp64h": 5}
MAX_N = 26
OUT_LEN = 4
KINDS = ("shift", "pass1", "pass2", "aux")
KIND_COUNT = 4

_lib = None


class SRE2Error(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().sre2_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} (status {code})")


def lib():
    """Load libsre2.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2512_24685_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    c_int, i64, sz = ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    sigs = {
        "sre2_version": ([], c_int),
        "sre2_strerror": ([c_int], ctypes.c_char_p),
        "sre2_create": ([ctypes.POINTER(vp), c_int], c_int),
        "sre2_destroy": ([vp], c_int),
        "sre2_set_scratch_limit": ([vp, sz], c_int),
        "sre2_set_row_pairs": ([vp, c_int], c_int),
        "sre2_half_slab_first_shift": ([c_int, c_int], i64),
        "sre2_workspace_bytes": ([c_int, c_int, c_int], sz),
        "sre2_m2": ([vp, vp, c_int, c_int, c_int, vp, vp, vp], c_int),
        "sre2_m2_noalloc": ([c_int, vp, c_int, c_int, c_int, vp, vp, vp], c_int),
        "sre2_partials": ([vp, vp, c_int, c_int, c_int, i64, i64, vp, vp], c_int),
        "sre2_m2_from_partials": ([vp, vp, c_int, c_int, c_int, vp, vp, vp], c_int),
        "sre2_moments": ([vp, vp, c_int, c_int, vp, vp], c_int),
        "sre2_sre": ([vp, vp, c_int, c_int, c_int, ctypes.c_double, vp, vp], c_int),
        "sre2_pauli_spectrum": ([vp, vp, c_int, c_int, c_int, c_int, vp, vp, vp], c_int),
        "sre2_m2_batched": ([vp, ctypes.POINTER(vp), ctypes.POINTER(c_int), c_int, c_int, c_int,
                             vp, vp], c_int),
        "sre2_set_timing": ([vp, c_int], c_int),
        "sre2_timing_read": ([vp, dp, ctypes.POINTER(i64)], c_int),
        "sre2_chunking": ([vp, c_int, c_int, ctypes.POINTER(i64), ctypes.POINTER(c_int)], c_int),
        "sre2_row_bits": ([c_int, c_int], c_int),
        "sre2_server_create": ([ctypes.POINTER(vp), c_int, c_int, sz, c_int], c_int),
        "sre2_server_submit": ([vp, vp, c_int, c_int, c_int, ctypes.POINTER(ctypes.c_uint64)],
                               c_int),
        "sre2_server_poll": ([vp, ctypes.c_uint64, ctypes.POINTER(c_int), dp, dp], c_int),
        "sre2_server_cancel": ([vp, ctypes.c_uint64], c_int),
        "sre2_server_drain": ([vp, ctypes.c_double], c_int),
        "sre2_server_stats": ([vp, ctypes.POINTER(i64), c_int], c_int),
        "sre2_server_destroy": ([vp], c_int),
        "sre2_sim_create": ([ctypes.POINTER(vp), c_int, c_int], c_int),
        "sre2_sim_destroy": ([vp], c_int),
        "sre2_sim_product_state": ([vp, dp, dp], c_int),
        "sre2_sim_apply_gates": ([vp, dp, ctypes.POINTER(c_int), c_int], c_int),
        "sre2_sim_tfim_step": ([vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double], c_int),
        "sre2_sim_state": ([vp, c_int, vp], c_int),
        "sre2_sim_run_tfim": ([vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, c_int, c_int, dp], c_int),
        "sre2_sim_run_circuit": ([vp, vp, dp, ctypes.POINTER(c_int), c_int, c_int, c_int, dp],
                                 c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/sre2.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sre2_[a-z0-9_]+)\s*\(", text)))


def half_slab_first_shift(N: int, form: str = "fp32") -> int:
    """First shift that takes a half slab (Hermitian pair, row pairs) in a
    default evaluation; 2^N when there is none."""
    v = lib().sre2_half_slab_first_shift(N, FORMS[form])
    if v < 0:
        raise ValueError(f"no two-pass geometry for N={N} form={form}")
    return int(v)


def row_bits(N: int, form: str = "fp32") -> int:
    """Pass-1 row bits for (N, form); 0 for the fused range."""
    v = lib().sre2_row_bits(int(N), FORMS[form])
    if v < 0:
        raise SRE2Error(EINVAL, "sre2_row_bits")
    return v


def strerror(code: int) -> str:
    return lib().sre2_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != OK:
        raise SRE2Error(rc, where)


class Context:
    """Owns a libsre2 context (device workspace) bound to one HIP device."""

    def __init__(self, device: int = 0):
        self._p = ctypes.c_void_p()
        _check(lib().sre2_create(ctypes.byref(self._p), int(device)), "sre2_create")
        self.device = int(device)

    @property
    def handle(self):
        return self._p

    def set_scratch_limit(self, nbytes: int):
        _check(lib().sre2_set_scratch_limit(self._p, int(nbytes)), "sre2_set_scratch_limit")

    def set_row_pairs(self, enable: bool):
        """Row-pair half slabs of the plain FP32 / FP64 forms (default on;
        results are bitwise the same either way)."""
        _check(lib().sre2_set_row_pairs(self._p, int(bool(enable))), "sre2_set_row_pairs")

    def set_timing(self, enable: bool):
        _check(lib().sre2_set_timing(self._p, int(bool(enable))), "sre2_set_timing")

    def timing_read(self) -> dict:
        """Per kernel class: (summed ms, launches) since the last read."""
        ms = (ctypes.c_double * KIND_COUNT)()
        cnt = (ctypes.c_int64 * KIND_COUNT)()
        _check(lib().sre2_timing_read(self._p, ms, cnt), "sre2_timing_read")
        return {name: (ms[k], cnt[k]) for k, name in enumerate(KINDS)}

    def chunking(self, N: int, form: str = "fp32") -> tuple[int, int]:
        cs, P = ctypes.c_int64(), ctypes.c_int()
        _check(lib().sre2_chunking(self._p, N, FORMS[form], ctypes.byref(cs), ctypes.byref(P)),
               "sre2_chunking")
        return cs.value, P.value

    def close(self):
        if self._p:
            lib().sre2_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_contexts: dict[tuple[int, int], Context] = {}


def context(device: int = 0, stream: int = 0) -> Context:
    """The default context of calls that pass no ctx: one per (device,
    stream handle).  A context's workspace must not be used by two streams at
    once (include/sre2.h), so calls on different streams never share one."""
    key = (int(device), int(stream))
    if key not in _contexts:
        _contexts[key] = Context(device)
    return _contexts[key]


def _ctx_stream(t, ctx, stream):
    """(context, stream handle) of a call on tensor t."""
    sp = _stream_ptr(t, stream)
    return (ctx or context(t.device.index or 0, sp)), sp


@dataclass
class Result:
    m2: float
    S: float
    n: float
    status: int
    partials: object = None  # torch tensor of S_x when requested


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex64:
        return C64
    if t.dtype == torch.complex128:
        return C128
    raise TypeError(f"state must be complex64 or complex128, got {t.dtype}")


def _nqubits(t) -> int:
    d = t.numel()
    N = d.bit_length() - 1
    if d < 2 or (1 << N) != d:
        raise ValueError("state length must be 2^N with N >= 1")
    return N


def _stream_ptr(t, stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(t.device)
    return int(s.cuda_stream)


def _prep(psi):
    torch = _torch()
    if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
        raise TypeError("psi must be a torch tensor on a GPU device")
    return psi.contiguous().reshape(-1)


def m2_async(psi, form: str = "fp32", partials: bool = False, ctx: Context | None = None,
             stream=None):
    """Enqueue one evaluation; returns (out tensor [4], partials tensor or None)."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(OUT_LEN, dtype=torch.float64, device=psi.device)
    part = torch.empty(1 << N, dtype=torch.float64, device=psi.device) if partials else None
    rc = lib().sre2_m2(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N, _dtype_code(psi),
                       FORMS[form], ctypes.c_void_p(sp),
                       ctypes.c_void_p(out.data_ptr()),
                       ctypes.c_void_p(part.data_ptr()) if part is not None else None)
    _check(rc, "sre2_m2")
    return out, part


def m2_noalloc_async(psi, out, form: str = "fp32", partials=None, stream=None):
    """sre2_m2_noalloc: one evaluation into the caller's `out` (float64
    device tensor of 4) and optional `partials` (float64 device tensor of
    2^N), with no device allocation by the library (its intermediate buffers
    live in a fixed device array shared by every such call on the device)."""
    psi = _prep(psi)
    N = _nqubits(psi)
    rc = lib().sre2_m2_noalloc(psi.device.index or 0, ctypes.c_void_p(psi.data_ptr()), N,
                               _dtype_code(psi), FORMS[form],
                               ctypes.c_void_p(_stream_ptr(psi, stream)),
                               ctypes.c_void_p(out.data_ptr()),
                               ctypes.c_void_p(partials.data_ptr()) if partials is not None
                               else None)
    _check(rc, "sre2_m2_noalloc")
    return out


def _result(out_row, part=None) -> Result:
    v = out_row.tolist()
    return Result(m2=v[0], S=v[1], n=v[2], status=int(v[3]), partials=part)


def m2(psi, form: str = "fp32", partials: bool = False, ctx: Context | None = None,
       stream=None) -> Result:
    """M2 of one device-resident state (synchronises to read the result)."""
    out, part = m2_async(psi, form, partials, ctx, stream)
    return _result(out.cpu(), part)


def sre(psi, alpha: float = 2.0, form: str = "fp32", ctx: Context | None = None,
        stream=None) -> Result:
    """Stabilizer Renyi entropy M_alpha (Eq. 1) of one device state, any
    alpha > 0 (alpha = 1: the limit); Result.m2 holds M_alpha and Result.S
    the Pauli sum.  alpha = 2 is exactly m2()."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(OUT_LEN, dtype=torch.float64, device=psi.device)
    rc = lib().sre2_sre(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N, _dtype_code(psi),
                        FORMS[form], float(alpha), ctypes.c_void_p(sp),
                        ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_sre")
    return _result(out.cpu())


def pauli_spectrum(psi, nbins: int = 32, form: str = "fp32", ctx: Context | None = None,
                   stream=None):
    """Histogram of |<P>|^2 over all 4^N Pauli strings in bins round(-log2 q)
    (last bin: everything beyond, and zeros).  Returns (counts as a numpy
    int64 array, Result with n and status)."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(OUT_LEN, dtype=torch.float64, device=psi.device)
    counts = torch.empty(int(nbins), dtype=torch.int64, device=psi.device)
    rc = lib().sre2_pauli_spectrum(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N,
                                   _dtype_code(psi), FORMS[form], int(nbins),
                                   ctypes.c_void_p(sp),
                                   ctypes.c_void_p(counts.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_pauli_spectrum")
    return counts.cpu().numpy(), _result(out.cpu())


def moments(psi, ctx: Context | None = None, stream=None):
    """(n, sum |psi|^4, non-finite count) of the state as given, in FP64
    (synchronises to read them)."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(3, dtype=torch.float64, device=psi.device)
    rc = lib().sre2_moments(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N, _dtype_code(psi),
                            ctypes.c_void_p(sp),
                            ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_moments")
    n, ipr, bad = out.cpu().tolist()
    return n, ipr, int(bad)


def shift_partials(psi, x_begin: int = 0, x_count: int | None = None, form: str = "fp32",
                   ctx: Context | None = None, stream=None):
    """S_x for x in [x_begin, x_begin + x_count) as a float64 device tensor."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    if x_count is None:
        x_count = (1 << N) - x_begin
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(max(int(x_count), 1), dtype=torch.float64, device=psi.device)
    rc = lib().sre2_partials(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N, _dtype_code(psi),
                             FORMS[form], int(x_begin), int(x_count),
                             ctypes.c_void_p(sp),
                             ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_partials")
    return out


def m2_from_partials(psi, partials, form: str = "fp32", ctx: Context | None = None,
                     stream=None) -> Result:
    """M2 of `psi` from all its S_x (float64 device tensor of 2^N, e.g.
    gathered from shift_partials over ranges): the norm, the fixed-order sum
    and the logarithm of sre2_m2 (synchronises to read the result)."""
    torch = _torch()
    psi = _prep(psi)
    N = _nqubits(psi)
    if (not isinstance(partials, torch.Tensor) or partials.dtype != torch.float64
            or partials.device != psi.device or partials.numel() != (1 << N)):
        raise ValueError("partials must be a float64 tensor of 2^N values on psi's device")
    partials = partials.contiguous()
    ctx, sp = _ctx_stream(psi, ctx, stream)
    out = torch.empty(OUT_LEN, dtype=torch.float64, device=psi.device)
    rc = lib().sre2_m2_from_partials(ctx.handle, ctypes.c_void_p(psi.data_ptr()), N,
                                     _dtype_code(psi), FORMS[form],
                                     ctypes.c_void_p(partials.data_ptr()), ctypes.c_void_p(sp),
                                     ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_m2_from_partials")
    return _result(out.cpu())


def m2_batched(psis, form: str = "fp32", ctx: Context | None = None, stream=None) -> list[Result]:
    """M2 of several device states of one dtype (mixed N allowed)."""
    torch = _torch()
    psis = [_prep(p) for p in psis]
    if not psis:
        return []
    dt = _dtype_code(psis[0])
    for p in psis:
        if _dtype_code(p) != dt:
            raise TypeError("all states of a batch must share one dtype")
    dev = psis[0].device
    ctx, sp = _ctx_stream(psis[0], ctx, stream)
    cnt = len(psis)
    ptrs = (ctypes.c_void_p * cnt)(*[p.data_ptr() for p in psis])
    Ns = (ctypes.c_int * cnt)(*[_nqubits(p) for p in psis])
    out = torch.empty(cnt * OUT_LEN, dtype=torch.float64, device=dev)
    rc = lib().sre2_m2_batched(ctx.handle, ptrs, Ns, cnt, dt, FORMS[form],
                               ctypes.c_void_p(sp),
                               ctypes.c_void_p(out.data_ptr()))
    _check(rc, "sre2_m2_batched")
    o = out.cpu().reshape(cnt, OUT_LEN)
    return [_result(o[i]) for i in range(cnt)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, 4
SERVER_STATS = ("submitted", "admitted", "completed", "cancelled", "packs", "packed_states",
                "singles", "peak_bytes", "peak_inflight")


class Server:
    """Continuous-batching serving loop (sre2_server_* in include/sre2.h)."""

    def __init__(self, device: int = 0, form: str = "fp32", hbm_budget: int = 8 << 30,
                 max_slots: int = 4096):
        self._p = ctypes.c_void_p()
        _check(lib().sre2_server_create(ctypes.byref(self._p), int(device), FORMS[form],
                                        int(hbm_budget), int(max_slots)), "sre2_server_create")

    def submit(self, psi) -> int:
        """Submit a numpy complex64/complex128 state (host memory, copied) or a
        torch GPU tensor (device memory; keep it alive until done)."""
        import numpy as np
        t = ctypes.c_uint64()
        if isinstance(psi, np.ndarray):
            a = np.ascontiguousarray(psi)
            if a.dtype not in (np.complex64, np.complex128):
                raise TypeError("state must be complex64 or complex128")
            N = a.size.bit_length() - 1
            if (1 << N) != a.size:
                raise ValueError("state length must be 2^N")
            rc = lib().sre2_server_submit(self._p, ctypes.c_void_p(a.ctypes.data), N,
                                          C64 if a.dtype == np.complex64 else C128, 0,
                                          ctypes.byref(t))
        else:
            p = _prep(psi)
            rc = lib().sre2_server_submit(self._p, ctypes.c_void_p(p.data_ptr()), _nqubits(p),
                                          _dtype_code(p), 1, ctypes.byref(t))
        _check(rc, "sre2_server_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """(state, Result or None, latency seconds or None); a final state
        releases the ticket."""
        st = ctypes.c_int()
        res = (ctypes.c_double * OUT_LEN)()
        lat = ctypes.c_double()
        _check(lib().sre2_server_poll(self._p, ctypes.c_uint64(ticket), ctypes.byref(st), res,
                                      ctypes.byref(lat)), "sre2_server_poll")
        if st.value in (REQ_DONE, REQ_CANCELLED, REQ_FAILED):
            return st.value, Result(m2=res[0], S=res[1], n=res[2], status=int(res[3])), lat.value
        return st.value, None, None

    def cancel(self, ticket: int):
        _check(lib().sre2_server_cancel(self._p, ctypes.c_uint64(ticket)), "sre2_server_cancel")

    def drain(self, timeout: float = 600.0):
        _check(lib().sre2_server_drain(self._p, float(timeout)), "sre2_server_drain")

    def stats(self) -> dict:
        v = (ctypes.c_int64 * len(SERVER_STATS))()
        _check(lib().sre2_server_stats(self._p, v, len(SERVER_STATS)), "sre2_server_stats")
        return dict(zip(SERVER_STATS, list(v)))

    def close(self):
        if self._p:
            rc = lib().sre2_server_destroy(self._p)
            self._p = ctypes.c_void_p()
            _check(rc, "sre2_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f64(a):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _gates_arg(gates):
    """complex (..., 4, 4) -> interleaved float64 buffer."""
    import numpy as np
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.complex128))
    return _f64(g.view(np.float64).reshape(-1))


def _pairs_arg(pairs):
    import numpy as np
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1))
    return p, p.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), p.size // 2


class Simulator:
    """Quench-dynamics state-vector simulator (sre2_sim_* in include/sre2.h):
    a complex128 state of N qubits on one device, qubit i = bit i."""

    def __init__(self, N: int, device: int = 0):
        self._p = ctypes.c_void_p()
        _check(lib().sre2_sim_create(ctypes.byref(self._p), int(device), int(N)),
               "sre2_sim_create")
        self.N = int(N)
        self.device = int(device)

    def product_state(self, theta, phi):
        th, thp = _f64(theta)
        ph, php = _f64(phi)
        if th.size != self.N or ph.size != self.N:
            raise ValueError("theta and phi need N entries")
        _check(lib().sre2_sim_product_state(self._p, thp, php), "sre2_sim_product_state")

    def apply_gates(self, gates, pairs):
        """gates: (count, 4, 4) complex; pairs: (count, 2) qubits."""
        g, gp = _gates_arg(gates)
        p, pp, cnt = _pairs_arg(pairs)
        if g.size != 32 * cnt:
            raise ValueError("one 4x4 gate per pair")
        _check(lib().sre2_sim_apply_gates(self._p, gp, pp, cnt), "sre2_sim_apply_gates")

    def tfim_step(self, J: float, hx: float, hz: float, dt: float):
        _check(lib().sre2_sim_tfim_step(self._p, J, hx, hz, dt), "sre2_sim_tfim_step")

    def state(self, dtype=None):
        """The current state as a new torch tensor (complex128 by default)."""
        torch = _torch()
        dtype = dtype or torch.complex128
        out = torch.empty(1 << self.N, dtype=dtype, device=f"cuda:{self.device}")
        _check(lib().sre2_sim_state(self._p, _dtype_code(out), ctypes.c_void_p(out.data_ptr())),
               "sre2_sim_state")
        return out

    def _results(self, buf, steps):
        return [Result(m2=buf[4 * t], S=buf[4 * t + 1], n=buf[4 * t + 2],
                       status=int(buf[4 * t + 3])) for t in range(steps + 1)]

    def run_tfim(self, server: "Server", J: float, hx: float, hz: float, dt: float,
                 steps: int, dtype: str = "complex64") -> list:
        """M2 of the state now and after each of `steps` TFIM steps, the
        snapshots streamed into `server` while the evolution goes on."""
        buf = (ctypes.c_double * (OUT_LEN * (steps + 1)))()
        _check(lib().sre2_sim_run_tfim(self._p, server._p, J, hx, hz, dt, int(steps),
                                       C64 if dtype == "complex64" else C128, buf),
               "sre2_sim_run_tfim")
        return self._results(buf, steps)

    def run_circuit(self, server: "Server", gates, pairs, dtype: str = "complex64") -> list:
        """gates: (steps, gates_per_step, 4, 4) complex; pairs: the bonds of a step."""
        import numpy as np
        gates = np.asarray(gates)
        steps = int(gates.shape[0])
        g, gp = _gates_arg(gates)
        p, pp, cnt = _pairs_arg(pairs)
        if g.size != 32 * cnt * steps:
            raise ValueError("gates must be (steps, len(pairs), 4, 4)")
        buf = (ctypes.c_double * (OUT_LEN * (steps + 1)))()
        _check(lib().sre2_sim_run_circuit(self._p, server._p, gp, pp, cnt, steps,
                                          C64 if dtype == "complex64" else C128, buf),
               "sre2_sim_run_circuit")
        return self._results(buf, steps)

    def close(self):
        if self._p:
            rc = lib().sre2_sim_destroy(self._p)
            self._p = ctypes.c_void_p()
            _check(rc, "sre2_sim_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
