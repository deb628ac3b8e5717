"""FP64 CPU oracle for M2 (arXiv:2512.24685) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU product path never
imports it and shares no code with it.

The arithmetic lives in ``sre2_oracle.c`` (plain scalar FP64 loops, see its
header for the definitions it follows).  This module only marshals numpy
arrays to it.

Functions
---------
m2(psi)                  M2 by Algorithm 1 over all shifts (Eq. final1 / Eq. 1).
total(psi)               (S, n): S = sum_{x,z} |W_x(z)|^4 and n = sum |psi|^2.
norm2(psi), ipr(psi)     n = sum |psi|^2 and sum |psi|^4 of the state as given.
partials(psi, xs)        S_x = sum_z |W_x(z)|^4 for selected shifts.
brute_sum(psi)           sum over all 4^N Pauli strings of |<P>|^4, O(8^N).
pauli_expect(psi, x, z)  <psi|X^x Z^z|psi> by the direct sum (Eq. Pauli_expect).
shift_transform(psi, x)  W_x(z) for all z (one FWHT).
fwht(a)                  unnormalised FWHT of a complex vector.
sre(psi, alpha)          M_alpha of Eq. 1 for any alpha > 0 (alpha = 1: the limit).
alpha_sum(psi, alpha)    sum over Pauli strings of w^alpha (w log2 w at alpha = 1).
brute_alpha_sum(...)     the same by the direct expectation values, O(8^N).
spectrum(psi, nbins)     Pauli-spectrum histogram of q = |<P>|^2 (bins round(-log2 q)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sre2_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsre2_oracle.so")
_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-Wall", "-Wextra", "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    c_int, c_u64, c_i64 = ctypes.c_int, ctypes.c_uint64, ctypes.c_int64
    sig = {
        "sre2o_pauli_expect": [dp, c_int, c_u64, c_u64, dp, dp],
        "sre2o_brute_sum": [dp, c_int, c_int, dp],
        "sre2o_fwht": [dp, c_int],
        "sre2o_shift_transform": [dp, c_int, c_u64, dp],
        "sre2o_shift_partials": [dp, c_int, i64p, c_i64, c_int, dp],
        "sre2o_all_partials": [dp, c_int, c_int, dp],
        "sre2o_sum_ascending": [dp, c_i64, dp],
        "sre2o_norm2": [dp, c_int, dp],
        "sre2o_ipr": [dp, c_int, dp],
        "sre2o_m2": [dp, c_int, c_int, dp, dp, dp],
        "sre2o_max_threads": [],
        "sre2o_alpha_sum": [dp, c_int, ctypes.c_double, c_int, c_int, dp],
        "sre2o_brute_alpha_sum": [dp, c_int, ctypes.c_double, c_int, c_int, dp],
        "sre2o_spectrum": [dp, c_int, c_int, ctypes.c_double, c_int, i64p, i64p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = c_int
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_c128(psi) -> tuple[np.ndarray, int]:
    a = np.ascontiguousarray(np.asarray(psi).astype(np.complex128, copy=False))
    d = a.size
    N = d.bit_length() - 1
    if d < 1 or (1 << N) != d:
        raise ValueError("state length must be a power of two")
    return a, N


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def max_threads() -> int:
    return int(_load().sre2o_max_threads())


def m2(psi, threads: int = 0) -> float:
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_m2(_dp(a), N, threads, ctypes.byref(out), None, None), "m2")
    return float(out.value)


def total(psi, threads: int = 0) -> tuple[float, float]:
    a, N = _as_c128(psi)
    m, s, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_load().sre2o_m2(_dp(a), N, threads, ctypes.byref(m), ctypes.byref(s),
                            ctypes.byref(n)), "m2")
    return float(s.value), float(n.value)


def m2_from_total(S: float, n: float, N: int) -> float:
    return float(-np.log2(S / (2.0 ** N * n ** 4)))


def norm2(psi) -> float:
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_norm2(_dp(a), N, ctypes.byref(out)), "norm2")
    return float(out.value)


def ipr(psi) -> float:
    """sum |psi|^4 of the state as given (FP64, compensated)."""
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_ipr(_dp(a), N, ctypes.byref(out)), "ipr")
    return float(out.value)


def partials(psi, xs=None, threads: int = 0) -> np.ndarray:
    a, N = _as_c128(psi)
    lib = _load()
    if xs is None:
        S = np.empty(1 << N, dtype=np.float64)
        _check(lib.sre2o_all_partials(_dp(a), N, threads, _dp(S)), "all_partials")
        return S
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.int64))
    S = np.empty(xs.size, dtype=np.float64)
    _check(lib.sre2o_shift_partials(
        _dp(a), N, xs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), xs.size,
        threads, _dp(S)), "shift_partials")
    return S


def sum_ascending(v) -> float:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    out = ctypes.c_double()
    _check(_load().sre2o_sum_ascending(_dp(v), v.size, ctypes.byref(out)), "sum")
    return float(out.value)


def brute_sum(psi, threads: int = 0) -> float:
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_brute_sum(_dp(a), N, threads, ctypes.byref(out)), "brute_sum")
    return float(out.value)


def brute_m2(psi, threads: int = 0) -> float:
    a, N = _as_c128(psi)
    return m2_from_total(brute_sum(a, threads), norm2(a), N)


def pauli_expect(psi, x: int, z: int) -> complex:
    a, N = _as_c128(psi)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(_load().sre2o_pauli_expect(_dp(a), N, x, z, ctypes.byref(re),
                                      ctypes.byref(im)), "pauli_expect")
    return complex(re.value, im.value)


def shift_transform(psi, x: int) -> np.ndarray:
    a, N = _as_c128(psi)
    W = np.empty(1 << N, dtype=np.complex128)
    _check(_load().sre2o_shift_transform(_dp(a), N, x, _dp(W)), "shift_transform")
    return W


def fwht(v) -> np.ndarray:
    a, N = _as_c128(v)
    out = a.copy()
    _check(_load().sre2o_fwht(_dp(out), N), "fwht")
    return out


def _kind(alpha: float) -> int:
    if not alpha > 0:
        raise ValueError("alpha must be positive")
    return 2 if alpha == 1 else 1


def alpha_sum(psi, alpha: float, threads: int = 0) -> float:
    """sum_{x,z} w^alpha (alpha != 1) or sum w log2 w (alpha = 1), w = |W_x(z)|^2."""
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_alpha_sum(_dp(a), N, float(alpha), _kind(alpha), threads,
                                   ctypes.byref(out)), "alpha_sum")
    return float(out.value)


def brute_alpha_sum(psi, alpha: float, threads: int = 0) -> float:
    a, N = _as_c128(psi)
    out = ctypes.c_double()
    _check(_load().sre2o_brute_alpha_sum(_dp(a), N, float(alpha), _kind(alpha), threads,
                                         ctypes.byref(out)), "brute_alpha_sum")
    return float(out.value)


def sre_from_sum(S: float, n: float, N: int, alpha: float) -> float:
    """M_alpha (Eq. 1) from the Pauli sum and n = sum |psi|^2."""
    if alpha == 1:
        return float(np.log2(n * n) - S / (2.0 ** N * n * n))
    return float((np.log2(S) - N - alpha * np.log2(n * n)) / (1.0 - alpha))


def sre(psi, alpha: float, threads: int = 0) -> float:
    a, N = _as_c128(psi)
    return sre_from_sum(alpha_sum(a, alpha, threads), norm2(a), N, alpha)


def spectrum(psi, nbins: int, eps: float = 1e-3, threads: int = 0):
    """(counts, near_edge): counts[b] = number of Pauli strings with
    round(-log2(|<P>|^2)) = b (last bin: everything beyond, and zeros);
    near_edge = strings within eps of a bin edge in -log2 units."""
    a, N = _as_c128(psi)
    counts = np.zeros(nbins, dtype=np.int64)
    near = ctypes.c_int64()
    _check(_load().sre2o_spectrum(_dp(a), N, nbins, float(eps), threads,
                                  counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  ctypes.byref(near)), "spectrum")
    return counts, int(near.value)
