"""Seeded state-vector generators.

Conventions
-----------
* A state on N qubits is a length-2^N complex vector indexed by the integer
  encoding of the computational bit string; qubit j is bit j of the index
  (least significant bit = qubit 0).  The paper leaves the endianness open;
  M2 does not depend on it, since permuting qubits is a Clifford operation.
* Every generator builds the state in float64 / complex128, normalises it in
  float64, and only then casts (``to_dtype``).  The oracle receives exactly the
  cast bytes, upcast to complex128.
* Random draws use ``numpy.random.default_rng`` (PCG64) with explicit seeds,
  one base seed per workload (``SEED_*``).
"""
from __future__ import annotations

import json
import os

import numpy as np

# The benchmark configurations (seeds, sizes) live in configs.json.
CONFIG_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs.json")
with open(CONFIG_FILE) as _f:
    CONFIGS = json.load(_f)


def _seed(name: str) -> int:
    for c in CONFIGS["configs"]:
        if c["name"] == name:
            return CONFIGS["base_seed"] + c["seed_offset"]
    raise KeyError(name)


BASE_SEED = CONFIGS["base_seed"]
SEED_N10 = _seed("n10_small")        # small single states, N = 10 (complex128)
SEED_N16_BATCH = _seed("n16_batch")  # batch of 40 states, N = 16
SEED_N20 = _seed("n20_single")       # single state, N = 20 (the throughput workload)
SEED_SERVING = _seed("serving")      # serving request stream, N = 8..18
SEED_LARGE = _seed("n22_n24_large")  # N = 22 / 24 states and the N = 20 Ising snapshots


def _indices(N: int) -> np.ndarray:
    return np.arange(1 << N, dtype=np.uint64)


def _bit(k: np.ndarray, j: int) -> np.ndarray:
    return ((k >> np.uint64(j)) & np.uint64(1)).astype(np.int64)


def to_dtype(psi: np.ndarray, dtype) -> np.ndarray:
    """Cast a complex128 state to complex64 or complex128 (contiguous)."""
    return np.ascontiguousarray(psi.astype(np.dtype(dtype)))


def haar(N: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Haar-random pure state: i.i.d. standard complex Gaussian amplitudes,
    normalised (the paper's benchmark workload)."""
    rng = np.random.default_rng(seed)
    d = 1 << N
    psi = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    psi /= np.sqrt(np.sum(np.abs(psi) ** 2))
    return to_dtype(psi, dtype)


def computational_basis(N: int, index: int = 0, dtype=np.complex128) -> np.ndarray:
    psi = np.zeros(1 << N, dtype=np.complex128)
    psi[index] = 1.0
    return to_dtype(psi, dtype)


def plus_state(N: int, dtype=np.complex128) -> np.ndarray:
    psi = np.full(1 << N, 2.0 ** (-N / 2), dtype=np.complex128)
    return to_dtype(psi, dtype)


def t_product(N: int, dtype=np.complex128) -> np.ndarray:
    """|T>^{(x)N} with |T> = (|0> + e^{i pi/4}|1>)/sqrt(2):
    psi(k) = 2^{-N/2} exp(i pi/4 * popcount(k))."""
    k = _indices(N)
    pc = np.bitwise_count(k).astype(np.float64)
    psi = np.exp(1j * np.pi / 4 * pc) * 2.0 ** (-N / 2)
    return to_dtype(psi, dtype)


def _graph_parity(N: int, adj: np.ndarray) -> np.ndarray:
    """sum_{i<j} A_ij k_i k_j mod 2 for every k (A strictly upper triangular)."""
    k = _indices(N)
    par = np.zeros(1 << N, dtype=np.int64)
    for i in range(N):
        mask = 0
        for j in range(i + 1, N):
            if adj[i, j]:
                mask |= 1 << j
        if mask == 0:
            continue
        cnt = np.bitwise_count(k & np.uint64(mask)).astype(np.int64)
        par ^= _bit(k, i) & (cnt & 1)
    return par


def random_adjacency(N: int, rng: np.random.Generator, p: float = 0.5) -> np.ndarray:
    """Erdos-Renyi adjacency: A_ij ~ Bernoulli(p) for i<j, drawn row-major."""
    adj = np.zeros((N, N), dtype=bool)
    for i in range(N):
        for j in range(i + 1, N):
            adj[i, j] = rng.random() < p
    return adj


def graph(N: int, seed: int, p: float = 0.5, dtype=np.complex128) -> np.ndarray:
    """Random graph state psi(k) = (-1)^{sum_{i<j} A_ij k_i k_j} / 2^{N/2}."""
    rng = np.random.default_rng(seed)
    adj = random_adjacency(N, rng, p)
    par = _graph_parity(N, adj)
    psi = (1.0 - 2.0 * par) * 2.0 ** (-N / 2)
    return to_dtype(psi.astype(np.complex128), dtype)


def graph_t(N: int, m: int, seed: int, p: float = 0.5, dtype=np.complex128):
    """Graph state with a diagonal T phase exp(i pi/4 k_j) on m random qubits:
    the CZ network applied to |T>^{(x)m} (x) |+>^{(x)(N-m)} (up to a qubit
    relabelling).  Returns (psi, subset)."""
    rng = np.random.default_rng(seed)
    adj = random_adjacency(N, rng, p)
    subset = np.sort(rng.choice(N, size=m, replace=False)) if m > 0 else np.zeros(0, int)
    par = _graph_parity(N, adj)
    k = _indices(N)
    tcount = np.zeros(1 << N, dtype=np.float64)
    for j in subset:
        tcount += _bit(k, int(j))
    psi = (1.0 - 2.0 * par) * np.exp(1j * np.pi / 4 * tcount) * 2.0 ** (-N / 2)
    return to_dtype(psi, dtype), subset


def ising_couplings(N: int, seed: int) -> np.ndarray:
    """All-to-all couplings J_ij uniform on {-1, +1} for i<j (row-major draws)."""
    rng = np.random.default_rng(seed)
    J = np.zeros((N, N), dtype=np.int64)
    for i in range(N):
        for j in range(i + 1, N):
            J[i, j] = 1 if rng.random() < 0.5 else -1
    return J


def _ising_energy(N: int, J: np.ndarray) -> np.ndarray:
    """h(k) = sum_{i<j} J_ij s_i s_j with s_i = 1 - 2 k_i (exact integers)."""
    k = _indices(N)
    h = np.zeros(1 << N, dtype=np.int64)
    bits = [_bit(k, i) for i in range(N)]
    for i in range(N):
        for j in range(i + 1, N):
            if J[i, j]:
                h += J[i, j] * (1 - 2 * (bits[i] ^ bits[j]))
    return h


def ising_snapshot(N: int, t: int, J: np.ndarray, steps: int = 64,
                   dtype=np.complex128, energy: np.ndarray | None = None) -> np.ndarray:
    """psi_t = diag(exp(i theta_t h(k))) H^{(x)N}|0>, theta_t = pi t / steps."""
    h = _ising_energy(N, J) if energy is None else energy
    theta = np.pi * t / steps
    psi = np.exp(1j * theta * h.astype(np.float64)) * 2.0 ** (-N / 2)
    return to_dtype(psi, dtype)


def ising_energy(N: int, J: np.ndarray) -> np.ndarray:
    return _ising_energy(N, J)


# ---------------------------------------------------------------------------
# Clifford gates on state vectors (for invariance checks of the inputs).
# ---------------------------------------------------------------------------

def _apply_1q(psi: np.ndarray, q: int, U: np.ndarray) -> np.ndarray:
    N = int(np.log2(psi.size))
    t = psi.reshape((2,) * N)            # axis 0 = most significant qubit
    ax = N - 1 - q
    t = np.moveaxis(np.tensordot(U, t, axes=([1], [ax])), 0, ax)
    return np.ascontiguousarray(t.reshape(-1))


def _apply_cz(psi: np.ndarray, a: int, b: int) -> np.ndarray:
    N = int(np.log2(psi.size))
    k = _indices(N)
    sign = 1 - 2 * (_bit(k, a) & _bit(k, b))
    return psi * sign


_H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2.0)
_S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)


def apply_random_clifford(psi: np.ndarray, seed: int, layers: int = 4) -> np.ndarray:
    """Apply `layers` random layers of H, S and CZ gates (complex128)."""
    rng = np.random.default_rng(seed)
    psi = np.asarray(psi, dtype=np.complex128).copy()
    N = int(np.log2(psi.size))
    for _ in range(layers):
        for q in range(N):
            r = rng.integers(3)
            if r == 0:
                psi = _apply_1q(psi, q, _H)
            elif r == 1:
                psi = _apply_1q(psi, q, _S)
        perm = rng.permutation(N)
        for i in range(0, N - 1, 2):
            psi = _apply_cz(psi, int(perm[i]), int(perm[i + 1]))
    return psi


# ---------------------------------------------------------------------------
# Workloads as concrete inputs.
# ---------------------------------------------------------------------------

WORKLOADS = ("n10_small", "n16_batch", "n20_single", "n22_n24_large")


def workload_inputs(name: str):
    """Inputs of a named workload as a list of (name, psi,
    expected_closed_form_or_None).  The serving stream is produced by
    `serving_requests`."""
    out = []
    if name == "n10_small":
        seed = SEED_N10
        out.append(("haar10", haar(10, seed), None))
        out.append(("t10", t_product(10), 10 * np.log2(4.0 / 3.0)))
        out.append(("graph10", graph(10, seed + 100), 0.0))
    elif name == "n16_batch":
        seed = SEED_N16_BATCH
        rng = np.random.default_rng(seed)
        for i in range(32):
            out.append((f"haar16_{i}", haar(16, seed * 1000 + i, np.complex64), None))
        for i in range(8):
            m = int(rng.integers(1, 9))
            psi, _ = graph_t(16, m, seed * 1000 + 500 + i, dtype=np.complex64)
            out.append((f"graphT16_{i}_m{m}", psi, m * np.log2(4.0 / 3.0)))
    elif name == "n20_single":
        seed = SEED_N20
        out.append(("haar20", haar(20, seed, np.complex64), None))
        psi, _ = graph_t(20, 10, seed + 1, dtype=np.complex64)
        out.append(("graphT20_m10", psi, 10 * np.log2(4.0 / 3.0)))
    elif name == "n22_n24_large":
        seed = SEED_LARGE
        out.append(("haar22", haar(22, seed, np.complex64), None))
        out.append(("haar24", haar(24, seed + 1, np.complex64), None))
    else:
        raise ValueError(f"unknown workload {name!r}")
    return out


def serving_requests(count: int = 4096, seed: int | None = None,
                     n_min: int = 8, n_max: int = 18):
    """Serving stream: N ~ U{n_min..n_max}; kind 50/50 Haar or graph+T with
    m ~ U{1..8}; complex64.  Returns a list of dicts with the request's N,
    kind, seed and m (states are built lazily with `build_request`)."""
    rng = np.random.default_rng(SEED_SERVING if seed is None else seed)
    reqs = []
    for i in range(count):
        N = int(rng.integers(n_min, n_max + 1))
        kind = "haar" if rng.random() < 0.5 else "graphT"
        m = int(rng.integers(1, 9)) if kind == "graphT" else 0
        m = min(m, N)
        reqs.append({"id": i, "N": N, "kind": kind, "m": m,
                     "seed": int(rng.integers(0, 2**62))})
    return reqs


def build_request(req) -> np.ndarray:
    if req["kind"] == "haar":
        return haar(req["N"], req["seed"], np.complex64)
    psi, _ = graph_t(req["N"], req["m"], req["seed"], dtype=np.complex64)
    return psi


def snapshot_couplings(N: int = 20) -> np.ndarray:
    """Couplings of the 64-snapshot Ising sequence."""
    return ising_couplings(N, SEED_LARGE + 2)


# ---------------------------------------------------------------------------
# Dynamics workloads (quench dynamics of the paper's examples): random
# product initial states, TFIM parameters, brickwork circuits of Haar U(4).
# ---------------------------------------------------------------------------

TFIM_PARAMS = {"J": 1.0, "hx": 1.5, "hz": 1.5, "dt": 0.2}


def product_angles(N: int, seed: int):
    """Angles of the random product state prod_i (cos(theta_i/2)|0> +
    e^{i phi_i} sin(theta_i/2)|1>): theta_i ~ U[0, pi], phi_i ~ U[0, 2 pi),
    independent (qubit i = bit i)."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, np.pi, N)
    phi = rng.uniform(0.0, 2.0 * np.pi, N)
    return theta, phi


def haar_u4(rng: np.random.Generator) -> np.ndarray:
    """One Haar-random 4x4 unitary: QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q (Mezzadri's construction)."""
    Z = (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))) / np.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))[None, :]


def brickwork_pairs(N: int):
    """Bonds of one brickwork time step on an open chain: even bonds
    (0,1), (2,3), ..., then odd bonds (1,2), (3,4), ..."""
    return [(q, q + 1) for q in range(0, N - 1, 2)] + [(q, q + 1) for q in range(1, N - 1, 2)]


def brickwork_gates(N: int, steps: int, seed: int):
    """(gates, pairs): gates[t][g] is the Haar U(4) of step t on bond
    pairs[g]; a gate acts on the index j = bit(q0) + 2 bit(q1) of its pair."""
    rng = np.random.default_rng(seed)
    pairs = brickwork_pairs(N)
    gates = np.array([[haar_u4(rng) for _ in pairs] for _ in range(steps)], dtype=np.complex128)
    return gates, pairs
