"""Plain CPU oracle of the dynamics workloads -- TEST INFRASTRUCTURE ONLY.

Only the test suite may import this module.  It shares no code with the GPU
simulator.  Everything is complex128 / float64 with textbook constructions:

* product_state     prod_i (cos(theta_i/2)|0> + e^{i phi_i} sin(theta_i/2)|1>)
                    (the random initial state of the Hamiltonian-quench
                    example), qubit i = bit i, built by Kronecker products.
* apply_2q          a 4x4 gate on qubits (q0, q1), index j = bit(q0) + 2 bit(q1),
                    by tensor contraction of the state reshaped to 2 x ... x 2.
* tfim_hamiltonian  H = -J sum_{i=0}^{N-2} Z_i Z_{i+1} - hx sum_i X_i - hz sum_i Z_i
                    (TFIM with a longitudinal field, open chain), a sparse
                    matrix assembled from Kronecker products of Pauli matrices.
* tfim_evolve       exp(-i H dt) psi with scipy.sparse.linalg.expm_multiply,
                    the routine the paper itself uses for this example.
* product_m2        M2 of a product state from its Bloch vectors: one qubit
                    has <X>, <Y>, <Z> = (sin t cos p, sin t sin p, cos t), so
                    (1/2) sum_P <P>^4 = (1 + x^4 + y^4 + z^4)/2, and M2 adds up.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def product_state(theta, phi) -> np.ndarray:
    psi = np.ones(1, dtype=np.complex128)
    for t, p in zip(theta, phi):
        v = np.array([np.cos(t / 2.0), np.exp(1j * p) * np.sin(t / 2.0)], dtype=np.complex128)
        psi = np.kron(v, psi)  # qubit i is bit i: later qubits are higher bits
    return psi


def apply_2q(psi: np.ndarray, U: np.ndarray, q0: int, q1: int) -> np.ndarray:
    N = psi.size.bit_length() - 1
    T = np.asarray(psi, dtype=np.complex128).reshape([2] * N)  # axis a = qubit N-1-a
    a0, a1 = N - 1 - q0, N - 1 - q1
    G = np.asarray(U, dtype=np.complex128).reshape(2, 2, 2, 2)  # [b1', b0', b1, b0]
    T = np.moveaxis(T, (a1, a0), (0, 1))
    out = np.tensordot(G, T, axes=([2, 3], [0, 1]))
    out = np.moveaxis(out, (0, 1), (a1, a0))
    return out.reshape(-1)


def _op(N: int, mats: dict) -> sps.csr_matrix:
    """Kronecker product with mats[q] on qubit q and identity elsewhere."""
    M = sps.identity(1, dtype=np.complex128, format="csr")
    for q in range(N):
        M = sps.kron(sps.csr_matrix(mats.get(q, _I)), M, format="csr")
    return M


def tfim_hamiltonian(N: int, J: float, hx: float, hz: float) -> sps.csr_matrix:
    d = 1 << N
    H = sps.csr_matrix((d, d), dtype=np.complex128)
    for i in range(N - 1):
        H = H - J * _op(N, {i: _Z, i + 1: _Z})
    for i in range(N):
        H = H - hx * _op(N, {i: _X}) - hz * _op(N, {i: _Z})
    return H.tocsr()


def tfim_evolve(psi: np.ndarray, H, dt: float, steps: int = 1) -> np.ndarray:
    out = np.asarray(psi, dtype=np.complex128)
    for _ in range(steps):
        out = spla.expm_multiply(-1j * dt * H, out)
    return out


def product_m2(theta, phi) -> float:
    m = 0.0
    for t, p in zip(theta, phi):
        x, y, z = np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)
        m += -np.log2((1.0 + x ** 4 + y ** 4 + z ** 4) / 2.0)
    return float(m)
