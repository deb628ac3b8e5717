"""Pins of the dynamics oracle (CPU only) against textbook constructions.

* Product states: M2 equals the sum of the one-qubit Bloch-vector closed form
  (additivity of Eq. 1 and <X>, <Y>, <Z> of one qubit).
* Two-qubit gates: tensor contraction equals the dense 2^N x 2^N matrix built
  from Kronecker products and a basis permutation (N <= 6), for neighbouring
  and distant qubits in either order; Haar U(4) samples are unitary.
* TFIM Hamiltonian: equals matrix elements <k'|H|k> written out per basis
  state; Hermitian; at J = hz = 0 its spectrum is hx (N - 2m) with
  multiplicity C(N, m); at hx = 0 it is diagonal with the Ising energies.
* Evolution: expm_multiply equals dense scipy expm (N <= 8), conserves the
  norm and the energy, and reverses under dt -> -dt.
"""
from math import comb

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import dynamics as D


def test_product_state_m2_closed_form(oracle_mod):
    for N, seed in ((1, 3), (4, 5), (9, 7)):
        th, ph = W.product_angles(N, seed)
        psi = D.product_state(th, ph)
        assert abs(np.vdot(psi, psi) - 1.0) < 1e-14
        assert abs(oracle_mod.m2(psi) - D.product_m2(th, ph)) < 1e-12
    # one qubit: amplitudes are the definition
    th, ph = W.product_angles(1, 11)
    psi = D.product_state(th, ph)
    assert np.allclose(psi, [np.cos(th[0] / 2), np.exp(1j * ph[0]) * np.sin(th[0] / 2)])


def _dense_2q(N, U, q0, q1):
    """<k'|G|k> for every basis pair, straight from the gate's definition."""
    d = 1 << N
    M = np.zeros((d, d), dtype=np.complex128)
    for k in range(d):
        j = ((k >> q0) & 1) + 2 * ((k >> q1) & 1)
        rest = k & ~((1 << q0) | (1 << q1))
        for i in range(4):
            kp = rest | ((i & 1) << q0) | (((i >> 1) & 1) << q1)
            M[kp, k] += U[i, j]
    return M


@pytest.mark.parametrize("N,q0,q1", [(2, 0, 1), (3, 1, 2), (5, 0, 4), (6, 4, 1), (6, 2, 3)])
def test_apply_2q_equals_dense(N, q0, q1):
    rng = np.random.default_rng(N * 10 + q0)
    U = W.haar_u4(rng)
    assert np.allclose(U.conj().T @ U, np.eye(4), atol=1e-14)
    psi = W.haar(N, 31 + N)
    ref = _dense_2q(N, U, q0, q1) @ psi
    assert np.allclose(D.apply_2q(psi, U, q0, q1), ref, atol=1e-14)
    if (q0, q1) == (0, 1):  # on two qubits the gate is the matrix itself
        assert np.allclose(_dense_2q(2, U, 0, 1), U)


def _tfim_elements(N, J, hx, hz):
    d = 1 << N
    H = np.zeros((d, d), dtype=np.complex128)
    for k in range(d):
        s = [1 - 2 * ((k >> i) & 1) for i in range(N)]  # Z eigenvalues, |0> = up
        H[k, k] = -J * sum(s[i] * s[i + 1] for i in range(N - 1)) - hz * sum(s)
        for i in range(N):
            H[k ^ (1 << i), k] += -hx
    return H


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_tfim_hamiltonian_elements(N):
    H = D.tfim_hamiltonian(N, 1.0, 1.5, 1.5).toarray()
    assert np.allclose(H, _tfim_elements(N, 1.0, 1.5, 1.5), atol=1e-14)
    assert np.allclose(H, H.conj().T)


def test_tfim_limits():
    N = 5
    ev = np.sort(np.linalg.eigvalsh(D.tfim_hamiltonian(N, 0.0, 0.7, 0.0).toarray()))
    ref = np.sort(np.concatenate([[0.7 * (N - 2 * m)] * comb(N, m) for m in range(N + 1)]))
    assert np.allclose(ev, ref, atol=1e-12)
    H = D.tfim_hamiltonian(N, 1.3, 0.0, 0.4).toarray()
    assert np.allclose(H, np.diag(np.diag(H)))


@pytest.mark.parametrize("N", [3, 6, 8])
def test_tfim_evolution(N):
    p = W.TFIM_PARAMS
    H = D.tfim_hamiltonian(N, p["J"], p["hx"], p["hz"])
    th, ph = W.product_angles(N, 17)
    psi0 = D.product_state(th, ph)
    U = scipy.linalg.expm(-1j * p["dt"] * H.toarray())
    psi1 = D.tfim_evolve(psi0, H, p["dt"])
    assert np.allclose(psi1, U @ psi0, atol=1e-12)
    psi5 = D.tfim_evolve(psi0, H, p["dt"], steps=5)
    assert abs(np.linalg.norm(psi5) - 1.0) < 1e-12
    e0 = np.vdot(psi0, H @ psi0).real
    assert abs(np.vdot(psi5, H @ psi5).real - e0) < 1e-10
    back = D.tfim_evolve(psi5, H, -p["dt"], steps=5)
    assert np.allclose(back, psi0, atol=1e-11)
