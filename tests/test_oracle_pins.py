"""Pins of the FP64 CPU oracle against things fixed by the paper and by the
mathematics, not by the oracle itself (CPU only).

* Textbook Pauli matrices: W_x(z) equals <psi| (X^x1 Z^z1) (x) ... |psi> built
  from dense 2x2 matrices and Kronecker products (N <= 5), element by element.
* Brute force over all Pauli strings (the definition, Eq. 1) equals the
  XOR-FWHT result (Eq. final1), N <= 7.
* FWHT equals the Sylvester Hadamard matrix of scipy; WHT identities of the
  SI (involution, XOR-convolution theorem, conjugation, Parseval).
* Closed forms: stabilizer states give 0 (faithfulness), |T>^N gives
  N log2(4/3) (Eq. 1 on one qubit + additivity), graph+T on m qubits gives
  m log2(4/3) (Clifford invariance), Ising snapshots vanish at Clifford angles
  and obey their period / reflection symmetries.
* Invariants: additivity, Clifford invariance, scale invariance, purity,
  per-shift Parseval, bounds, the real / imaginary pattern of W, Haar average.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import workloads as W

LOG43 = np.log2(4.0 / 3.0)

_I = np.eye(2, dtype=np.complex128)
_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _pauli_matrix(N, x, z):
    """X^x Z^z as a dense matrix; qubit j = bit j, so qubit N-1 is the
    leftmost Kronecker factor."""
    M = np.ones((1, 1), dtype=np.complex128)
    for j in reversed(range(N)):
        f = _I
        if (x >> j) & 1:
            f = f @ _X
        if (z >> j) & 1:
            f = f @ _Z
        M = np.kron(M, f)
    return M


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_transform_equals_textbook_pauli_expectations(oracle_mod, N):
    psi = W.haar(N, 100 + N)
    d = 1 << N
    for x in range(d):
        Wx = oracle_mod.shift_transform(psi, x)
        for z in range(d):
            ref = np.vdot(psi, _pauli_matrix(N, x, z) @ psi)
            assert abs(Wx[z] - ref) < 1e-13, (x, z)
    # the direct-sum expectation agrees as well
    for x, z in [(0, 0), (1, d - 1), (d - 1, 1), (d // 2, d // 2 + 1 if d > 2 else 0)]:
        ref = np.vdot(psi, _pauli_matrix(N, x, z) @ psi)
        assert abs(oracle_mod.pauli_expect(psi, x, z) - ref) < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_brute_force_equals_xor_fwht(oracle_mod, N):
    psi = W.haar(N, 200 + N)
    S_fwht, n = oracle_mod.total(psi)
    S_brute = oracle_mod.brute_sum(psi)
    assert abs(S_fwht - S_brute) <= 1e-13 * S_brute
    assert abs(oracle_mod.m2(psi) - oracle_mod.brute_m2(psi)) < 1e-12


def test_brute_force_matches_dense_definition(oracle_mod):
    """Eq. 1 with alpha=2 over all 4^N Pauli matrices, N=3."""
    N = 3
    psi = W.haar(N, 5)
    s = 0.0
    for x, z in itertools.product(range(8), range(8)):
        s += abs(np.vdot(psi, _pauli_matrix(N, x, z) @ psi)) ** 4
    assert abs(oracle_mod.brute_sum(psi) - s) < 1e-13 * s


@pytest.mark.parametrize("N", [0, 1, 3, 6, 10])
def test_fwht_equals_sylvester_hadamard(oracle_mod, N):
    rng = np.random.default_rng(N)
    a = rng.standard_normal(1 << N) + 1j * rng.standard_normal(1 << N)
    H = scipy.linalg.hadamard(1 << N).astype(np.float64)
    assert np.allclose(oracle_mod.fwht(a), H @ a, atol=1e-11, rtol=0)


@pytest.mark.parametrize("N", [2, 5, 9])
def test_wht_identities(oracle_mod, N):
    rng = np.random.default_rng(10 + N)
    d = 1 << N
    f = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    g = rng.standard_normal(d) + 1j * rng.standard_normal(d)
    Ff, Fg = oracle_mod.fwht(f), oracle_mod.fwht(g)
    # involution: FWHT(FWHT f) = 2^N f
    assert np.allclose(oracle_mod.fwht(Ff), d * f, atol=1e-10)
    # XOR convolution theorem (unnormalised form): FWHT(f *xor g) = FWHT f . FWHT g
    idx = np.arange(d)
    conv = np.array([np.sum(f * g[x ^ idx]) for x in range(d)])
    assert np.allclose(oracle_mod.fwht(conv), Ff * Fg, atol=1e-9)
    # conjugation
    assert np.allclose(oracle_mod.fwht(np.conj(f)), np.conj(Ff), atol=1e-12)
    # Parseval (unnormalised): sum |FWHT f|^2 = 2^N sum |f|^2
    assert abs(np.sum(abs(Ff) ** 2) - d * np.sum(abs(f) ** 2)) < 1e-10 * d * np.sum(abs(f) ** 2)


def test_single_qubit_t_state_pauli_values(oracle_mod):
    """|T>: <I>=1, <X>=<Y>=1/sqrt2, <Z>=0, so sum |<P>|^4 = 3/2."""
    psi = W.t_product(1)
    vals = {(x, z): oracle_mod.pauli_expect(psi, x, z) for x in (0, 1) for z in (0, 1)}
    assert abs(vals[(0, 0)] - 1) < 1e-15
    assert abs(abs(vals[(1, 0)]) - 2 ** -0.5) < 1e-15
    assert abs(abs(vals[(1, 1)]) - 2 ** -0.5) < 1e-15
    assert abs(vals[(0, 1)]) < 1e-15
    assert abs(oracle_mod.brute_sum(psi) - 1.5) < 1e-14


@pytest.mark.parametrize("N", list(range(1, 11)))
def test_t_product_closed_form(oracle_mod, N):
    assert abs(oracle_mod.m2(W.t_product(N)) - N * LOG43) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 5, 9, 10, 12])
def test_stabilizer_states_vanish(oracle_mod, N):
    for psi in (W.computational_basis(N, (1 << N) - 1), W.plus_state(N),
                W.graph(N, 300 + N)):
        assert abs(oracle_mod.m2(psi)) < 1e-12


@pytest.mark.parametrize("N,m", [(7, 0), (7, 1), (7, 3), (7, 6), (9, 9), (10, 4)])
def test_graph_t_closed_form(oracle_mod, N, m):
    psi, _ = W.graph_t(N, m, 400 + 10 * N + m)
    assert abs(oracle_mod.m2(psi) - m * LOG43) < 1e-12


def test_ising_snapshot_clifford_points_and_symmetries(oracle_mod):
    N = 7
    J = W.ising_couplings(N, 17)
    h = W.ising_energy(N, J)
    m = {t: oracle_mod.m2(W.ising_snapshot(N, t, J, energy=h)) for t in range(0, 64)}
    for t in (0, 16, 32, 48):
        assert abs(m[t]) < 1e-12
    for t in range(1, 32):
        assert abs(m[t] - m[t + 32]) < 1e-11
        assert abs(m[t] - m[32 - t]) < 1e-11
    # theta -> pi/4 - theta: psi becomes a diagonal Clifford (the bond phases
    # at pi/4) times conj(psi), so M2(t) = M2(16 - t)
    for t in range(1, 16):
        assert abs(m[t] - m[16 - t]) < 1e-11
    assert max(m.values()) > 0.5  # non-trivial away from Clifford angles


def test_stored_n20_snapshots_obey_the_reflections():
    """The oracle's stored N = 20 snapshot values at t = 5 and 21 agree as
    M2(t) = M2(16 - t) = M2(32 - t) requires (21 -> 11 -> 5).  This is a
    consistency check, not an independent value: with all-to-all +-1
    couplings at N = 20 the energy h(k) is a sum of 190 odd terms, hence
    even, so psi_21 = psi_5 times a diagonal of fourth roots of unity, i.e. a
    phase Clifford, and Clifford invariance forces equality."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_values.json")
    with open(path) as f:
        g = json.load(f)
    assert abs(g["ising20_t5"]["m2"] - g["ising20_t21"]["m2"]) < 1e-12
    assert g["ising20_t5"]["m2"] > 1.0
    J = W.snapshot_couplings(20)
    h = W.ising_energy(20, J)
    assert np.all(np.asarray(h) % 2 == 0)  # the phase ratio is i^(h/2)


def test_additivity(oracle_mod):
    a, b = W.haar(3, 1), W.haar(4, 2)
    ab = np.kron(a, b)
    assert abs(oracle_mod.m2(ab) - oracle_mod.m2(a) - oracle_mod.m2(b)) < 1e-12


def test_clifford_invariance(oracle_mod):
    psi = W.haar(6, 3)
    phi = W.apply_random_clifford(psi, seed=4, layers=5)
    assert abs(np.linalg.norm(phi) - 1) < 1e-12
    assert abs(oracle_mod.m2(phi) - oracle_mod.m2(psi)) < 1e-12


def test_scale_invariance(oracle_mod):
    psi = W.haar(8, 9)
    assert abs(oracle_mod.m2(psi * (0.37 - 1.1j)) - oracle_mod.m2(psi)) < 1e-12


def test_purity_parseval_hermiticity_bounds(oracle_mod):
    N = 6
    d = 1 << N
    psi = W.haar(N, 11) * 1.7  # unnormalised on purpose
    n = np.sum(abs(psi) ** 2)
    total2 = 0.0
    for x in range(d):
        Wx = oracle_mod.shift_transform(psi, x)
        f = np.conj(psi[np.arange(d) ^ x]) * psi
        # per-shift Parseval
        assert abs(np.sum(abs(Wx) ** 2) - d * np.sum(abs(f) ** 2)) < 1e-11 * d
        total2 += np.sum(abs(Wx) ** 2)
        # W is real for even popcount(x & z), imaginary for odd
        par = np.array([bin(x & z).count("1") & 1 for z in range(d)])
        assert np.all(abs(Wx.imag[par == 0]) < 1e-13)
        assert np.all(abs(Wx.real[par == 1]) < 1e-13)
        assert np.all(abs(Wx) <= n * (1 + 1e-13))
        if x == 0:
            assert abs(Wx[0] - n) < 1e-13
    # purity: sum_{x,z} |W|^2 = 2^N n^2
    assert abs(total2 - d * n * n) < 1e-11 * d * n * n
    m = oracle_mod.m2(psi)
    assert 0.0 <= m <= N


def test_norm_and_ipr(oracle_mod):
    """n and sum |psi|^4: basis state (1, 1), |+>^N (1, 2^-N), a scaled
    state (c^2 n, c^4 IPR), Parseval on the x = 0 transform
    (sum_z |W_0(z)|^2 = 2^N sum |psi|^4), and the Haar mean 2 / (2^N + 1)."""
    N = 7
    d = 1 << N
    e = np.zeros(d, np.complex128)
    e[37] = 1.0
    assert oracle_mod.norm2(e) == 1.0 and oracle_mod.ipr(e) == 1.0
    plus = np.full(d, 2.0 ** (-N / 2), np.complex128)
    assert abs(oracle_mod.norm2(plus) - 1.0) < 1e-15
    assert abs(oracle_mod.ipr(plus) / 2.0 ** -N - 1.0) < 1e-14
    psi = W.haar(N, 21)
    c = 1.3
    assert abs(oracle_mod.norm2(c * psi) - c * c * oracle_mod.norm2(psi)) < 1e-14
    assert abs(oracle_mod.ipr(c * psi) - c ** 4 * oracle_mod.ipr(psi)) < 1e-14
    W0 = oracle_mod.shift_transform(psi, 0)
    assert abs(np.sum(abs(W0) ** 2) - d * oracle_mod.ipr(psi)) < 1e-12 * d
    vals = [oracle_mod.ipr(W.haar(10, 700 + i)) for i in range(8)]
    assert abs(np.mean(vals) * (2 ** 10 + 1) / 2 - 1.0) < 0.05


def test_haar_average_law(oracle_mod):
    """Fig. 1(b): Haar average close to log2(2^N + 3) - 2 (statistical)."""
    N = 10
    vals = [oracle_mod.m2(W.haar(N, 500 + i)) for i in range(4)]
    assert abs(np.mean(vals) - (np.log2(2 ** N + 3) - 2)) < 0.02


def test_partials_match_full_and_sum(oracle_mod):
    psi = W.haar(9, 12)
    S_all = oracle_mod.partials(psi)
    xs = [0, 5, 511, 256]
    assert np.array_equal(oracle_mod.partials(psi, xs), S_all[xs])
    S, n = oracle_mod.total(psi)
    assert abs(oracle_mod.sum_ascending(S_all) - S) <= 1e-15 * S
    # S_0 = sum_z |FWHT(|psi|^2)(z)|^4
    F = oracle_mod.fwht(abs(psi) ** 2)
    assert abs(S_all[0] - np.sum(abs(F) ** 4)) < 1e-13 * S_all[0]


# ---------------------------------------------------------------------------
# General Renyi index (Eq. 1) and the Pauli spectrum.
# ---------------------------------------------------------------------------

ALPHAS = [0.5, 1.0, 1.5, 2.0, 3.0]


def _t_single(alpha):
    """M_alpha of one |T> qubit from Eq. 1: the four expectation values are
    1 (identity), 1/sqrt2 (X, Y) and 0 (Z), so (1/2) sum |<P>|^(2 alpha) =
    (1 + 2^(1 - alpha)) / 2; the alpha -> 1 limit is the Shannon form with
    Xi = (1/2, 1/4, 1/4, 0): H = 3/2 bits, minus N = 1."""
    if alpha == 1:
        return 0.5
    return np.log2((1.0 + 2.0 ** (1.0 - alpha)) / 2.0) / (1.0 - alpha)


def _brute_spectrum(psi, nbins):
    """Histogram straight from the textbook Pauli matrices (N <= 4)."""
    N = psi.size.bit_length() - 1
    n = np.vdot(psi, psi).real
    counts = np.zeros(nbins, dtype=np.int64)
    for x in range(1 << N):
        for z in range(1 << N):
            q = abs(np.vdot(psi, _pauli_matrix(N, x, z) @ psi)) ** 2 / n ** 2
            if q < 1e-24:
                counts[-1] += 1
            else:
                counts[min(nbins - 1, max(0, int(np.floor(-np.log2(q) + 0.5))))] += 1
    return counts


@pytest.mark.parametrize("alpha", ALPHAS)
@pytest.mark.parametrize("N", [1, 3, 5])
def test_alpha_sum_equals_brute_force(oracle_mod, N, alpha):
    psi = W.haar(N, 700 + N)
    a = oracle_mod.alpha_sum(psi, alpha)
    b = oracle_mod.brute_alpha_sum(psi, alpha)
    assert abs(a - b) <= 1e-12 * max(1.0, abs(b))
    # against the textbook matrices for the smallest case
    if N == 1:
        ws = [abs(np.vdot(psi, _pauli_matrix(1, x, z) @ psi)) ** 2 for x in (0, 1) for z in (0, 1)]
        ref = sum(w * np.log2(w) if alpha == 1 else w ** alpha for w in ws if w > 0)
        assert abs(a - ref) <= 1e-13


@pytest.mark.parametrize("alpha", ALPHAS)
def test_alpha_closed_forms(oracle_mod, alpha):
    for N in (1, 2, 4, 6):
        assert abs(oracle_mod.sre(W.t_product(N), alpha) - N * _t_single(alpha)) < 1e-12
    # faithfulness: stabilizer states give 0 for every index
    for psi in (W.graph(6, 3), W.computational_basis(5, 9), W.plus_state(4)):
        assert abs(oracle_mod.sre(psi, alpha)) < 1e-12
    # alpha = 2 is M2
    psi = W.haar(6, 71)
    if alpha == 2:
        assert abs(oracle_mod.sre(psi, 2.0) - oracle_mod.m2(psi)) < 1e-12


@pytest.mark.parametrize("alpha", ALPHAS)
def test_alpha_invariants(oracle_mod, alpha):
    a, b = W.haar(3, 81), W.haar(4, 82)
    ab = np.kron(b, a)  # qubits of a are the low bits
    assert abs(oracle_mod.sre(ab, alpha) - oracle_mod.sre(a, alpha)
               - oracle_mod.sre(b, alpha)) < 1e-11  # additivity
    psi = W.haar(6, 83)
    m = oracle_mod.sre(psi, alpha)
    assert abs(oracle_mod.sre(W.apply_random_clifford(psi, 5), alpha) - m) < 1e-11
    assert abs(oracle_mod.sre((2.5 - 1j) * psi, alpha) - m) < 1e-11  # scale invariance
    assert 0.0 <= m <= 6.0 + 1e-12


def test_alpha_limit_and_monotonicity(oracle_mod):
    psi = W.haar(6, 91)
    m1 = oracle_mod.sre(psi, 1.0)
    for h in (1e-3, 1e-4):
        assert abs(oracle_mod.sre(psi, 1.0 + h) - m1) < 10 * h
        assert abs(oracle_mod.sre(psi, 1.0 - h) - m1) < 10 * h
    ms = [oracle_mod.sre(psi, a) for a in (0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0)]
    assert all(x >= y - 1e-12 for x, y in zip(ms, ms[1:]))  # Renyi order


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_spectrum_equals_textbook(oracle_mod, N):
    for psi in (W.haar(N, 300 + N), W.t_product(N), W.graph(N, 4)):
        counts, _ = oracle_mod.spectrum(psi, 12)
        assert np.array_equal(counts, _brute_spectrum(psi, 12))
        assert counts.sum() == 4 ** N


def _near_edges_textbook(psi, nbins, eps):
    """Strings whose -log2 q (q from the textbook matrices, q > 0) lies within
    eps of an edge b + 1/2 between bins b and b + 1, b = 0 .. nbins - 2."""
    N = psi.size.bit_length() - 1
    n = np.vdot(psi, psi).real
    edges = np.arange(nbins - 1) + 0.5
    near = 0
    for x in range(1 << N):
        for z in range(1 << N):
            q = abs(np.vdot(psi, _pauli_matrix(N, x, z) @ psi)) ** 2 / n ** 2
            if q > 1e-24 and np.min(np.abs(-np.log2(q) - edges)) <= eps:
                near += 1
    return near


@pytest.mark.parametrize("eps", [0.0, 0.05, 0.2, 0.45])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_spectrum_near_edge_equals_textbook(oracle_mod, N, eps):
    for psi in (W.haar(N, 310 + N), W.haar(N, 320 + N), W.t_product(N)):
        _, near = oracle_mod.spectrum(psi, 8, eps=eps)
        assert near == _near_edges_textbook(psi, 8, eps), (N, eps)


def test_spectrum_near_edge_closed_form(oracle_mod):
    """One qubit cos(th/2)|0> + sin(th/2)|1>: q = 1 (I), sin^2 th (X),
    cos^2 th (Z), 0 (Y).  With sin^2 th = 2^-(3/2 + 1/100), X sits 0.01 above
    the edge 3/2 and Z at -log2(1 - 2^-1.51) = 0.62396..., 0.12396 above the
    edge 1/2; I sits 1/2 below that edge."""
    s2 = 2.0 ** -1.51
    th = np.arcsin(np.sqrt(s2))
    psi = np.array([np.cos(th / 2), np.sin(th / 2)], np.complex128)
    dz = -np.log2(1.0 - s2) - 0.5
    assert 0.1239 < dz < 0.1240
    counts, _ = oracle_mod.spectrum(psi, 4, eps=0.0)
    assert list(counts) == [1, 1, 1, 1]  # I in bin 0, Z in bin 1, X in bin 2, Y last
    for eps, want in ((0.0, 0), (0.009, 0), (0.011, 1), (0.12, 1), (0.13, 2), (0.49, 2)):
        assert oracle_mod.spectrum(psi, 4, eps=eps)[1] == want, eps
    # X at 1.51 is also 0.99 from the edge 2.5, Z 0.876 from 1.5: only the
    # nearest edge counts, so no string is counted twice
    assert oracle_mod.spectrum(psi, 4, eps=0.999)[1] == 3  # I at distance 0.5 joins


def test_spectrum_closed_forms(oracle_mod):
    from math import comb
    for N in (3, 5):
        d = 1 << N
        counts, near = oracle_mod.spectrum(W.graph(N, 12), 10)
        assert counts[0] == d and counts[-1] == d * d - d and counts[1:-1].sum() == 0
        assert near == 0
        counts, near = oracle_mod.spectrum(W.t_product(N), N + 2)
        for k in range(N + 1):  # q = 2^-k for C(N, k) 2^k strings
            assert counts[k] == comb(N, k) * 2 ** k
        assert counts[-1] == 4 ** N - 3 ** N and near == 0
    # scale invariance
    psi = W.haar(5, 13)
    assert np.array_equal(oracle_mod.spectrum(psi, 20)[0],
                          oracle_mod.spectrum(3.0 * psi, 20)[0])
