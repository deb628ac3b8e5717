"""CPU checks of the GPU tile engine's layout plans (no GPU needed).

The constexpr plan builder of the kernels (paper_2512_24685_amd/csrc/sre2_plan.h)
is compiled into a small host probe.  The tests then replay, with numpy, the
exact index arithmetic of the kernels - global load mapping, register
butterflies, swizzled LDS transposes between rounds, final mapping, two-pass
scratch layout - and compare with the Walsh-Hadamard transform over the same
bits and with the oracle's per-shift sums.  They also check that every round's
LDS accesses hit distinct bank slots within each group of 2^SB lanes.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "plan_probe.cpp")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("probe") / "plan_probe.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", "-o", so, SRC], check=True)
    lib = ctypes.CDLL(so)
    lib.probe_plan.restype = ctypes.c_int
    lib.probe_swz.restype = ctypes.c_uint
    return lib


FUSED, PASS1, PASS2, LIMITS = 0, 1, 2, 3


def geo(lib, precision, kind, param=0):
    """(TB, RB, SB) of a kernel: fused(N), pass1, pass2(H); LIMITS gives
    (largest fused N, pass-1 row bits, largest N)."""
    tb, rb, sb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = lib.probe_geometry(precision, kind, param, ctypes.byref(tb), ctypes.byref(rb),
                            ctypes.byref(sb))
    assert rc == 0, (precision, kind, param)
    return tb.value, rb.value, sb.value


def plan(lib, tb, rb, sb, lo, hi):
    out = (ctypes.c_uint * 32)()
    n = lib.probe_plan(tb, rb, sb, lo, hi, out)
    return [tuple(out[4 * j:4 * j + 4]) for j in range(n)]


def pdep(v: np.ndarray, mask: int) -> np.ndarray:
    r = np.zeros_like(v)
    k = 0
    for b in range(32):
        if (mask >> b) & 1:
            r |= ((v >> k) & 1) << b
            k += 1
    return r


def swz_np(sb, e):
    h = e >> sb
    f = np.zeros_like(e)
    while np.any(h):
        f ^= h & ((1 << sb) - 1)
        h >>= sb
    return e ^ f


def mapping(rd, tb, rb):
    T = 1 << (tb - rb)
    t = np.arange(T, dtype=np.int64)
    base = pdep(t & 63, rd[2]) | pdep(t >> 6, rd[3])
    i = np.arange(1 << rb, dtype=np.int64)
    return base[:, None] | pdep(i, rd[0])[None, :]


def bfly(V, reg, bf):
    V = V.copy()
    for b in range(32):
        if (bf >> b) & 1:
            rbit = bin(reg & ((1 << b) - 1)).count("1")
            i = np.arange(V.shape[1])
            lo = i[((i >> rbit) & 1) == 0]
            hi = lo | (1 << rbit)
            a, c = V[:, lo].copy(), V[:, hi].copy()
            V[:, lo], V[:, hi] = a + c, a - c
    return V


def run_tile(X, rounds, tb, rb, sb):
    """Replay one tile through the plan; returns the tile after the transform."""
    E = [mapping(rd, tb, rb) for rd in rounds]
    V = X[E[0]]
    V = bfly(V, rounds[0][0], rounds[0][1])
    for j in range(1, len(rounds)):
        lds = np.full(1 << tb, np.nan + 0j)
        lds[swz_np(sb, E[j - 1])] = V
        V = lds[swz_np(sb, E[j])]
        V = bfly(V, rounds[j][0], rounds[j][1])
    out = np.empty_like(X)
    out[E[-1]] = V
    return out


def wht_bits(X, lo, hi):
    """Unnormalised Walsh-Hadamard transform along index bits [lo, hi)."""
    X = X.copy()
    for b in range(lo, hi):
        Y = X.reshape(-1, 2, 1 << b)
        a, c = Y[:, 0, :].copy(), Y[:, 1, :].copy()
        Y[:, 0, :], Y[:, 1, :] = a + c, a - c
        X = Y.reshape(-1)
    return X


def test_wht_bits_helper_is_sylvester():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    assert np.allclose(wht_bits(x, 0, 6), scipy.linalg.hadamard(64) @ x)
    # transform along bits [2, 5) only = I_2 (x) H_8 (x) I_4
    H = np.kron(np.kron(np.eye(2), scipy.linalg.hadamard(8)), np.eye(4))
    assert np.allclose(wht_bits(x, 2, 5), H @ x)


def all_plans(lib):
    """Every (tile geometry, transform range) a compiled kernel uses."""
    for prec in (0, 1):
        fmax, row, nmax = geo(lib, prec, LIMITS)
        rbf = geo(lib, prec, FUSED, fmax)[1]
        for N in range(rbf, fmax + 1):
            tb, rb, sb = geo(lib, prec, FUSED, N)
            yield prec, "fused", N, (tb, rb, sb, 0, N)
        tb, rb, sb = geo(lib, prec, PASS1)
        assert tb == row
        yield prec, "pass1", tb, (tb, rb, sb, 0, tb)
        for H in range(1, nmax - row + 1):
            tb, rb, sb = geo(lib, prec, PASS2, H)
            yield prec, "pass2", H, (tb, rb, sb, tb - H, tb)


def test_geometry_limits(probe):
    for prec in (0, 1):
        fmax, row, nmax = geo(probe, prec, LIMITS)
        assert row <= fmax < nmax and nmax >= 24
        for H in range(1, nmax - row + 1):
            tb, rb, _ = geo(probe, prec, PASS2, H)
            assert H <= tb and tb - H <= row and tb - rb >= 6
        for N in range(geo(probe, prec, FUSED, fmax)[1], fmax + 1):
            tb, rb, _ = geo(probe, prec, FUSED, N)
            assert tb >= N and tb - rb >= 6


def test_plan_structure(probe):
    for prec, kind, par, args in all_plans(probe):
        tb, rb, sb, lo, hi = args
        rounds = plan(probe, *args)
        full = (1 << tb) - 1
        tmask = sum(1 << b for b in range(lo, hi))
        seen = 0
        for reg, bf, lane, wave in rounds:
            assert reg & lane == 0 and reg & wave == 0 and lane & wave == 0
            assert reg | lane | wave == full
            assert bin(reg).count("1") == rb and bin(lane).count("1") == 6
            assert bf & ~reg == 0 and bf & seen == 0
            seen |= bf
        assert seen == tmask, (prec, kind, par)
        if kind == "fused":  # last round holds one shift per thread
            assert rounds[-1][0] & ~((1 << par) - 1) == 0
        # first round: lanes on the lowest tile bits outside the registers
        reg0, _, lane0, _ = rounds[0]
        free = [b for b in range(tb) if not (reg0 >> b) & 1]
        low = sum(1 << b for b in free[:4])
        assert lane0 & low == low, (prec, kind, par)  # coalesced global access


def test_swizzle_bijective_and_linear(probe):
    for sb in (4, 5):
        e = np.arange(1 << 14, dtype=np.int64)
        s = np.array([probe.probe_swz(sb, int(v)) for v in e[:4096]])
        assert np.array_equal(s, swz_np(sb, e[:4096]))
        full = swz_np(sb, e)
        assert np.array_equal(np.sort(full), e)
        a, b = 0x1234 & 0x3FFF, 0x0F0F & 0x3FFF
        assert swz_np(sb, np.array([a ^ b]))[0] == swz_np(sb, np.array([a]))[0] ^ swz_np(sb, np.array([b]))[0]


def test_lds_bank_slots_distinct(probe):
    for prec, kind, par, args in all_plans(probe):
        tb, rb, sb, lo, hi = args
        rounds = plan(probe, *args)
        if len(rounds) == 1:
            continue
        for rd in rounds:
            E = swz_np(sb, mapping(rd, tb, rb))
            slots = E & ((1 << sb) - 1)
            g = 1 << sb
            T = E.shape[0]
            for t0 in range(0, T, g):
                blk = slots[t0:t0 + g]  # lanes of one group, every register index
                for i in range(blk.shape[1]):
                    assert len(set(blk[:, i].tolist())) == g, (prec, kind, par, rd, t0, i)


def test_tile_transform_matches_wht(probe):
    rng = np.random.default_rng(3)
    for prec, kind, par, (tb, rb, sb, lo, hi) in all_plans(probe):
        X = rng.standard_normal(1 << tb) + 1j * rng.standard_normal(1 << tb)
        out = run_tile(X, plan(probe, tb, rb, sb, lo, hi), tb, rb, sb)
        assert np.allclose(out, wht_bits(X, lo, hi)), (prec, kind, par)


def insert0(v, hb):
    return ((v >> hb) << (hb + 1)) | (v & ((1 << hb) - 1))


def reduce4(v, herm):
    if herm:  # Hermitian pair: 16 (Re^4 + Im^4)
        return 16.0 * np.sum(v.real ** 4 + v.imag ** 4)
    return np.sum(np.abs(v) ** 4)


def emulate_fused_partials(probe, psi, prec, herm=False, x_begin=0):
    """Per-shift sums exactly as k_fused indexes them (tile of 2^(TB-NT) shifts)."""
    N = psi.size.bit_length() - 1
    NT = N - int(herm)
    tb, rb, sb = geo(probe, prec, FUSED, NT)
    rounds = plan(probe, tb, rb, sb, 0, NT)
    spt = 1 << (tb - NT)
    d = 1 << N
    S = {}
    e = np.arange(1 << tb)
    for t0 in range(x_begin, d, spt):
        out = np.zeros(1 << tb, dtype=np.complex128)
        X = np.zeros(1 << tb, dtype=np.complex128)
        for j in range(spt):
            x = t0 + j
            if x >= d:
                continue
            kp = e[j << NT:(j + 1) << NT] & ((1 << NT) - 1)
            k = insert0(kp, x.bit_length() - 1) if herm else kp
            X[j << NT:(j + 1) << NT] = np.conj(psi[k ^ x]) * psi[k]
        out = run_tile(X, rounds, tb, rb, sb)
        for j in range(spt):
            if t0 + j < d:
                S[t0 + j] = reduce4(out[j << NT:(j + 1) << NT], herm)
    return np.array([S[x] for x in range(x_begin, d)])


def emulate_two_pass_partials(probe, psi, prec, xs, herm=False):
    """Per-shift sums as k_pass1 / k_pass2 index them (row slab, then columns)."""
    N = psi.size.bit_length() - 1
    NS = N - int(herm)
    L, rb1, sb = geo(probe, prec, PASS1)
    HT = NS - L
    tb2, rb2, _ = geo(probe, prec, PASS2, HT)
    p1 = plan(probe, L, rb1, sb, 0, L)
    p2 = plan(probe, tb2, rb2, sb, tb2 - HT, tb2)
    e1 = np.arange(1 << L)
    e2 = np.arange(1 << tb2)
    cb = tb2 - HT
    out = []
    for x in xs:
        assert not herm or x >= (1 << L)
        slab = np.empty(1 << NS, dtype=np.complex128)
        for srow in range(1 << HT):
            row = insert0(srow, x.bit_length() - 1 - L) if herm else srow
            rowbase = row << L
            prow = rowbase ^ (x & ~((1 << L) - 1))
            X = np.conj(psi[prow + (e1 ^ (x & ((1 << L) - 1)))]) * psi[rowbase + e1]
            slab[srow << L:(srow + 1) << L] = run_tile(X, p1, L, rb1, sb)
        acc = 0.0
        for ct in range(1 << (L - cb)):
            src = (e2 >> cb << L) + (ct << cb) + (e2 & ((1 << cb) - 1))
            acc += reduce4(run_tile(slab[src], p2, tb2, rb2, sb), herm)
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("prec,N,herm", [(0, 6, False), (0, 9, False), (1, 5, False),
                                         (1, 8, False), (0, 6, True), (0, 9, True), (1, 5, True),
                                         (1, 8, True)])
def test_fused_indexing_matches_oracle(probe, oracle_mod, prec, N, herm):
    psi = W.haar(N, 42 + N)
    x0 = 1 if herm else 0
    S = emulate_fused_partials(probe, psi, prec, herm, x0)
    ref = oracle_mod.partials(psi)[x0:]
    assert np.allclose(S, ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("prec,extra,herm", [(0, 1, False), (0, 3, False), (1, 1, False),
                                             (1, 3, False), (0, 1, True), (0, 3, True),
                                             (1, 1, True), (1, 3, True)])
def test_two_pass_indexing_matches_oracle(probe, oracle_mod, prec, extra, herm):
    fmax, L, _ = geo(probe, prec, LIMITS)
    N = fmax + extra
    psi = W.haar(N, 7)
    if herm:
        xs = [1 << L, (1 << N) - 1, 0x2A5A % (1 << N) | (1 << L), 1 << (N - 1), 3 << (N - 2)]
    else:
        xs = [0, 1, (1 << N) - 1, 0x2A5A % (1 << N), 1 << (N - 1)]
    S = emulate_two_pass_partials(probe, psi, prec, xs, herm)
    ref = oracle_mod.partials(psi, xs)
    assert np.allclose(S, ref, rtol=1e-11, atol=0)


# ---------------------------------------------------------------------------
# Split-FP16 MFMA form: remainder butterflies in round 0, then H_16 factors on
# the LDS tile with the MFMA lane addressing (rows 4g+j on factor bits,
# columns on the lowest four other bits, blocks on the rest).
# ---------------------------------------------------------------------------

def low_bits_mask(m, count):
    r = 0
    for b in range(32):
        if count == 0:
            break
        if (m >> b) & 1:
            r |= 1 << b
            count -= 1
    return r


def top_bits_mask(m, count):
    r = 0
    for b in reversed(range(32)):
        if count == 0:
            break
        if (m >> b) & 1:
            r |= 1 << b
            count -= 1
    return r


H16 = np.array([[(-1) ** bin(i & k).count("1") for k in range(16)] for i in range(16)], float)


def mfma_h16_emul(lds, tb, sb, F):
    full = (1 << tb) - 1
    CM = low_bits_mask(full & ~F, 4)
    BM = full & ~F & ~CM
    lanes = np.arange(64)
    for b in range(1 << (tb - 8)):
        eb = pdep(np.array([b]), BM)[0]
        ecol = pdep(lanes & 15, CM)
        rows = [pdep(4 * (lanes >> 4) + j, F) | ecol | eb for j in range(4)]
        X = np.zeros((16, 16), dtype=np.complex128)  # [k][n]
        for j in range(4):
            X[4 * (lanes >> 4) + j, lanes & 15] = lds[swz_np(sb, rows[j])]
        D = H16 @ X
        for j in range(4):
            lds[swz_np(sb, rows[j])] = D[4 * (lanes >> 4) + j, lanes & 15]


def run_tile_split(X, rounds, tb, rb, sb):
    T = 0
    for rd in rounds:
        T |= rd[1]
    r0, rl = rounds[0], rounds[-1]
    REM = top_bits_mask(r0[0] & T, bin(T).count("1") % 4)
    FB = T & ~REM
    E0 = mapping(r0, tb, rb)
    V = bfly(X[E0], r0[0], REM)
    if FB == 0:
        out = np.empty_like(X)
        out[E0] = V
        return out
    lds = np.full(1 << tb, np.nan + 0j)
    lds[swz_np(sb, E0)] = V
    while FB:
        F = low_bits_mask(FB, 4)
        mfma_h16_emul(lds, tb, sb, F)
        FB &= ~F
    El = mapping(rl, tb, rb)
    V = lds[swz_np(sb, El)]
    out = np.empty_like(X)
    out[El] = V
    return out


def test_split_transform_matches_wht(probe):
    rng = np.random.default_rng(5)
    for prec, kind, par, (tb, rb, sb, lo, hi) in all_plans(probe):
        if prec != 0:
            continue
        X = rng.standard_normal(1 << tb) + 1j * rng.standard_normal(1 << tb)
        out = run_tile_split(X, plan(probe, tb, rb, sb, lo, hi), tb, rb, sb)
        assert np.allclose(out, wht_bits(X, lo, hi)), (kind, par)
