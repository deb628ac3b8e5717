"""CPU checks of the GPU tile engine's layout plans (no GPU needed).

The constexpr plan builder of the kernels (paper_2512_24685_amd/csrc/sre2_plan.h)
is compiled into a small host probe.  The tests then replay, with numpy, the
exact index arithmetic of the kernels - global load mapping, register
butterflies, the split form's H_16 factors in the matrix-core operand layout,
padded or swizzled LDS transposes between rounds, final mapping, two-pass scratch
layout - and compare with the Walsh-Hadamard transform over the same bits and
with the oracle's per-shift sums.  They also check that every round's LDS
accesses hit distinct bank slots within each group of 2^SB lanes.
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
    lib.probe_pad.restype = ctypes.c_uint
    lib.probe_swz.restype = ctypes.c_uint
    return lib


FUSED, PASS1, PASS2, LIMITS = 0, 1, 2, 3


def geo(lib, precision, kind, param=0):
    """(TB, RB, SB) of a kernel: fused(N), pass1(NS: slab bits; 0 = the
    smallest row), pass2(H); LIMITS gives (largest fused N, smallest pass-1
    row bits, largest N)."""
    tb, rb, sb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = lib.probe_geometry(precision, kind, param, ctypes.byref(tb), ctypes.byref(rb),
                            ctypes.byref(sb))
    assert rc == 0, (precision, kind, param)
    return tb.value, rb.value, sb.value


class Rounds(list):
    """A plan's rounds; half = True for a half-LDS plan (the top tile bit is
    the top register-index bit of every round and each transpose moves the
    register halves with that bit 0, then 1, through half the tile);
    padded = True when its LDS slots are padded, else swizzled."""
    half = False
    padded = False


KINDS = {"fused": 0, "pass1": 1, "pass2": 2}


def plan(lib, tb, rb, sb, lo, hi, split=0, kind="pass1"):
    """Rounds (reg, bfly, lane, wave, lperm, mf) as the kernel of `kind`
    selects them; split 0 = plain plan, else the split-FP16 plan with tail
    split - 1 (1: pass-1 store round, 2: fused); half-LDS plans for two-pass
    tiles above 64 KiB and for the largest plain fused tiles."""
    out = (ctypes.c_uint * 48)()
    n = lib.probe_plan(tb, rb, sb, lo, hi, split, KINDS[kind], out)
    r = Rounds(tuple(out[6 * j:6 * j + 6]) for j in range(n % 100))
    r.half = (n % 1000) >= 100
    r.padded = n >= 1000
    return r


def fusedrb(lib, prec, N, split=0):
    """Registers (log2) per fused thread for transforms of N bits."""
    return lib.probe_fused_rb(prec, N, split)


def p1rb(lib, prec, L, split=0):
    """Registers (log2) per pass-1 thread for rows of L bits."""
    return lib.probe_pass1_rb(prec, L, split)


def lane_bits(rd):
    """Tile bit of each lane-id bit 0..5."""
    return [(rd[4] >> (5 * i)) & 31 for i in range(6)]


def pdep(v: np.ndarray, mask: int) -> np.ndarray:
    r = np.zeros_like(v)
    k = 0
    for b in range(32):
        if (mask >> b) & 1:
            r |= ((v >> k) & 1) << b
            k += 1
    return r


def pad_np(sb, e):
    """Padded LDS slot of tile element e: e + (e >> sb) + (e >> 2 sb) + ..."""
    s = np.zeros_like(e)
    h = np.array(e, copy=True)
    while np.any(h):
        s += h
        h >>= sb
    return s


def swz_np(sb, e):
    """Swizzled LDS slot: the low sb bits XORed with every higher sb-bit chunk."""
    h = e >> sb
    f = np.zeros_like(e)
    while np.any(h):
        f ^= h & ((1 << sb) - 1)
        h >>= sb
    return e ^ f


def slot_np(rounds, sb, e):
    return pad_np(sb, e) if rounds.padded else swz_np(sb, e)


def lds_slots(rounds, sb, t):
    """Slots of the LDS buffer of a tile with t bits in LDS."""
    return int(pad_np(sb, np.array([(1 << t) - 1]))[0]) + 1 if rounds.padded else 1 << t


def mapping(rd, tb, rb):
    T = 1 << (tb - rb)
    t = np.arange(T, dtype=np.int64)
    base = pdep(t >> 6, rd[3])
    for i, b in enumerate(lane_bits(rd)):
        base |= ((t >> i) & 1) << b
    i = np.arange(1 << rb, dtype=np.int64)
    return base[:, None] | pdep(i, rd[0])[None, :]


H16 = np.array([[(-1) ** bin(i & k).count("1") for k in range(16)] for i in range(16)], float)


def mf_reg_index(rd):
    """Register-index bit of the lower of the factor's two register bits."""
    m = rd[5] & rd[0]
    low = m & -m
    return bin(rd[0] & (low - 1)).count("1")


def mf_apply(V, a):
    """H_16 on every register group as the matrix cores compute it: for each
    setting q of the register-index bits other than a, a + 1, lane 16g + c
    supplies rows 4g + j (j = register-index bits a, a + 1) of column c and
    receives rows 4g + r of the product in the same registers.  V is
    (..., threads, registers)."""
    V = V.copy()
    T, R = V.shape[-2:]
    lanes = np.arange(64)
    g, c = lanes >> 4, lanes & 15
    for w in range(0, T, 64):
        for q in range(R // 4):
            b = (q & ((1 << a) - 1)) | ((q >> a) << (a + 2))
            B = np.zeros(V.shape[:-2] + (16, 16), dtype=V.dtype)
            for j in range(4):
                B[..., 4 * g + j, c] = V[..., w + lanes, b + (j << a)]
            D = H16 @ B
            for r in range(4):
                V[..., w + lanes, b + (r << a)] = D[..., 4 * g + r, c]
    return V


def round_math(V, rd):
    V = bfly(V, rd[0], rd[1])
    return mf_apply(V, mf_reg_index(rd)) if rd[5] else V


def bfly(V, reg, bf):
    """Butterflies on register bits; V is (..., threads, registers)."""
    V = V.copy()
    for b in range(32):
        if (bf >> b) & 1:
            rbit = bin(reg & ((1 << b) - 1)).count("1")
            i = np.arange(V.shape[-1])
            lo = i[((i >> rbit) & 1) == 0]
            hi = lo | (1 << rbit)
            a, c = V[..., lo].copy(), V[..., hi].copy()
            V[..., lo], V[..., hi] = a + c, a - c
    return V


def run_tile(X, rounds, tb, rb, sb):
    """Replay tiles through the plan; X is (..., 2^tb), one tile per leading
    index; returns the tiles after the transform.  Half-LDS plans move the
    two register halves through a buffer of 2^(tb-1) slots (the top tile bit
    dropped from the slot), as the kernels do."""
    E = [mapping(rd, tb, rb) for rd in rounds]
    V = round_math(X[..., E[0]], rounds[0])
    half = getattr(rounds, "half", False)
    top, hr = 1 << (tb - 1), 1 << (rb - 1)
    for j in range(1, len(rounds)):
        if not half:
            lds = np.full(X.shape[:-1] + (lds_slots(rounds, sb, tb),), np.nan + 0j)
            lds[..., slot_np(rounds, sb, E[j - 1])] = V
            V = round_math(lds[..., slot_np(rounds, sb, E[j])], rounds[j])
            continue
        W = np.empty_like(V)
        for h in (0, 1):
            regs = slice(h * hr, (h + 1) * hr)
            # the register half holds exactly the elements with top bit h
            assert np.all((E[j - 1][:, regs] & top) == h * top)
            assert np.all((E[j][:, regs] & top) == h * top)
            lds = np.full(X.shape[:-1] + (lds_slots(rounds, sb, tb - 1),), np.nan + 0j)
            lds[..., slot_np(rounds, sb, E[j - 1][:, regs] & (top - 1))] = V[..., regs]
            W[..., regs] = lds[..., slot_np(rounds, sb, E[j][:, regs] & (top - 1))]
            assert not np.isnan(W[..., regs]).any()
        V = round_math(W, rounds[j])
    out = np.empty_like(X)
    out[..., E[-1]] = V
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
    """Every (tile geometry, transform range, split flag) a compiled kernel
    uses; the split form exists for complex64 tiles only."""
    for prec in (0, 1):
        fmax, row, nmax = geo(lib, prec, LIMITS)
        rbf = fusedrb(lib, prec, 1)  # smallest fused N
        for split in ((0, 1) if prec == 0 else (0,)):
            for N in range(rbf, fmax + 1):
                tb, _, sb = geo(lib, prec, FUSED, N)
                yield prec, "fused", N, (tb, fusedrb(lib, prec, N, split), sb, 0, N, 3 * split)
            assert geo(lib, prec, PASS1)[0] == row
            rows, hs = set(), set()
            for NS in range(fmax, nmax + 1):  # every slab size of two-pass
                L = geo(lib, prec, PASS1, NS)[0]
                rows.add(L)
                hs.add(NS - L)
            sb = geo(lib, prec, PASS1)[2]
            for L in sorted(rows):
                yield prec, "pass1", L, (L, p1rb(lib, prec, L, split), sb, 0, L, 2 * split)
            for H in sorted(hs):
                tb, rb, sb = geo(lib, prec, PASS2, H)
                yield prec, "pass2", H, (tb, rb, sb, tb - H, tb, split)


def test_geometry_limits(probe):
    for prec in (0, 1):
        fmax, row, nmax = geo(probe, prec, LIMITS)
        assert row <= fmax < nmax and nmax >= 24
        for NS in range(fmax, nmax + 1):
            L, rb1, _ = geo(probe, prec, PASS1, NS)
            H = NS - L
            assert L >= row and L - rb1 >= 6
            tb, rb, _ = geo(probe, prec, PASS2, H)
            assert H <= tb and tb - H <= L and tb - rb >= 6
            # rows grow until pass 2 keeps <= 10 row bits or the tile is full
            assert H <= 10 or L == (14 if prec == 0 else 13)
            if H <= 10 and L > row:
                assert H == 10
        for N in range(geo(probe, prec, FUSED, fmax)[1], fmax + 1):
            tb, rb, _ = geo(probe, prec, FUSED, N)
            assert tb >= N and tb - rb >= 6


def test_plan_structure(probe):
    for prec, kind, par, args in all_plans(probe):
        tb, rb, sb, lo, hi, split = args
        rounds = plan(probe, *args, kind=kind)
        full = (1 << tb) - 1
        tmask = sum(1 << b for b in range(lo, hi))
        seen = 0
        case = (prec, kind, par, split)
        for reg, bf, lane, wave, lperm, mf in rounds:
            assert reg & lane == 0 and reg & wave == 0 and lane & wave == 0
            assert reg | lane | wave == full
            assert bin(reg).count("1") == rb and bin(lane).count("1") == 6
            lb = lane_bits((reg, bf, lane, wave, lperm, mf))
            assert sum(1 << b for b in lb) == lane, case  # lperm is a bijection onto lane
            assert bf & ~reg == 0 and bf & seen == 0
            if mf:  # H_16 on neighbouring register-index bits and lane-id bits 4, 5
                assert split and bin(mf).count("1") == 4 and mf & (bf | seen) == 0
                rbits = [b for b in range(tb) if (reg >> b) & 1]
                a = mf_reg_index((reg, bf, lane, wave, lperm, mf))
                assert a + 1 < rb
                assert mf == (1 << rbits[a]) | (1 << rbits[a + 1]) | (1 << lb[4]) | (1 << lb[5]), case
                assert bin(mf & reg).count("1") == 2
            seen |= bf | mf
        assert seen == tmask, case
        # tiles above the half-LDS size transpose through half the LDS
        big = bool(probe.probe_half_lds(prec, tb))
        if kind != "fused":
            assert rounds.half == (big and hi == tb), case
        elif rounds.half:
            assert big and hi == tb and not split, case
        if rounds.half:
            assert all((reg >> (tb - 1)) & 1 for reg, *_ in rounds), case
            assert rounds[0][1] >> (tb - 1) & 1, case  # butterflied in the first round
        if kind == "fused":  # last round holds one shift per thread
            assert rounds[-1][0] & ~((1 << par) - 1) == 0, case
        if split == 2:  # pass-1 store round: lanes on the lowest bits
            assert rounds[-1][1] == 0 and rounds[-1][5] == 0
            assert lane_bits(rounds[-1])[:4] == [0, 1, 2, 3], case
        # first round: the lanes cover the four lowest tile bits outside the
        # registers and the H_16 factor (each wave access spans >= 128
        # contiguous bytes: coalesced global loads); small fused tiles
        # (inputs of at most 2^10 values, cache resident) may trade that for
        # conflict-free LDS slots
        busy = rounds[0][0] | rounds[0][5]
        free = [b for b in range(tb) if not (busy >> b) & 1]
        if not (kind == "fused" and par <= 10):
            assert set(free[:4]) <= set(lane_bits(rounds[0])), case


def test_half_lds_above_64_kib(probe):
    """Two-pass tiles of more than 64 KiB (one workgroup per CU) take the
    half-LDS plans; 64 KiB and less keep full tiles."""
    for prec in (0, 1):
        for tb in range(6, 15):
            big = (8 if prec == 0 else 16) << tb > 65536
            assert bool(probe.probe_half_lds(prec, tb)) == big, (prec, tb)


def test_padding_injective_and_additive(probe):
    """pad is strictly increasing (so injective), additive over disjoint bits
    (the kernels add a register element's pad to the thread's), one tile bit
    moves the slot by 2^(b mod sb) modulo 2^sb, and a 2^tb tile takes
    pad(2^tb - 1) + 1 slots."""
    for sb in (3, 4, 5):
        e = np.arange(1 << 14, dtype=np.int64)
        s = np.array([probe.probe_pad(sb, int(v)) for v in e[:4096]])
        assert np.array_equal(s, pad_np(sb, e[:4096]))
        full = pad_np(sb, e)
        assert np.all(np.diff(full) > 0)
        rng = np.random.default_rng(sb)
        for _ in range(200):
            a = int(rng.integers(0, 1 << 14))
            b = int(rng.integers(0, 1 << 14)) & ~a
            assert full[a | b] == full[a] + full[b]
        for b in range(14):
            assert full[1 << b] % (1 << sb) == (1 << (b % sb)) % (1 << sb)


def test_swizzle_bijective_and_linear(probe):
    for sb in (3, 4, 5):
        e = np.arange(1 << 14, dtype=np.int64)
        s = np.array([probe.probe_swz(sb, int(v)) for v in e[:4096]])
        assert np.array_equal(s, swz_np(sb, e[:4096]))
        full = swz_np(sb, e)
        assert np.array_equal(np.sort(full), e)
        a, b = 0x1234 & 0x3FFF, 0x0F0F & 0x3FFF
        assert swz_np(sb, np.array([a ^ b]))[0] == swz_np(sb, np.array([a]))[0] ^ swz_np(sb, np.array([b]))[0]


def test_lds_layout_per_plan(probe):
    """A plan's LDS is padded exactly when its values are 8 bytes (SB = 5) and
    the padded buffer fits 64 KiB (the reach of the ds instructions' 16-bit
    offsets), and the kernel declares pad(2^t - 1) + 1 values then, else 2^t
    (t = the tile bits in LDS)."""
    seen = set()
    for prec, kind, par, args in all_plans(probe):
        tb, rb, sb, lo, hi, split = args
        rounds = plan(probe, *args, kind=kind)
        if len(rounds) < 2:
            continue
        t = tb - 1 if rounds.half else tb
        padded_bytes = (int(pad_np(sb, np.array([(1 << t) - 1]))[0]) + 1) * (256 >> sb)
        assert rounds.padded == (sb == 5 and padded_bytes <= 65536), (prec, kind, par, args)
        want = padded_bytes // (256 >> sb) if rounds.padded else 1 << t
        assert probe.probe_lds_values(*args, KINDS[kind]) == want
        seen.add(rounds.padded)
    assert seen == {True, False}


def test_lds_bank_slots_distinct(probe):
    """Every LDS access of a round hits 2^SB distinct slots modulo 2^SB in
    each group of 2^SB lanes (256 bytes) and distinct slots modulo 2^(SB-1)
    in each half group (128 bytes per LDS cycle).  Small split-form fused
    tiles (N <= 11) are exempt from the half-group rule and may share a slot
    between two lanes: their matrix-core factor fixes lane-id bits 4 and 5 to
    factor bits, and too few bits are left to choose them from.  16-byte
    values (SB = 4) also meet the rule measured for 16-byte reads: each
    eight-lane group hits eight distinct slots of one 128-byte half of the
    bank row (slot bit 3 equal), and the halves alternate with lane bit 3."""
    for prec, kind, par, args in all_plans(probe):
        tb, rb, sb, lo, hi, split = args
        rounds = plan(probe, *args, kind=kind)
        if len(rounds) == 1:
            continue
        for j, rd in enumerate(rounds):
            M = mapping(rd, tb, rb)
            E = slot_np(rounds, sb, M & ((1 << (tb - 1)) - 1) if rounds.half else M)
            slots = E & ((1 << sb) - 1)
            g = 1 << sb
            T = E.shape[0]
            allowed = 2 if (split and kind == "fused" and par <= 11) else 1
            for t0 in range(0, T, g):
                blk = slots[t0:t0 + g]  # lanes of one group, every register index
                for i in range(blk.shape[1]):
                    ways = np.bincount(blk[:, i], minlength=g).max()
                    assert ways <= allowed, (prec, kind, par, split, j, rd, t0, i)
                    if allowed == 1:  # each 128-byte half group on its own
                        for h in (0, g // 2):
                            half = blk[h:h + g // 2, i] % (g // 2)
                            assert len(set(half.tolist())) == g // 2, (prec, kind, par, split,
                                                                      j, rd, t0, i, h)
            if sb == 4:
                for t0 in range(0, T, 64):
                    for i in range(slots.shape[1]):
                        w = slots[t0:t0 + 64, i]
                        for q in range(len(w) // 8):
                            grp = w[8 * q:8 * q + 8]
                            assert len(set(grp.tolist())) == 8, (prec, kind, par, j, t0, i, q)
                            assert set((grp >> 3).tolist()) == {(w[0] >> 3) ^ (q & 1)}, (
                                prec, kind, par, j, t0, i, q)


def test_tile_transform_matches_wht(probe):
    rng = np.random.default_rng(3)
    for prec, kind, par, (tb, rb, sb, lo, hi, split) in all_plans(probe):
        X = rng.standard_normal(1 << tb) + 1j * rng.standard_normal(1 << tb)
        out = run_tile(X, plan(probe, tb, rb, sb, lo, hi, split, kind), tb, rb, sb)
        assert np.allclose(out, wht_bits(X, lo, hi)), (prec, kind, par, split)


def insert0(v, hb):
    return ((v >> hb) << (hb + 1)) | (v & ((1 << hb) - 1))


def reduce4(v, herm):
    if herm:  # Hermitian pair: 16 (Re^4 + Im^4)
        return 16.0 * np.sum(v.real ** 4 + v.imag ** 4)
    return np.sum(np.abs(v) ** 4)


def test_gather_address_decomposition(probe):
    """The gathers of f_x split each index into a per-thread and a uniform
    per-register-element part: with e = base | r (disjoint bits, r inside the
    first round's register mask REG), e ^ x = (base ^ (x & ~REG)) +
    (r ^ (x & REG)); in the Hermitian one-shift tiles k = insert0(e, hb) =
    insert0(base, hb) + insert0(r, hb) and k ^ x splits the same way over
    R = insert0(REG, hb).  Checked on every first round of the fused and
    pass-1 plans, for random shifts."""
    rng = np.random.default_rng(7)
    for prec, kind, par, args in all_plans(probe):
        if kind == "pass2":
            continue
        tb, rb, sb, lo, hi, split = args
        rd = plan(probe, *args, kind=kind)[0]
        reg = rd[0] & ((1 << tb) - 1)
        M = mapping(rd, tb, rb)
        base = M[:, :1]
        r = pdep(np.arange(1 << rb, dtype=np.int64), reg)[None, :]
        assert np.all((base & r) == 0) and np.all((base | r) == M)
        for x in rng.integers(1, 1 << (tb + 1), size=12):
            x = int(x)
            xl = x & ((1 << tb) - 1)
            assert np.array_equal(M ^ xl, (base ^ (xl & ~reg)) + (r ^ (xl & reg)))
            hb = x.bit_length() - 1  # Hermitian tiles: shifts of tb + 1 bits
            R = insert0(reg, hb)
            kb, kr = insert0(base, hb), insert0(r, hb)
            k = insert0(M, hb)
            assert np.array_equal(k, kb + kr)
            assert np.array_equal(k ^ x, (kb ^ (x & ~R)) + (kr ^ (x & R)))


def emulate_fused_partials(probe, psi, prec, herm=False, x_begin=0, split=0):
    """Per-shift sums exactly as k_fused indexes them (tile of 2^(TB-NT) shifts)."""
    N = psi.size.bit_length() - 1
    NT = N - int(herm)
    tb, _, sb = geo(probe, prec, FUSED, NT)
    rb = fusedrb(probe, prec, NT, split)
    rounds = plan(probe, tb, rb, sb, 0, NT, 3 * split, "fused")
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


def emulate_two_pass_partials(probe, psi, prec, xs, herm=False, split=0, L=None):
    """Per-shift sums as k_pass1 / k_pass2 index them (row slab, then columns);
    L overrides the slab's pass-1 row bits (the kernels are generic in it)."""
    N = psi.size.bit_length() - 1
    NS = N - int(herm)
    L0, _, sb = geo(probe, prec, PASS1, NS)
    L = L0 if L is None else L
    rb1 = p1rb(probe, prec, L, split)
    HT = NS - L
    tb2, rb2, _ = geo(probe, prec, PASS2, HT)
    p1 = plan(probe, L, rb1, sb, 0, L, 2 * split, "pass1")
    p2 = plan(probe, tb2, rb2, sb, tb2 - HT, tb2, split, "pass2")
    e1 = np.arange(1 << L)
    e2 = np.arange(1 << tb2)
    cb = tb2 - HT
    srows = np.arange(1 << HT)
    out = []
    for x in xs:
        assert not herm or x >= (1 << L)
        rows = insert0(srows, x.bit_length() - 1 - L) if herm else srows
        rowbase = (rows << L)[:, None]
        prow = rowbase ^ (x & ~((1 << L) - 1))
        X = np.conj(psi[prow + (e1 ^ (x & ((1 << L) - 1)))[None, :]]) * psi[rowbase + e1[None, :]]
        slab = run_tile(X, p1, L, rb1, sb).reshape(-1)  # all rows at once
        cts = np.arange(1 << (L - cb))[:, None]
        src = (e2 >> cb << L)[None, :] + (cts << cb) + (e2 & ((1 << cb) - 1))[None, :]
        out.append(reduce4(run_tile(slab[src], p2, tb2, rb2, sb), herm))
    return np.array(out)


@pytest.mark.parametrize("prec,N,herm,split", [
    (0, 6, False, 0), (0, 9, False, 0), (1, 5, False, 0), (1, 8, False, 0), (0, 6, True, 0),
    (0, 9, True, 0), (1, 5, True, 0), (1, 8, True, 0), (0, 6, False, 1), (0, 9, False, 1),
    (0, 7, True, 1)])
def test_fused_indexing_matches_oracle(probe, oracle_mod, prec, N, herm, split):
    psi = W.haar(N, 42 + N)
    x0 = 1 if herm else 0
    S = emulate_fused_partials(probe, psi, prec, herm, x0, split)
    ref = oracle_mod.partials(psi)[x0:]
    assert np.allclose(S, ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("prec", [0, 1])
def test_fused_largest_tiles_match_oracle(probe, oracle_mod, prec):
    """The largest fused tile (2^14 complex64 / 2^13 complex128) on its
    last shifts, in the plan and register count the kernel takes."""
    N = geo(probe, prec, LIMITS)[0]
    tb, rb, sb = geo(probe, prec, FUSED, N)
    assert rb == fusedrb(probe, prec, N)
    psi = W.haar(N, 77)
    x0 = (1 << N) - 3
    S = emulate_fused_partials(probe, psi, prec, False, x0)
    assert np.allclose(S, oracle_mod.partials(psi, np.arange(x0, 1 << N)), rtol=1e-11, atol=0)


@pytest.mark.parametrize("prec,extra,herm,split", [
    (0, 1, False, 0), (0, 3, False, 0), (1, 1, False, 0), (1, 3, False, 0), (0, 1, True, 0),
    (0, 3, True, 0), (1, 1, True, 0), (1, 3, True, 0), (0, 1, False, 1), (0, 3, True, 1)])
def test_two_pass_indexing_matches_oracle(probe, oracle_mod, prec, extra, herm, split):
    fmax, L, _ = geo(probe, prec, LIMITS)
    N = fmax + extra
    psi = W.haar(N, 7)
    if herm:
        xs = [1 << L, (1 << N) - 1, 0x2A5A % (1 << N) | (1 << L), 1 << (N - 1), 3 << (N - 2)]
    else:
        xs = [0, 1, (1 << N) - 1, 0x2A5A % (1 << N), 1 << (N - 1)]
    S = emulate_two_pass_partials(probe, psi, prec, xs, herm, split)
    ref = oracle_mod.partials(psi, xs)
    assert np.allclose(S, ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("prec,L,herm,split", [(0, 13, False, 0), (0, 14, False, 0),
                                               (0, 14, True, 0), (0, 13, False, 1),
                                               (0, 14, False, 1), (1, 12, False, 0),
                                               (1, 13, True, 0)])
def test_two_pass_long_rows_match_oracle(probe, oracle_mod, prec, L, herm, split):
    """Pass-1 rows longer than the smallest row (taken by large slabs), on a
    small slab: every row and column tile of the longer-row kernels."""
    _, row, nmax = geo(probe, prec, LIMITS)
    assert L > row
    assert any(geo(probe, prec, PASS1, NS)[0] == L for NS in range(row, nmax + 1))
    N = L + 3 + int(herm)
    psi = W.haar(N, 13 + L)
    xs = [1 << L, (1 << N) - 1] if herm else [0, (1 << N) - 1 - 0x155, 1 << (N - 1)]
    S = emulate_two_pass_partials(probe, psi, prec, xs, herm, split, L=L)
    assert np.allclose(S, oracle_mod.partials(psi, xs), rtol=1e-11, atol=0)


def remove_bit(v, b):
    return ((v >> (b + 1)) << b) | (v & ((1 << b) - 1))


def popc_np(v):
    v = np.asarray(v, dtype=np.int64)
    c = np.zeros_like(v)
    while np.any(v):
        c += v & 1
        v = v >> 1
    return c


def half_row_bit(xh, pref):
    p = xh & pref
    return (p & -p).bit_length() - 1 if p else xh.bit_length() - 1


def pair_sources(rd, tb, rb, cb, L, x, ct):
    """Row-pair pass-2 loads exactly as k_pass2<PAIR> forms them, per thread
    and register element: offset in the shift's half slab and the sign flips
    of the real and imaginary parts (1 = flip)."""
    reg = rd[0] & ((1 << tb) - 1)
    M = mapping(rd, tb, rb)
    base = M[:, :1]
    r = pdep(np.arange(1 << rb, dtype=np.int64), reg)[None, :]
    cmask = (1 << cb) - 1
    rrow = reg >> cb
    xh, xl = x >> L, x & ((1 << L) - 1)
    j = half_row_bit(xh, rrow)
    rowT, colT = base >> cb, base & cmask
    vb0 = (remove_bit(rowT, j) << L) + colT
    vb1 = (remove_bit(rowT ^ (xh & ~rrow), j) << L) + colT
    cto = ct << cb
    mT = (popc_np(colT & xl) ^ popc_np(np.array(cto & xl))) & 1
    R, cr = r >> cb, r & cmask
    sc = popc_np(cr & xl) & 1
    if (rrow >> j) & 1:
        flag = (R >> j) & 1
        off = np.where(flag, vb1 + (remove_bit(R ^ (xh & rrow), j) << L) + cto + cr,
                       vb0 + (remove_bit(R, j) << L) + cto + cr)
        m = np.where(flag, mT ^ sc, 0)
        return M, j, off, m, np.where(flag, m ^ 1, 0)
    ft = (rowT >> j) & 1
    off = np.where(ft, vb1, vb0) + (remove_bit(R, j) << L) + cto + cr
    m = ft & (mT ^ sc)
    return M, j, off, m, m ^ ft


def pair_shifts(rd, tb, cb, N, L, rng):
    """Shifts x >= 2^L of N bits: random ones, each single row bit, and row
    parts on thread row bits only (the pair_load_thr case)."""
    HT = N - L
    rrow = (rd[0] & ((1 << tb) - 1)) >> cb
    trow = ((1 << HT) - 1) & ~rrow
    xs = [int(v) for v in rng.integers(1 << L, 1 << N, size=6)]
    xs += [(1 << (L + b)) | int(rng.integers(0, 1 << L)) for b in range(HT)]
    if trow:
        xs += [((int(rng.integers(1, 1 << HT)) & trow or (trow & -trow)) << L)
               | int(rng.integers(0, 1 << L)) for _ in range(4)]
    return xs


def test_row_pair_sources(probe):
    """Every pass-2 plan (both precisions and the split form, every row
    count H): the row-pair
    loads fetch, for tile element e = (row r, column c) of column tile ct, the
    stored row remove_bit(r, j) when bit j of r is clear, else the partner
    remove_bit(r ^ xh, j) with the real part negated iff
    popcount(z & xl) is odd and the imaginary part iff it is even
    (z = ct 2^cb + c): row(r ^ xh)[z] = (-1)^popcount(z & xl) conj row(r)[z]."""
    rng = np.random.default_rng(11)
    for prec, split in ((0, 0), (1, 0), (0, 1)):
        fmax, _, nmax = geo(probe, prec, LIMITS)
        for N in range(fmax + 1, nmax + 1):
            L = geo(probe, prec, PASS1, N)[0]
            HT = N - L
            tb, rb, sb = geo(probe, prec, PASS2, HT)
            cb = tb - HT
            rd = plan(probe, tb, rb, sb, cb, tb, split, "pass2")[0]
            for x in pair_shifts(rd, tb, cb, N, L, rng):
                for ct in (0, (1 << (L - cb)) - 1):
                    M, j, off, fx, fy = pair_sources(rd, tb, rb, cb, L, x, ct)
                    xh, xl = x >> L, x & ((1 << L) - 1)
                    assert (xh >> j) & 1
                    row, c = M >> cb, M & ((1 << cb) - 1)
                    z = (ct << cb) + c
                    part = (row >> j) & 1
                    want = np.where(part, remove_bit(row ^ xh, j), remove_bit(row, j)) << L
                    assert np.array_equal(off, want + z), (prec, N, x, ct)
                    sig = popc_np(z & xl) & 1
                    assert np.array_equal(fx, np.where(part, sig, 0)), (prec, N, x)
                    assert np.array_equal(fy, np.where(part, sig ^ 1, 0)), (prec, N, x)
                    assert off.min() >= 0 and off.max() < 1 << (N - 1)


def emulate_row_pairs(probe, psi, prec, xs, split=0):
    """Per-shift sums with row-pair slabs: pass 1 builds only the rows with
    bit j clear (j preferred among the register row bits of pass 2's plan,
    the split form's own plan in the split form), pass 2 loads through
    pair_sources."""
    N = psi.size.bit_length() - 1
    L, _, sb = geo(probe, prec, PASS1, N)
    rb1 = p1rb(probe, prec, L, split)
    HT = N - L
    tb2, rb2, _ = geo(probe, prec, PASS2, HT)
    cb = tb2 - HT
    p1 = plan(probe, L, rb1, sb, 0, L, 2 * split, "pass1")
    p2 = plan(probe, tb2, rb2, sb, cb, tb2, split, "pass2")
    rrow = (p2[0][0] & ((1 << tb2) - 1)) >> cb
    e1 = np.arange(1 << L)
    out = []
    for x in xs:
        assert x >= 1 << L
        j = half_row_bit(x >> L, rrow)
        rows = insert0(np.arange(1 << (HT - 1)), j)
        rowbase = (rows << L)[:, None]
        prow = rowbase ^ (x & ~((1 << L) - 1))
        X = np.conj(psi[prow + (e1 ^ (x & ((1 << L) - 1)))[None, :]]) * psi[rowbase + e1[None, :]]
        half = run_tile(X, p1, L, rb1, sb).reshape(-1)
        acc = 0.0
        for ct in range(1 << (L - cb)):
            M, _, off, fx, fy = pair_sources(p2[0], tb2, rb2, cb, L, x, ct)
            v = half[off]
            v = np.where(fx, -1.0, 1.0) * v.real + 1j * np.where(fy, -1.0, 1.0) * v.imag
            tile = np.zeros(1 << tb2, dtype=np.complex128)
            tile[M] = v
            acc += reduce4(run_tile(tile, p2, tb2, rb2, sb), False)
        out.append(acc)
    return np.array(out)


@pytest.mark.parametrize("prec,extra,split", [(0, 1, 0), (0, 3, 0), (1, 1, 0), (1, 3, 0),
                                               (0, 1, 1), (0, 3, 1)])
def test_row_pairs_match_oracle(probe, oracle_mod, prec, extra, split):
    fmax, L, _ = geo(probe, prec, LIMITS)
    N = fmax + extra
    psi = W.haar(N, 17)
    L = geo(probe, prec, PASS1, N)[0]
    xs = [1 << L, (1 << N) - 1, 0x2A5A % (1 << N) | (1 << L), 1 << (N - 1), 3 << (N - 2),
          (1 << L) | 5]
    S = emulate_row_pairs(probe, psi, prec, xs, split)
    assert np.allclose(S, oracle_mod.partials(psi, xs), rtol=1e-11, atol=0)


def _fwht_rows_f32(re, im):
    """Unnormalised FWHT along the last axis in float32, one stage per bit
    ((u, v) -> (u + v, u - v)), every operation rounded to float32."""
    re, im = re.copy(), im.copy()
    n = re.shape[-1]
    h = 1
    while h < n:
        a = re.reshape(re.shape[:-1] + (n // (2 * h), 2, h))
        b = im.reshape(im.shape[:-1] + (n // (2 * h), 2, h))
        ua, va = a[..., 0, :].copy(), a[..., 1, :].copy()
        ub, vb = b[..., 0, :].copy(), b[..., 1, :].copy()
        a[..., 0, :], a[..., 1, :] = ua + va, ua - va
        b[..., 0, :], b[..., 1, :] = ub + vb, ub - vb
        h *= 2
    return re, im


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_row_pair_identity_is_exact_in_float32(seed):
    """The identity the row pairs rely on, in IEEE float32 with every
    operation rounded: the row transform of slab row r ^ xh equals
    (-1)^popcount(z & xl) conj of that of row r bit for bit, when the
    products conj(a) b round their imaginary part as two products and a
    difference (the real part is symmetric in a and b either way)."""
    rng = np.random.default_rng(seed)
    N, L = 10, 6
    psi = (rng.standard_normal(1 << N) + 1j * rng.standard_normal(1 << N)).astype(np.complex64)
    pr, pi = psi.real.astype(np.float32), psi.imag.astype(np.float32)
    k = np.arange(1 << N)
    for x in rng.integers(1 << L, 1 << N, size=8):
        x = int(x)
        a_r, a_i = pr[k ^ x], pi[k ^ x]
        # conj(a) * b with a = psi[k ^ x], b = psi[k]
        fr = (a_r * pr + a_i * pi).astype(np.float32)
        fi = ((a_r * pi).astype(np.float32) - (a_i * pr).astype(np.float32)).astype(np.float32)
        rows_r, rows_i = _fwht_rows_f32(fr.reshape(-1, 1 << L), fi.reshape(-1, 1 << L))
        xh, xl = x >> L, x & ((1 << L) - 1)
        z = np.arange(1 << L)
        neg = (popc_np(z & xl) & 1).astype(bool)
        for r in range(1 << (N - L)):
            want_r = np.where(neg, -rows_r[r], rows_r[r])
            want_i = np.where(neg, rows_i[r], -rows_i[r])
            assert np.array_equal(rows_r[r ^ xh].view(np.uint32), want_r.view(np.uint32))
            assert np.array_equal(rows_i[r ^ xh].view(np.uint32), want_i.view(np.uint32))
