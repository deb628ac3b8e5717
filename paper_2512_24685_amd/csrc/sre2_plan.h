// sre2_plan.h - compile-time layout plans for the register/LDS Walsh-Hadamard
// tile engine (gfx950).
//
// A workgroup owns a tile of 2^TB complex values.  Each of its T = 2^(TB-RB)
// threads holds 2^RB of them in registers.  A "round" fixes which TB tile-index
// bits are register bits (RB of them), which 6 are lane bits and which are
// wave bits.  Radix-2 butterflies (a, b) -> (a + b, a - b) act on register bits
// only; between rounds the tile is re-distributed through LDS.  The unnormalised
// Walsh-Hadamard transform is H_2 applied once along every index bit (SI, fast
// WHT section: H_{2^N} = H_2^{(x)N}), and those per-bit stages commute, so any
// order of bits across rounds gives the same transform.
//
// LDS addresses: a slot is one complex value (SB = 5 for 8-byte, 4 for
// 16-byte values: 2^SB slots are 256 bytes, the 64 four-byte banks).
// 8-byte values sit in slot pad(e) = e + (e >> SB) + (e >> 2 SB) + ... of
// tile element e, or, where that padded buffer would not fit 64 KiB, in slot
// swz(e) = e with its low SB bits XORed with every higher SB-bit chunk (a
// bijection, no growth); 16-byte values always take swz.  Under either map
// tile bit b alone moves the slot by 2^(b mod SB) modulo 2^SB.  Measured on
// gfx950 with rocprof's LDS bank-conflict counter:
//  - an 8-byte access is free of conflicts when each group of 32 lanes hits
//    32 distinct slots modulo 32 and, inside it, each half group (128 bytes)
//    distinct slots modulo 16: lane bits 0..3 may map onto slot bits 0..3 in
//    any order, but lane bit 4 must map onto slot bit 4;
//  - a 16-byte read is served eight lanes (128 bytes) at a time: each
//    eight-lane group must hit eight distinct slots of one 128-byte half of
//    the bank row (slot bits 0..2 distinct, bit 3 equal), and consecutive
//    groups must alternate between the halves, i.e. slot bit 3 must follow
//    lane bit 3 and no other lane bit.  (16-byte writes showed no such
//    constraint.)
// So lane bit i of every round sits on a tile bit of residue i mod SB
// (i < SB), and with SB = 4 the lane bits above 3 avoid residue 3.  Lane bits
// of distinct residues contribute distinct powers of two, and the wave and
// register bits the same amount to every lane, so each access is free of
// conflicts.  pad is additive over disjoint bits (pad(a | b) = pad(a) +
// pad(b) when a & b = 0: shifting a carry-free sum carries nothing), so a
// register element's slot is the thread's slot plus a constant, the
// instruction's immediate offset; the swizzle needs one XOR per element.
// Additive padding cannot meet the 16-byte read rule: the lane bits' sums
// carry into slot bit 3.  ds_read / ds_write offsets are 16 bits, so a
// padded buffer above 64 KiB would need address registers instead, which
// costs the largest tiles more than the XOR: those keep the swizzle.
//
// Tiles above 64 KiB would leave one workgroup per CU (160 KiB of LDS); their
// half-LDS plans keep the top tile bit in every round's registers, so each
// transpose moves half the tile at a time through a buffer of 2^(TB-1)
// slots (make_plan_half).
#pragma once
#include <stdint.h>

namespace sre2 {

struct Round {
    uint32_t reg;    // tile bits held in registers (RB bits)
    uint32_t bfly;   // register bits that receive butterflies in this round
    uint32_t lane;   // tile bits indexed by the lane id (6 bits)
    uint32_t wave;   // tile bits indexed by the wave id
    uint32_t lperm;  // tile bit of lane-id bit i, 5 bits each (i = 0..5)
    uint32_t mf;     // split form: the four tile bits of this round's H_16
                     // factor (two neighbouring register-index bits and
                     // lane-id bits 4, 5)
};

// Register-index bit of the lower of a factor's two register bits.
__host__ __device__ constexpr int mf_reg_index(const Round& rd) {
    uint32_t below = 0;
    for (int b = 0; b < 32; ++b)
        if (((rd.mf & rd.reg) >> b) & 1u) {
            below = rd.reg & ((1u << b) - 1u);
            break;
        }
    int n = 0;
    for (int b = 0; b < 32; ++b) n += (below >> b) & 1u;
    return n;
}

// Lane permutation packing: lane-id bit i -> tile bit (lperm >> 5i) & 31.
__host__ __device__ constexpr uint32_t lperm_of_mask(uint32_t lane) {
    uint32_t p = 0;
    int i = 0;
    for (int b = 0; b < 32; ++b)
        if ((lane >> b) & 1u) p |= (uint32_t)b << (5 * i++);
    return p;
}

constexpr int kMaxRounds = 8;
constexpr int kMaxTileBits = 16;

struct Plan {
    int tb = 0, rb = 0, nrounds = 0;
    int sb = 5;  // slot bits of one value (LDS padding period)
    // half: every round holds the top tile bit in its top register-index
    // bit, so each LDS transpose runs in two phases (register halves with
    // that bit 0, then 1) through an LDS buffer of half the tile
    bool half = false;
    Round r[kMaxRounds] = {};
};

__host__ __device__ constexpr int popc(uint32_t v) {
    int c = 0;
    while (v) { c += v & 1u; v >>= 1; }
    return c;
}

__host__ __device__ constexpr uint32_t bits_range(int lo, int hi) {  // [lo, hi)
    uint32_t m = 0;
    for (int b = lo; b < hi; ++b) m |= 1u << b;
    return m;
}

// Parallel bit deposit: the low popc(mask) bits of v go to the set bits of mask.
__host__ __device__ constexpr uint32_t pdep(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
    int k = 0;
    for (int b = 0; b < 32; ++b) {
        if ((mask >> b) & 1u) {
            if ((v >> k) & 1u) r |= 1u << b;
            ++k;
        }
    }
    return r;
}

// Parallel bit extract (inverse of pdep on mask).
__host__ __device__ constexpr uint32_t pext(uint32_t v, uint32_t mask) {
    uint32_t r = 0;
    int k = 0;
    for (int b = 0; b < 32; ++b) {
        if ((mask >> b) & 1u) {
            if ((v >> b) & 1u) r |= 1u << k;
            ++k;
        }
    }
    return r;
}

// Bank swizzle: XOR the low SB bits with every higher SB-bit chunk (GF(2)-linear
// and a bijection on any power-of-two range).
template <int SB>
__host__ __device__ constexpr uint32_t swz(uint32_t e) {
    uint32_t h = e >> SB, f = 0;
    while (h) {
        f ^= h & ((1u << SB) - 1u);
        h >>= SB;
    }
    return e ^ f;
}

// LDS slot of tile element e: pad(e) = sum over j >= 0 of (e >> SB j).
template <int SB>
__host__ __device__ constexpr uint32_t pad(uint32_t e) {
    uint32_t s = 0;
    while (e) {
        s += e;
        e >>= SB;
    }
    return s;
}
// The same sum for e < 2^16 (every tile here has at most 2^14 elements) as a
// fixed, branch-free sequence of shifts and adds, for slots formed at run time.
template <int SB>
__host__ __device__ constexpr uint32_t pad16(uint32_t e) {
    uint32_t s = e;
    for (int j = SB; j < 16; j += SB) s += e >> j;
    return s;
}
__host__ __device__ constexpr uint32_t pad_rt(uint32_t e, int sb) {
    uint32_t s = 0;
    while (e) {
        s += e;
        e >>= sb;
    }
    return s;
}

// LDS layout of a plan: the tile bits held in LDS (a half-LDS plan keeps the
// top bit in registers), whether the buffer is padded (8-byte values, when the
// padded buffer fits 64 KiB) or swizzled, and the values it declares (1 when
// the plan has a single round and no transpose).
__host__ __device__ constexpr int lds_bits(const Plan& P) { return P.half ? P.tb - 1 : P.tb; }
__host__ __device__ constexpr bool lds_padded(const Plan& P) {
    return P.sb >= 5 && (pad_rt((1u << lds_bits(P)) - 1u, P.sb) + 1u) * (256u >> P.sb) <= 65536u;
}
__host__ __device__ constexpr int lds_values(const Plan& P) {
    return P.nrounds < 2 ? 1
                         : (lds_padded(P) ? (int)pad_rt((1u << lds_bits(P)) - 1u, P.sb) + 1
                                          : 1 << lds_bits(P));
}

// Highest `count` set bits of `m`.
__host__ __device__ constexpr uint32_t top_bits(uint32_t m, int count) {
    uint32_t r = 0;
    for (int b = 31; b >= 0 && count > 0; --b)
        if ((m >> b) & 1u) { r |= 1u << b; --count; }
    return r;
}

__host__ __device__ constexpr uint32_t low_bits(uint32_t m, int count) {
    uint32_t r = 0;
    for (int b = 0; b < 32 && count > 0; ++b)
        if ((m >> b) & 1u) { r |= 1u << b; --count; }
    return r;
}

// Lane / wave assignment for a given register mask.
__host__ __device__ constexpr Round make_round(int tb, int sb, uint32_t reg, uint32_t bfly) {
    Round rd{};
    rd.reg = reg;
    rd.bfly = bfly;
    uint32_t free_bits = bits_range(0, tb) & ~reg;
    uint32_t matched = 0;
    for (int i = 0; i < sb && i < 6; ++i) {  // residue-matched lanes
        for (int b = 0; b < tb; ++b) {
            if (((free_bits >> b) & 1u) && (b % sb) == i) {
                matched |= 1u << b;
                free_bits &= ~(1u << b);
                break;
            }
        }
    }
    // lane-id bit i takes the matched bit of residue i, the lowest remaining
    // bits fill the rest; with 16-byte slots (sb = 4) the fill avoids residue
    // 3 where it can, so that slot bit 3 follows lane bit 3 alone
    const int nfill = 6 - popc(matched);
    uint32_t off_top = 0;
    for (int b = 0; b < tb; ++b)
        if (((free_bits >> b) & 1u) && !(sb == 4 && b % sb == sb - 1)) off_top |= 1u << b;
    uint32_t fill = low_bits(off_top, nfill);
    if (popc(fill) < nfill) fill |= low_bits(free_bits & ~fill, nfill - popc(fill));
    uint32_t lp = 0;
    int nl = 0;
    for (int i = 0; i < sb && i < 6; ++i)
        for (int b = 0; b < tb; ++b)
            if (((matched >> b) & 1u) && (b % sb) == i) lp |= (uint32_t)b << (5 * nl++);
    for (int b = 0; b < tb; ++b)
        if ((fill >> b) & 1u) lp |= (uint32_t)b << (5 * nl++);
    rd.lane = matched | fill;
    rd.wave = free_bits & ~fill;
    rd.lperm = lp;
    rd.mf = 0;
    return rd;
}

// Plan for a transform over the tile bits in `tmask` (a contiguous range
// [lo, hi) of the tile index).  The first round holds the top RB transform bits
// in registers, so lanes run over the lowest tile bits (coalesced global loads).
// The second holds the bottom RB transform bits.  The rest follow from the top
// down; the last round is padded with transform bits that are already done,
// taken from the top so that lanes stay on low bits.
__host__ __device__ constexpr Plan make_plan(int tb, int rb, int sb, int lo, int hi) {
    Plan p{};
    p.tb = tb;
    p.rb = rb;
    p.sb = sb;
    const uint32_t tmask = bits_range(lo, hi);
    const int n = hi - lo;
    uint32_t todo = tmask;
    uint32_t done = 0;
    int k = 0;
    if (n <= rb) {
        // Single round: all transform bits plus padding from the bits just above
        // (or below) the range.
        uint32_t reg = tmask;
        uint32_t pad_pool = bits_range(hi, tb);
        reg |= low_bits(pad_pool, rb - n);
        if (popc(reg) < rb) reg |= top_bits(bits_range(0, lo), rb - popc(reg));
        p.r[k++] = make_round(tb, sb, reg, tmask);
        p.nrounds = k;
        return p;
    }
    // round 1: top rb transform bits
    {
        uint32_t reg = top_bits(todo, rb);
        p.r[k++] = make_round(tb, sb, reg, reg);
        todo &= ~reg;
        done |= reg;
    }
    // round 2: bottom rb transform bits (overlapping done bits only if needed)
    {
        uint32_t reg = low_bits(tmask, rb);
        uint32_t b = reg & todo;
        p.r[k++] = make_round(tb, sb, reg, b);
        todo &= ~b;
        done |= b;
    }
    while (todo) {
        int cnt = popc(todo);
        uint32_t b = top_bits(todo, cnt < rb ? cnt : rb);
        uint32_t reg = b;
        if (popc(reg) < rb) reg |= top_bits(done & ~reg, rb - popc(reg));
        p.r[k++] = make_round(tb, sb, reg, b);
        todo &= ~b;
        done |= b;
    }
    p.nrounds = k;
    return p;
}

// Half-LDS plan for a transform over [lo, tb) of a 2^tb tile (lo < tb - 1):
// the plan of the lower tb - 1 bits with rb - 1 registers per thread (its
// lanes, waves, bank residues and round order unchanged), with the top tile
// bit added to every round's registers as the top register-index bit and
// butterflied in the first round.  The thread count is that of the full
// plan, 2^(tb - rb), and each transpose moves half the tile at a time.
__host__ __device__ constexpr Plan make_plan_half(int tb, int rb, int sb, int lo) {
    Plan p = make_plan(tb - 1, rb - 1, sb, lo, tb - 1);
    const uint32_t top = 1u << (tb - 1);
    for (int j = 0; j < p.nrounds; ++j) p.r[j].reg |= top;
    p.r[0].bfly |= top;
    p.tb = tb;
    p.rb = rb;
    p.half = true;
    return p;
}

__host__ __device__ constexpr int high_bit(uint32_t m) {
    int h = -1;
    for (int b = 0; b < 32; ++b)
        if ((m >> b) & 1u) h = b;
    return h;
}

// Pads `reg` up to RB bits with bits of `pool`, from the top, taking only
// bits whose removal leaves a non-register bit of every bank residue mod SB.
__host__ __device__ constexpr uint32_t pad_keeping_residues(uint32_t reg, uint32_t pool, int rb,
                                                           int tb, int sb) {
    for (int b = tb - 1; b >= 0 && popc(reg) < rb; --b) {
        if (!((pool >> b) & 1u) || ((reg >> b) & 1u)) continue;
        const uint32_t rest = bits_range(0, tb) & ~reg & ~(1u << b);
        bool covers = true;
        for (int r = 0; r < sb; ++r) {
            bool any = false;
            for (int c = r; c < tb; c += sb) any = any || ((rest >> c) & 1u);
            covers = covers && any;
        }
        if (covers) reg |= 1u << b;
    }
    return reg;
}

// Round with an H_16 factor on the matrix cores.  MF = {two bits MREG held
// in registers at neighbouring register-index bits, and two bits on lane-id
// bits 4 (L4) and 5}; V = register bits butterflied in FP32.  The other
// RB - 2 - |V| register bits are padding (done bits first, never between the
// factor's register bits); lane-id bits 0..3 (the MFMA's 16 columns) take the
// lowest free bits in the first round (coalesced loads), else bits whose bank
// slots are distinct from each other's and from L4's.
__host__ __device__ constexpr Round make_mf_round_as(int tb, int rb, int sb, uint32_t mf,
                                                     uint32_t mreg, int l4, uint32_t v,
                                                     uint32_t pad_pool, bool first) {
    Round rd{};
    const uint32_t mlane = mf & ~mreg;
    const int l5 = high_bit(mlane & ~(1u << l4));
    const int m0 = high_bit(low_bits(mreg, 1)), m1 = high_bit(mreg);
    const uint32_t between = bits_range(m0 + 1, m1);
    const uint32_t avail = bits_range(0, tb) & ~mreg & ~v & ~mlane & ~between;
    uint32_t reg = pad_keeping_residues(mreg | v, avail & pad_pool, rb, tb, sb);
    reg = pad_keeping_residues(reg, avail, rb, tb, sb);
    reg |= top_bits(avail & ~reg, rb - popc(reg));
    rd.reg = reg;
    rd.bfly = v;
    rd.mf = mf;
    uint32_t free_bits = bits_range(0, tb) & ~reg & ~mlane;
    int cols[4] = {0, 0, 0, 0};
    int nc = 0;
    if (first) {
        for (int b = 0; b < tb && nc < 4; ++b)
            if ((free_bits >> b) & 1u) cols[nc++] = b;
    } else {
        uint32_t used_res = 1u << (l4 % sb);
        for (int b = 0; b < tb && nc < 4; ++b)
            if (((free_bits >> b) & 1u) && !((used_res >> (b % sb)) & 1u)) {
                cols[nc++] = b;
                used_res |= 1u << (b % sb);
            }
        for (int b = 0; b < tb && nc < 4; ++b) {
            bool taken = false;
            for (int j = 0; j < nc; ++j) taken = taken || cols[j] == b;
            if (((free_bits >> b) & 1u) && !taken) cols[nc++] = b;
        }
    }
    uint32_t lane = mlane;
    uint32_t lp = 0;
    for (int j = 0; j < 4; ++j) {
        lane |= 1u << cols[j];
        lp |= (uint32_t)cols[j] << (5 * j);
    }
    lp |= (uint32_t)l4 << 20;
    lp |= (uint32_t)l5 << 25;
    rd.lane = lane;
    rd.lperm = lp;
    rd.wave = bits_range(0, tb) & ~reg & ~lane;
    return rd;
}

// True when lane-id bits 0..SB-2 of a round sit on residues 0..SB-2 (in any
// order) and lane-id bit SB-1 on residue SB-1.
__host__ __device__ constexpr bool lanes_conflict_free(const Round& rd, int sb) {
    if ((int)(((rd.lperm >> (5 * (sb - 1))) & 31u) % sb) != sb - 1) return false;
    uint32_t used = 0;
    for (int i = 0; i < sb && i < 6; ++i) {
        const uint32_t r = 1u << (((rd.lperm >> (5 * i)) & 31u) % sb);
        if (used & r) return false;
        used |= r;
    }
    return true;
}

// The factor's register bits are its two lowest bits and L4 the lower of
// the other two, unless another of the twelve assignments is free of bank
// conflicts where that one is not: in the first round with the lowest-bit
// columns if one allows it, else (every round) with columns chosen by bank
// slot.
__host__ __device__ constexpr Round make_mf_round(int tb, int rb, int sb, uint32_t mf, uint32_t v,
                                                  uint32_t pad_pool, bool first) {
    const uint32_t mreg0 = low_bits(mf, 2);
    const int l40 = high_bit(low_bits(mf & ~mreg0, 1));
    const Round dflt = make_mf_round_as(tb, rb, sb, mf, mreg0, l40, v, pad_pool, first);
    if (lanes_conflict_free(dflt, sb)) return dflt;
    int fb[4] = {0, 0, 0, 0};
    int n = 0;
    for (int b = 0; b < 32; ++b)
        if ((mf >> b) & 1u) fb[n++] = b;
    for (int pass = first ? 0 : 1; pass < 2; ++pass)
        for (int a = 0; a < 4; ++a)
            for (int c = a + 1; c < 4; ++c) {
                const uint32_t mreg = (1u << fb[a]) | (1u << fb[c]);
                for (int k = 0; k < 4; ++k) {
                    if (k == a || k == c) continue;
                    const Round rd =
                        make_mf_round_as(tb, rb, sb, mf, mreg, fb[k], v, pad_pool, pass == 0);
                    if (lanes_conflict_free(rd, sb)) return rd;
                }
            }
    return first ? make_mf_round_as(tb, rb, sb, mf, mreg0, l40, v, pad_pool, false) : dflt;
}

// A first round whose lane-id bits 0..3 run over the four lowest tile bits
// outside its registers and factor, with conflict-free bank slots.
__host__ __device__ constexpr bool first_round_ok(const Round& rd, int tb, int sb) {
    const uint32_t free_bits = bits_range(0, tb) & ~rd.reg & ~rd.mf;
    int j = 0;
    for (int b = 0; b < tb && j < 4; ++b)
        if ((free_bits >> b) & 1u) {
            if (((rd.lperm >> (5 * j)) & 31u) != (uint32_t)b) return false;
            ++j;
        }
    return lanes_conflict_free(rd, sb);
}

// Plan of the split form over tile bits [lo, hi): rounds with an H_16 factor
// plus up to RB - 2 FP32 butterfly bits while at least four bits remain, then
// FP32-only rounds.  A round without arithmetic may close the plan: tail = 1
// puts the lanes on the lowest tile bits (coalesced stores); tail = 2 brings
// the registers inside [0, hi) when they are not (one shift per thread).
__host__ __device__ constexpr Plan make_split_plan(int tb, int rb, int sb, int lo, int hi,
                                                   int tail) {
    Plan p{};
    p.tb = tb;
    p.rb = rb;
    p.sb = sb;
    const uint32_t tmask = bits_range(lo, hi);
    uint32_t todo = tmask, done = 0;
    int k = 0;
    bool first = true;
    while (todo && k < kMaxRounds - 1) {
        const int n = popc(todo);
        if (n >= 4 && rb >= 2) {
            const int nv = (rb - 2) < (n - 4) ? (rb - 2) : (n - 4);
            uint32_t mf = 0, v = 0;
            if (first) {
                // the top 4 + nv bits, the factor on the lowest four of them,
                // unless another four (or, failing that, fewer FP32 bits) give
                // conflict-free lanes on the lowest free bits
                const uint32_t u0 = top_bits(todo, nv + 4);
                mf = low_bits(u0, 4);
                v = u0 & ~mf;
                bool found = first_round_ok(make_mf_round(tb, rb, sb, mf, v, done, true), tb, sb);
                for (int w = nv; w >= 0 && !found; --w) {
                    const uint32_t u = top_bits(todo, w + 4);
                    int ub[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    int nu = 0;
                    for (int b = 0; b < 32; ++b)
                        if ((u >> b) & 1u) ub[nu++] = b;
                    for (uint32_t sel = 0; sel < (1u << nu) && !found; ++sel) {
                        if (popc(sel) != 4) continue;
                        uint32_t m = 0;
                        for (int i = 0; i < nu; ++i)
                            if ((sel >> i) & 1u) m |= 1u << ub[i];
                        if (first_round_ok(make_mf_round(tb, rb, sb, m, u & ~m, done, true), tb, sb)) {
                            mf = m;
                            v = u & ~m;
                            found = true;
                        }
                    }
                }
            } else {
                // the factor on the lowest four bits, unless another four of
                // the remaining bits give conflict-free lanes (lane-id bit
                // SB - 1, a factor bit, needs a tile bit of residue SB - 1)
                mf = low_bits(todo, 4);
                v = top_bits(todo & ~mf, nv);
                if (!lanes_conflict_free(make_mf_round(tb, rb, sb, mf, v, done, false), sb)) {
                    int tbits[kMaxTileBits] = {};
                    int nt = 0;
                    for (int b = 0; b < 32 && nt < kMaxTileBits; ++b)
                        if ((todo >> b) & 1u) tbits[nt++] = b;
                    bool found = false;
                    for (uint32_t sel = 0; sel < (1u << nt) && !found; ++sel) {
                        if (popc(sel) != 4) continue;
                        uint32_t m = 0;
                        for (int i = 0; i < nt; ++i)
                            if ((sel >> i) & 1u) m |= 1u << tbits[i];
                        const uint32_t vv = top_bits(todo & ~m, nv);
                        if (lanes_conflict_free(make_mf_round(tb, rb, sb, m, vv, done, false), sb)) {
                            mf = m;
                            v = vv;
                            found = true;
                        }
                    }
                }
            }
            p.r[k++] = make_mf_round(tb, rb, sb, mf, v, done, first);
            todo &= ~(mf | v);
            done |= mf | v;
        } else {
            // FP32-only round over the remaining bits, padded with done bits
            // (from the top, keeping a free bit of every bank residue)
            uint32_t reg = pad_keeping_residues(todo, done, rb, tb, sb);
            reg |= top_bits(bits_range(0, tb) & ~reg, rb - popc(reg));
            p.r[k++] = make_round(tb, sb, reg, todo);
            done |= todo;
            todo = 0;
        }
        first = false;
    }
    if (tail == 1) p.r[k++] = make_round(tb, sb, top_bits(bits_range(0, tb), rb), 0);
    if (tail == 2 && (p.r[k - 1].reg & ~bits_range(0, hi)))
        p.r[k++] = make_round(tb, sb, top_bits(bits_range(0, hi), rb), 0);
    p.nrounds = k;
    return p;
}

// Per-precision constants: slot bits of one complex value and the largest tile
// that fits the 160 KiB LDS (128 KiB of tile).
template <typename Real> struct Prec;
template <> struct Prec<float> {
    static constexpr int SB = 5;      // 8-byte complex64 slots
    static constexpr int MAXTB = 14;  // 2^14 complex64 = 128 KiB
};
template <> struct Prec<double> {
    static constexpr int SB = 4;      // 16-byte complex128 slots
    static constexpr int MAXTB = 13;  // 2^13 complex128 = 128 KiB
};


// Half-LDS split plan (see make_plan_half): the split plan of the lower
// tb - 1 bits with rb - 1 registers per thread, plus the top tile bit as the
// top register-index bit of every round, butterflied in FP32 in the first.
__host__ __device__ constexpr Plan make_split_plan_half(int tb, int rb, int sb, int lo, int tail) {
    Plan p = make_split_plan(tb - 1, rb - 1, sb, lo, tb - 1, tail);
    const uint32_t top = 1u << (tb - 1);
    for (int j = 0; j < p.nrounds; ++j) p.r[j].reg |= top;
    p.r[0].bfly |= top;
    p.tb = tb;
    p.rb = rb;
    p.half = true;
    return p;
}

}  // namespace sre2
