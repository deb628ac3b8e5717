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
// LDS addresses are XOR-swizzled: tile bit b feeds bank slot bit (b mod SB),
// where a slot is one complex value (SB = 5 for 8-byte, 4 for 16-byte values).
// Lane bits 0..SB-1 of every round are placed on tile bits with distinct
// residues mod SB, so each group of 2^SB lanes touches 2^SB distinct slots.
#pragma once
#include <stdint.h>

namespace sre2 {

struct Round {
    uint32_t reg;   // tile bits held in registers (RB bits)
    uint32_t bfly;  // register bits that receive butterflies in this round
    uint32_t lane;  // tile bits indexed by the lane id (6 bits)
    uint32_t wave;  // tile bits indexed by the wave id
};

constexpr int kMaxRounds = 8;

struct Plan {
    int tb = 0, rb = 0, nrounds = 0;
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
    uint32_t lane = 0;
    int nl = 0;
    for (int i = 0; i < sb && i < 6; ++i) {  // residue-matched lanes
        for (int b = 0; b < tb; ++b) {
            if (((free_bits >> b) & 1u) && (b % sb) == i) {
                lane |= 1u << b;
                free_bits &= ~(1u << b);
                ++nl;
                break;
            }
        }
    }
    while (nl < 6) {  // fill with the lowest remaining bits
        uint32_t b = low_bits(free_bits, 1);
        if (!b) break;
        lane |= b;
        free_bits &= ~b;
        ++nl;
    }
    rd.lane = lane;
    rd.wave = free_bits;
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

}  // namespace sre2
