// sre2_geometry.h - tile geometry of every kernel of libsre2 (compile-time).
// Shared by the kernels and by the host-side plan checks, so both see the
// same layouts.
#pragma once
#include "sre2_plan.h"

namespace sre2 {

constexpr int kMaxNAll = 26;

// ---------------------------------------------------------------------------
// Tile geometry per kernel (compile-time; the macros exist for tuning sweeps).
//   RB_*        log2 of complex values per thread
//   FUSED_MIN   smallest fused tile (tiles of smaller N hold several shifts)
//   FUSED_MAX   largest N evaluated by the fused kernel
//   ROW         smallest row bits L of pass 1 (its tile is exactly one row)
//   P2_ROWS     largest number of row bits H = NS - L left to pass 2 while L
//               can still grow (up to the largest tile): with H <= P2_ROWS a
//               pass-2 tile holds at least 128 contiguous bytes of every row
//   P2_MIN      smallest pass-2 tile; a pass-2 tile holds all 2^H rows and at
//               least 2^P2_COLS consecutive columns when the LDS allows it
// ---------------------------------------------------------------------------
#ifndef SRE2_F32_RB_FUSED
#define SRE2_F32_RB_FUSED 5
#endif
#ifndef SRE2_F32_FUSED_MIN
#define SRE2_F32_FUSED_MIN 12
#endif
#ifndef SRE2_F32_FUSED_MAX
#define SRE2_F32_FUSED_MAX 14
#endif
#ifndef SRE2_F32_ROW
#define SRE2_F32_ROW 12
#endif
#ifndef SRE2_F32_RB1
#define SRE2_F32_RB1 4
#endif
#ifndef SRE2_F32_RB2
#define SRE2_F32_RB2 5
#endif
#ifndef SRE2_F32_P2_MIN
#define SRE2_F32_P2_MIN 12
#endif
#ifndef SRE2_F32_P2_COLS
#define SRE2_F32_P2_COLS 4
#endif
#ifndef SRE2_P2_ROWS
#define SRE2_P2_ROWS 10
#endif
#ifndef SRE2_F64_RB_FUSED
#define SRE2_F64_RB_FUSED 4
#endif
#ifndef SRE2_F64_FUSED_MIN
#define SRE2_F64_FUSED_MIN 11
#endif
#ifndef SRE2_F64_FUSED_MAX
#define SRE2_F64_FUSED_MAX 13
#endif
#ifndef SRE2_F64_ROW
#define SRE2_F64_ROW 11
#endif
#ifndef SRE2_F64_RB1
#define SRE2_F64_RB1 4
#endif
#ifndef SRE2_F64_RB2
#define SRE2_F64_RB2 4
#endif
#ifndef SRE2_F64_P2_MIN
#define SRE2_F64_P2_MIN 11
#endif
#ifndef SRE2_F64_P2_COLS
#define SRE2_F64_P2_COLS 3
#endif

template <typename Real> struct Tune;
template <> struct Tune<float> {
    static constexpr int RBF = SRE2_F32_RB_FUSED, FMIN = SRE2_F32_FUSED_MIN;
    static constexpr int FMAX = SRE2_F32_FUSED_MAX, ROW = SRE2_F32_ROW;
    static constexpr int RB1 = SRE2_F32_RB1, RB2 = SRE2_F32_RB2, P2MIN = SRE2_F32_P2_MIN;
    static constexpr int P2COLS = SRE2_F32_P2_COLS;
};
template <> struct Tune<double> {
    static constexpr int RBF = SRE2_F64_RB_FUSED, FMIN = SRE2_F64_FUSED_MIN;
    static constexpr int FMAX = SRE2_F64_FUSED_MAX, ROW = SRE2_F64_ROW;
    static constexpr int RB1 = SRE2_F64_RB1, RB2 = SRE2_F64_RB2, P2MIN = SRE2_F64_P2_MIN;
    static constexpr int P2COLS = SRE2_F64_P2_COLS;
};

// Row bits of pass 1 for a slab of NS bits (NS = N, or N - 1 in the
// Hermitian-pair forms): ROW, grown so that pass 2 keeps at most P2_ROWS row
// bits, up to the largest tile.  Longer rows cost pass 1 some occupancy but
// keep pass 2's column reads in full 128-byte segments, which pays from
// NS = 23 (FP32) / 22 (FP64) on.
template <typename Real>
constexpr int row_bits_of(int NS) {
    int L = NS - SRE2_P2_ROWS;
    if (L < Tune<Real>::ROW) L = Tune<Real>::ROW;
    if (L > Prec<Real>::MAXTB) L = Prec<Real>::MAXTB;
    return L;
}

// Two-pass tiles above 64 KiB (2^14 complex64, 2^13 complex128) transpose
// through half the LDS (make_plan_half, make_split_plan_half), so that two
// workgroups fit a CU; pass 1 then takes one more register bit per thread, so
// that the round count stays that of the smaller tile.  Fused tiles: see
// fused_half.
#ifndef SRE2_HALF_ABOVE
#define SRE2_HALF_ABOVE 65536  // bytes of a tile above which it goes half-LDS
#endif
#ifndef SRE2_P1_HALF_RB
#define SRE2_P1_HALF_RB 1
#endif
template <typename Real>
constexpr bool half_lds(int tb) {
    return ((int64_t)(2 * sizeof(Real)) << tb) > SRE2_HALF_ABOVE;
}
template <typename Real>
constexpr int pass1_rb(int tb, bool split) {
    (void)split;  // the split form takes the same geometry
    return Tune<Real>::RB1 + (half_lds<Real>(tb) ? SRE2_P1_HALF_RB : 0);
}

template <typename Real>
constexpr int fused_tb(int N) {
    return N > Tune<Real>::FMIN ? N : Tune<Real>::FMIN;
}
// Half-LDS fused tiles (plain forms) take SRE2_FUSED_HALF_RB more register
// bits per thread.  Measured on the largest tiles: the FP64 one (2^13) runs
// 1.7x faster so; the FP32 one (2^14, 64 values per thread) spills at the
// 256 registers that two workgroups per CU leave and runs 1.7x slower, so it
// keeps its full tile.
#ifndef SRE2_F32_FUSED_HALF
#define SRE2_F32_FUSED_HALF 0
#endif
#ifndef SRE2_F64_FUSED_HALF
#define SRE2_F64_FUSED_HALF 1
#endif
#ifndef SRE2_F32_FUSED_HALF_RB
#define SRE2_F32_FUSED_HALF_RB 1
#endif
#ifndef SRE2_F64_FUSED_HALF_RB
#define SRE2_F64_FUSED_HALF_RB 1
#endif
template <typename Real>
constexpr bool fused_half(int N) {
    return (sizeof(Real) == 4 ? SRE2_F32_FUSED_HALF : SRE2_F64_FUSED_HALF) &&
           half_lds<Real>(fused_tb<Real>(N)) && N == fused_tb<Real>(N);
}
// Registers (log2) per fused thread for transforms of N bits.
template <typename Real>
constexpr int fused_rb(int N, bool split) {
    return Tune<Real>::RBF +
           (!split && fused_half<Real>(N)
                ? (sizeof(Real) == 4 ? SRE2_F32_FUSED_HALF_RB : SRE2_F64_FUSED_HALF_RB)
                : 0);
}
template <typename Real>
constexpr int pass2_tb(int H) {
    const int want = H + Tune<Real>::P2COLS;
    int tb = want > Tune<Real>::P2MIN ? want : Tune<Real>::P2MIN;
    if (tb > Prec<Real>::MAXTB) tb = Prec<Real>::MAXTB;
    if (tb < H) tb = H;
    if (tb < Tune<Real>::RB2 + 6) tb = Tune<Real>::RB2 + 6;
    return tb;
}

static_assert(Tune<float>::FMAX <= Prec<float>::MAXTB && Tune<double>::FMAX <= Prec<double>::MAXTB);
static_assert(Tune<float>::ROW <= Tune<float>::FMAX && Tune<double>::ROW <= Tune<double>::FMAX);
// every tile holds at least one full wave of threads
static_assert(Tune<float>::FMIN >= Tune<float>::RBF + 6 && Tune<double>::FMIN >= Tune<double>::RBF + 6);
static_assert(Tune<float>::ROW >= Tune<float>::RB1 + 6 && Tune<double>::ROW >= Tune<double>::RB1 + 6);
// Largest N per precision: a pass-2 tile must hold all 2^(N - ROW) rows.
template <typename Real>
constexpr int max_n_of() {
    return kMaxNAll < Tune<Real>::ROW + Prec<Real>::MAXTB ? kMaxNAll : Tune<Real>::ROW + Prec<Real>::MAXTB;
}

// A pass-2 tile reads whole columns inside one row of pass 1's output, and
// every slab size above the fused range splits into valid rows and columns.
template <typename Real>
constexpr bool pass2_tiles_fit() {
    for (int NS = Tune<Real>::FMAX; NS <= max_n_of<Real>(); ++NS) {
        const int L = row_bits_of<Real>(NS), H = NS - L;
        if (H < 1 || L < Tune<Real>::RB1 + 6 || L > Prec<Real>::MAXTB) return false;
        const int tb = pass2_tb<Real>(H);
        if (tb < H || tb - H > L || tb > Prec<Real>::MAXTB) return false;
    }
    return true;
}
// Largest pass-2 row count over all slab sizes.
template <typename Real>
constexpr int pass2_max_rows() {
    int h = 0;
    for (int NS = Tune<Real>::FMAX; NS <= max_n_of<Real>(); ++NS)
        if (NS - row_bits_of<Real>(NS) > h) h = NS - row_bits_of<Real>(NS);
    return h;
}
static_assert(pass2_tiles_fit<float>() && pass2_tiles_fit<double>());

}  // namespace sre2
