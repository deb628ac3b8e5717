// Host-only probe of the tile-engine layout plans (sre2_plan.h) and of the
// kernels' tile geometry (sre2_geometry.h), compiled with g++ by
// tests/test_plan.py so the layouts can be checked without a GPU.
#define __host__
#define __device__
#include "../paper_2512_24685_amd/csrc/sre2_geometry.h"

namespace {
template <typename Real>
int geometry(int kind, int param, int* tb, int* rb, int* sb) {
    using T = sre2::Tune<Real>;
    *sb = sre2::Prec<Real>::SB;
    switch (kind) {
        case 0:  // fused, param = N
            if (param < T::RBF || param > T::FMAX) return -1;
            *tb = sre2::fused_tb<Real>(param);
            *rb = sre2::fused_rb<Real>(param, false);
            return 0;
        case 1:  // pass 1, param = slab bits NS (0: the smallest row); plain forms
            *tb = param ? sre2::row_bits_of<Real>(param) : T::ROW;
            *rb = sre2::pass1_rb<Real>(*tb, false);
            return 0;
        case 2:  // pass 2, param = H
            if (param < 1 || param > sre2::pass2_max_rows<Real>()) return -1;
            *tb = sre2::pass2_tb<Real>(param);
            *rb = T::RB2;
            return 0;
        case 3:  // limits: tb = largest fused N, rb = smallest row bits, sb = largest N
            *tb = T::FMAX;
            *rb = T::ROW;
            *sb = sre2::max_n_of<Real>();
            return 0;
    }
    return -1;
}
}  // namespace

extern "C" {

// precision 0 = float (complex64 tiles), 1 = double (complex128 tiles)
int probe_geometry(int precision, int kind, int param, int* tb, int* rb, int* sb) {
    return precision == 0 ? geometry<float>(kind, param, tb, rb, sb)
                          : geometry<double>(kind, param, tb, rb, sb);
}

// 1 when tiles of tb bits transpose through half the LDS in two-pass kernels.
int probe_half_lds(int precision, int tb) {
    return precision == 0 ? sre2::half_lds<float>(tb) : sre2::half_lds<double>(tb);
}

// Registers per fused thread (log2) for transforms of N bits.
int probe_fused_rb(int precision, int N, int split) {
    return precision == 0 ? sre2::fused_rb<float>(N, split != 0)
                          : sre2::fused_rb<double>(N, split != 0);
}

// Registers per pass-1 thread (log2) for a row of tb bits.
int probe_pass1_rb(int precision, int tb, int split) {
    return precision == 0 ? sre2::pass1_rb<float>(tb, split != 0)
                          : sre2::pass1_rb<double>(tb, split != 0);
}

// Rounds of a plan, six words each: reg, bfly, lane, wave, lperm, mf, as the
// kernel of `kind` (0 fused, 1 pass 1, 2 pass 2) selects it (sb = 5:
// complex64 tiles, 4: complex128).  split = 0: plain plan, otherwise the
// split-FP16 plan with tail split - 1 (0 none, 1 store round, 2 registers
// inside [0, hi) at the end); half-LDS plans for the two-pass tiles above
// 64 KiB and the fused tiles of fused_half.  Returns the round count, plus
// 100 for a half-LDS plan, plus 1000 when its LDS buffer is padded (else
// swizzled).
int probe_plan(int tb, int rb, int sb, int lo, int hi, int split, int kind, unsigned* out) {
    const bool f32 = sb == 5;
    const bool big = f32 ? sre2::half_lds<float>(tb) : sre2::half_lds<double>(tb);
    const bool half =
        kind == 0 ? !split && (f32 ? sre2::fused_half<float>(hi) : sre2::fused_half<double>(hi))
                  : big && hi == tb && lo < tb - 1;
    const sre2::Plan p =
        split ? (half ? sre2::make_split_plan_half(tb, rb, sb, lo, split - 1)
                      : sre2::make_split_plan(tb, rb, sb, lo, hi, split - 1))
              : (half ? sre2::make_plan_half(tb, rb, sb, lo) : sre2::make_plan(tb, rb, sb, lo, hi));
    for (int j = 0; j < p.nrounds; ++j) {
        out[6 * j + 0] = p.r[j].reg;
        out[6 * j + 1] = p.r[j].bfly;
        out[6 * j + 2] = p.r[j].lane;
        out[6 * j + 3] = p.r[j].wave;
        out[6 * j + 4] = p.r[j].lperm;
        out[6 * j + 5] = p.r[j].mf;
    }
    return p.nrounds + (p.half ? 100 : 0) + (sre2::lds_padded(p) ? 1000 : 0);
}

// LDS values a kernel with this plan declares.
int probe_lds_values(int tb, int rb, int sb, int lo, int hi, int split, int kind) {
    unsigned out[48];
    (void)out;
    const bool f32 = sb == 5;
    const bool big = f32 ? sre2::half_lds<float>(tb) : sre2::half_lds<double>(tb);
    const bool half =
        kind == 0 ? !split && (f32 ? sre2::fused_half<float>(hi) : sre2::fused_half<double>(hi))
                  : big && hi == tb && lo < tb - 1;
    const sre2::Plan p =
        split ? (half ? sre2::make_split_plan_half(tb, rb, sb, lo, split - 1)
                      : sre2::make_split_plan(tb, rb, sb, lo, hi, split - 1))
              : (half ? sre2::make_plan_half(tb, rb, sb, lo) : sre2::make_plan(tb, rb, sb, lo, hi));
    return sre2::lds_values(p);
}

unsigned probe_pad(int sb, unsigned e) {
    return sb == 5 ? sre2::pad<5>(e) : sb == 4 ? sre2::pad<4>(e) : sre2::pad<3>(e);
}

unsigned probe_swz(int sb, unsigned e) {
    return sb == 5 ? sre2::swz<5>(e) : sb == 4 ? sre2::swz<4>(e) : sre2::swz<3>(e);
}
}
