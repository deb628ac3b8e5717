// Host-only probe of the tile-engine layout plans (sre2_plan.h), compiled with
// g++ by tests/test_plan.py so the plans can be checked on a machine without a
// GPU.  It exposes exactly the constexpr plan builder the kernels use.
#define __host__
#define __device__
#include "../paper_2512_24685_amd/csrc/sre2_plan.h"

extern "C" {

// precision 0 = float (complex64 tiles), 1 = double (complex128 tiles)
void probe_geo(int precision, int* tb, int* rb, int* sb) {
    if (precision == 0) {
        *tb = sre2::Geo<float>::TB;
        *rb = sre2::Geo<float>::RB;
        *sb = sre2::Geo<float>::SB;
    } else {
        *tb = sre2::Geo<double>::TB;
        *rb = sre2::Geo<double>::RB;
        *sb = sre2::Geo<double>::SB;
    }
}

int probe_plan(int tb, int rb, int sb, int lo, int hi, unsigned* out) {
    const sre2::Plan p = sre2::make_plan(tb, rb, sb, lo, hi);
    for (int j = 0; j < p.nrounds; ++j) {
        out[4 * j + 0] = p.r[j].reg;
        out[4 * j + 1] = p.r[j].bfly;
        out[4 * j + 2] = p.r[j].lane;
        out[4 * j + 3] = p.r[j].wave;
    }
    return p.nrounds;
}

unsigned probe_swz(int sb, unsigned e) {
    return sb == 5 ? sre2::swz<5>(e) : sre2::swz<4>(e);
}
}
