// sre2_queries.hip - host-side geometry queries of the kernels (which N take
// the fused kernel, pass-1 row bits, pass-2 column tiles), answered from the
// compile-time tile geometry of sre2_geometry.h that the kernels use.
#include <stdint.h>

#include "sre2_geometry.h"
#include "sre2_internal.h"

namespace sre2 {

template <typename Real>
int max_n() {
    return max_n_of<Real>();
}
template <typename Real>
int fused_max_n() {
    return Tune<Real>::FMAX;
}
template <typename Real>
int pass1_row_bits(int NS) {
    return row_bits_of<Real>(NS);
}
template <typename Real>
int herm_min_n() {
    return Tune<Real>::RBF + 1;
}
template <typename Real>
int64_t pass2_col_tiles(int N, bool herm) {
    const int NS = N - (herm ? 1 : 0);
    const int HT = NS - row_bits_of<Real>(NS);
    const int tb = HT >= 1 && HT <= Prec<Real>::MAXTB ? pass2_tb<Real>(HT) : 0;
    return tb > 0 ? (int64_t)1 << (NS - tb) : 0;
}
template int max_n<float>();
template int max_n<double>();
template int fused_max_n<float>();
template int fused_max_n<double>();
template int pass1_row_bits<float>(int);
template int pass1_row_bits<double>(int);
template int herm_min_n<float>();
template int herm_min_n<double>();
template int64_t pass2_col_tiles<float>(int, bool);
template int64_t pass2_col_tiles<double>(int, bool);

}  // namespace sre2
