// Test-only stand-ins for the kernel launchers of sre2_kernels.hip, so the
// host code of libsre2 (argument checks, workspace sizing, contexts, the
// serving loop's and simulator's setup) can be built with the host address
// and undefined-behaviour sanitizers without compiling the kernels.  Every
// launcher reports that no device is present; the driver only takes paths
// that return before any launch.
#include <hip/hip_runtime.h>

#include "../../paper_2512_24685_amd/csrc/sre2_internal.h"

namespace sre2 {
template <typename Real>
hipError_t launch_shift_kernel(const void*, int, bool, int, int64_t, int64_t, double*,
                               const int*, const Pack&, const Spec*, hipStream_t) {
    return hipErrorNoDevice;
}
template <typename Real>
hipError_t launch_pass1(const void*, int, int, int, int64_t, int, void*, const int*,
                        hipStream_t) {
    return hipErrorNoDevice;
}
template <typename Real>
hipError_t launch_pass2(const void*, int, int, int, int64_t, int, int, double*, const int*,
                        const Spec*, hipStream_t) {
    return hipErrorNoDevice;
}
template hipError_t launch_shift_kernel<float>(const void*, int, bool, int, int64_t, int64_t,
                                               double*, const int*, const Pack&, const Spec*,
                                               hipStream_t);
template hipError_t launch_shift_kernel<double>(const void*, int, bool, int, int64_t, int64_t,
                                                double*, const int*, const Pack&, const Spec*,
                                                hipStream_t);
// the host rule without the plans: row pairs from 2^L
template <typename Real>
int64_t pair_first_shift(int N, int) {
    return (int64_t)1 << pass1_row_bits<Real>(N);
}
template int64_t pair_first_shift<float>(int, int);
template int64_t pair_first_shift<double>(int, int);
template hipError_t launch_pass1<float>(const void*, int, int, int, int64_t, int, void*,
                                        const int*, hipStream_t);
template hipError_t launch_pass1<double>(const void*, int, int, int, int64_t, int, void*,
                                         const int*, hipStream_t);
template hipError_t launch_pass2<float>(const void*, int, int, int, int64_t, int, int, double*,
                                        const int*, const Spec*, hipStream_t);
template hipError_t launch_pass2<double>(const void*, int, int, int, int64_t, int, int, double*,
                                         const int*, const Spec*, hipStream_t);
hipError_t launch_moments(const void*, int, int64_t, int, double*, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_norm_total(const double*, int, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_zero_u64(unsigned long long*, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_split_scale(const double*, int, int*, const Pack&, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_convert(const void*, int, void*, int, int64_t, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_norm(const void*, int, int64_t, int, double*, double*, const Pack&,
                       hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_sum(const double*, int64_t, int, int, double*, double*, const Pack&,
                      hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_group_sum(const double*, int64_t, int, double*, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_final(const double*, int, const double*, const double*, int, int, double*,
                        const Pack&, int, double, hipStream_t) {
    return hipErrorNoDevice;
}
}  // namespace sre2
