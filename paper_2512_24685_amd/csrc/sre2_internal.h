// sre2_internal.h - declarations shared by the kernel and API translation units
// of libsre2 (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace sre2 {

constexpr int kMaxN = 26;
constexpr int kC64 = 0;
constexpr int kC128 = 1;

// Geometry queries.  Two-pass is used for N > fused_max_n; pass 1 transforms
// the low L = pass1_row_bits bits.  The Hermitian-pair forms need
// N >= herm_min_n (fused) and shifts x >= 1 (fused) or x >= 2^L (two-pass);
// other shifts go through the plain kernels.
template <typename Real> int max_n();
template <typename Real> int fused_max_n();
template <typename Real> int pass1_row_bits();
template <typename Real> int herm_min_n();
// Column tiles per shift in pass 2 (upper bound of the column groups P).
template <typename Real> int64_t pass2_col_tiles(int N, bool herm);

// S[i] = S_{x0+i} for shifts [x0, x0 + xc): tiny kernel (plain, N < RB) or
// fused kernel (N <= fused_max_n).  `split` selects the split-FP16 MFMA
// transform (FP32 only, not with herm); it reads the scale exponent *se.
template <typename Real>
hipError_t launch_shift_kernel(const void* psi, int N, bool herm, bool split, int64_t x0,
                               int64_t xc, double* S, const int* se, hipStream_t st);
// Two-pass, one chunk of cs shifts starting at x0: pass 1 writes the
// row-transformed slabs (cs * 2^(N - herm) complex values) to `scratch`;
// pass 2 writes part[s*P + p], the p-th column-group partial of shift x0+s.
template <typename Real>
hipError_t launch_pass1(const void* psi, int N, bool herm, bool split, int64_t x0, int cs,
                        void* scratch, const int* se, hipStream_t st);
template <typename Real>
hipError_t launch_pass2(const void* scratch, int N, bool herm, bool split, int cs, int P,
                        double* part, const int* se, hipStream_t st);
// Scale exponent of the split form from the norm partials.
hipError_t launch_split_scale(const double* npart, int nb, int* se, hipStream_t st);

hipError_t launch_convert(const void* in, int in_dtype, void* out, int out_dtype, int64_t n,
                          hipStream_t st);
hipError_t launch_norm(const void* psi, int dtype, int64_t n, int nblocks, double* part,
                       double* flag, hipStream_t st);
hipError_t launch_sum(const double* v, int64_t nshift, int P, int nblocks, double* part,
                      double* Sx, hipStream_t st);
hipError_t launch_group_sum(const double* part, int64_t ns, int P, double* Sx, hipStream_t st);
hipError_t launch_final(const double* spart, int ns, const double* npart, const double* nflag,
                        int nn, int N, double* out, hipStream_t st);

}  // namespace sre2
