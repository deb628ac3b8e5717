// sre2_internal.h - declarations shared by the kernel and API translation units
// of libsre2 (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <utility>

namespace sre2 {

constexpr int kMaxN = 26;
// Kernels read psi and one shift's slab through buffer resources with 32-bit
// byte offsets: 2^kMaxN complex128 values must stay below 4 GiB.
static_assert((16ull << kMaxN) < (1ull << 32), "psi and a shift's slab need 32-bit offsets");

constexpr int kMaxRed = 1024;  // upper bound of reduction blocks per state
constexpr int kMaxPack = 64;   // states per packed launch

// States of one packed launch: several states of the same N in one grid, the
// grid's y index selecting the state.  Passed to the kernels by value.  Each
// state owns a workspace block ws of pack_ws_doubles(N) doubles laid out as
// S_x (2^N) | norm partials | non-finite flags | S partials (kMaxRed each) |
// split scale exponent (one int in the last double).
struct Pack {
    int count = 0;  // 0: an ordinary single-state launch
    int N = 0;
    const void* psi[kMaxPack] = {};
    double* ws[kMaxPack] = {};
    double* out[kMaxPack] = {};
};

__host__ __device__ inline int64_t pack_ws_doubles(int N) {
    return ((int64_t)1 << N) + 3 * kMaxRed + 1;
}
__host__ __device__ inline double* pk_sx(double* ws, int) { return ws; }
__host__ __device__ inline double* pk_npart(double* ws, int N) { return ws + ((int64_t)1 << N); }
__host__ __device__ inline double* pk_nflag(double* ws, int N) {
    return ws + ((int64_t)1 << N) + kMaxRed;
}
__host__ __device__ inline double* pk_spart(double* ws, int N) {
    return ws + ((int64_t)1 << N) + 2 * kMaxRed;
}
__host__ __device__ inline int* pk_se(double* ws, int N) {
    return reinterpret_cast<int*>(ws + ((int64_t)1 << N) + 3 * kMaxRed);
}
constexpr int kC64 = 0;
constexpr int kC128 = 1;

// Reduction of the transformed values (step a5) other than the default sum of
// |W|^4: w = |W_x(z)|^2 of every Pauli string feeds
//   kRedPow      sum w^alpha          (Renyi index alpha of Eq. 1)
//   kRedShannon  sum w log2 w         (the alpha -> 1 limit)
//   kRedHist     hist[b] += 1, b = round(-log2(w / n^2)) clamped to
//                [0, nbins - 1], w = 0 in the last bin (Pauli spectrum)
// Passed to the kernels by value; a null Spec* selects the default path.
constexpr int kRedQuartic = 0;
constexpr int kRedPow = 1;
constexpr int kRedShannon = 2;
constexpr int kRedHist = 3;
constexpr int kMaxBins = 64;
struct Spec {
    int kind = kRedQuartic;
    int nbins = 0;
    double alpha = 2.0;
    const double* nrm = nullptr;         // device: n = sum |psi|^2 (histogram)
    unsigned long long* hist = nullptr;  // device: nbins counters (histogram)
};

// Geometry queries.  Two-pass is used for N > fused_max_n; pass 1 transforms
// the low L = pass1_row_bits(NS) bits of a slab of NS bits (NS = N, or N - 1
// in the Hermitian-pair forms).  The Hermitian-pair forms need
// N >= herm_min_n (fused) and shifts x >= 1 (fused) or x >= 2^L (two-pass);
// other shifts go through the plain kernels.
template <typename Real> int max_n();
template <typename Real> int fused_max_n();
template <typename Real> int pass1_row_bits(int NS);
template <typename Real> int herm_min_n();
// Column tiles per shift in pass 2 (upper bound of the column groups P).
template <typename Real> int64_t pass2_col_tiles(int N, bool herm);

// S[i] = S_{x0+i} for shifts [x0, x0 + xc): tiny kernel (plain, N < RB) or
// fused kernel (N <= fused_max_n).  `split` selects the split MFMA transform
// (0 none, 1 FP16 halves, 2 BF16 halves; FP32 only, not with herm); it reads
// the scale exponent *se.
// With pk.count > 0 the launch covers pk.count states of the same N (grid
// y = state); psi / S / se then come from the pack (S = S_x of state y + x0).
// sp != nullptr selects the general reduction (not with split or packs).
template <typename Real>
hipError_t launch_shift_kernel(const void* psi, int N, bool herm, int split, int64_t x0,
                               int64_t xc, double* S, const int* se, const Pack& pk,
                               const Spec* sp, hipStream_t st);
// Two-pass slab kinds: the full slab of 2^N values per shift; the Hermitian
// pair's half slab (2^(N-1) values, rows of pass1_row_bits(N - 1) bits); the
// row pairs of the plain and split M2 forms (half the rows of the full slab,
// rows of pass1_row_bits(N) bits; pass 2 rebuilds the other half from them
// by sign flips: in the plain FP32 / FP64 forms S_x is then bit for bit that
// of the full slab, in the split forms it differs by rounding only).  The
// half slabs need x >= 2^L.
constexpr int kSlabFull = 0;
constexpr int kSlabHerm = 1;
constexpr int kSlabPairs = 2;
// Two-pass, one chunk of cs shifts starting at x0: pass 1 writes the
// row-transformed slabs (cs * 2^N or cs * 2^(N-1) complex values) to
// `scratch`; pass 2 writes part[s*P + p], the p-th column-group partial of
// shift x0+s.
// First shift of the row-pair range (shifts below it take the full slab):
// 2^L, or 2^(L + r) when the plain pass-2 tile is a half-LDS tile (r: the
// lowest register row bit of its plan); 2^N when N is fused.
template <typename Real>
int64_t pair_first_shift(int N, int split);
template <typename Real>
hipError_t launch_pass1(const void* psi, int N, int slab, int split, int64_t x0, int cs,
                        void* scratch, const int* se, hipStream_t st);
template <typename Real>
hipError_t launch_pass2(const void* scratch, int N, int slab, int split, int64_t x0, int cs,
                        int P, double* part, const int* se, const Spec* sp, hipStream_t st);
// out[0..2] = (sum |psi|^2, sum |psi|^4, non-finite count) of the input as
// given, in FP64; m holds 3 kMaxRed doubles of block partials.
hipError_t launch_moments(const void* psi, int dtype, int64_t n, int nblocks, double* m,
                          double* out, hipStream_t st);
// *nrm = sum of the norm partials (for the histogram's normalisation).
hipError_t launch_norm_total(const double* npart, int nb, double* nrm, hipStream_t st);
// p[0 .. count) = 0 (a kernel, so that callers may capture it in a graph).
hipError_t launch_zero_u64(unsigned long long* p, int count, hipStream_t st);
// Scale exponent of the split form from the norm partials.
hipError_t launch_split_scale(const double* npart, int nb, int* se, const Pack& pk, hipStream_t st);

hipError_t launch_convert(const void* in, int in_dtype, void* out, int out_dtype, int64_t n,
                          hipStream_t st);
// The reduction launchers also accept a packed launch (pk.count > 0).
hipError_t launch_norm(const void* psi, int dtype, int64_t n, int nblocks, double* part,
                       double* flag, const Pack& pk, hipStream_t st);
hipError_t launch_sum(const double* v, int64_t nshift, int P, int nblocks, double* part,
                      double* Sx, const Pack& pk, hipStream_t st);
hipError_t launch_group_sum(const double* part, int64_t ns, int P, double* Sx, hipStream_t st);
// out = {M, S, n, status}: M2 for kind kRedQuartic, M_alpha for kRedPow,
// M_1 for kRedShannon, NaN for kRedHist.
hipError_t launch_final(const double* spart, int ns, const double* npart, const double* nflag,
                        int nn, int N, double* out, const Pack& pk, int kind, double alpha,
                        hipStream_t st);

}  // namespace sre2
