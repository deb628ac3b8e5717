// sre2_kernels.hip - gfx950 kernels for the XOR-FWHT evaluation of the
// second-order stabilizer Renyi entropy (arXiv:2512.24685, Algorithm 1 and
// Eq. final1):
//
//   S_x = sum_z |W_x(z)|^4,  W_x = FWHT_k( conj(psi[k ^ x]) * psi[k] ),
//   S   = sum_x S_x,          M2  = -log2( S / (2^N n^4) ),  n = sum_k |psi[k]|^2.
//
// W_x(z) equals <psi| X^x Z^z |psi> (Eq. Pauli_expect), so every W is a Pauli
// expectation.  Shifts x are independent units of work (main text: the shift
// loop is parallel); each kernel below owns a set of shifts or a slice of one.
//
//  k_tiny      N < RB: one thread per shift, whole transform in registers.
//  k_fused     RB <= N <= TB: a workgroup holds 2^(TB-N) complete shifts in a
//              2^TB tile; rounds of register butterflies with LDS transposes.
//              Workgroups loop over tiles; FP32 one-shift tiles keep psi[k]
//              in registers across them.
//  k_pass1     N > TB: row transform over the low TB bits of k, f_x built on
//              the fly from psi, written to a scratch slab (for shifts
//              x >= 2^TB only half its rows: Hermitian pair, row pairs).
//  k_pass2     N > TB: column transform over the high N-TB bits, |W|^4 and a
//              per-workgroup FP64 partial sum; nothing is written back.  The
//              row-pair form rebuilds the rows pass 1 left out, exactly.
//  k_convert / k_norm_part / k_sum_part / k_final: input staging, FP64 norm,
//              fixed-order FP64 reductions and the logarithm.
//  k_moment_part / k_moment_final: sum |psi|^2, sum |psi|^4 and non-finite
//              count of an input (sre2_moments).
//
// Forms: FP32 or FP64 butterflies; the Hermitian pair (half the transform
// of shifts x >= 1); the split forms, whose H_16 factors run on the matrix
// cores with FP16 or BF16 hi/lo halves (SPLIT = 1, 2).
//
// Accumulation: |W|^2 is formed in the working precision, squared and summed
// in FP64 per element; per-thread sums are combined by fixed-shape trees, so a
// result depends only on (psi, N, form), never on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "sre2_plan.h"
#include "sre2_geometry.h"
#include "sre2_internal.h"

namespace sre2 {

template <typename Real> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

// conj(a) * b.  The imaginary part rounds both products before the
// difference (no fused multiply-add), so that cmul_conj_a(b, a) is exactly
// conj(cmul_conj_a(a, b)): f_x(k ^ x) = conj f_x(k) then holds bit for bit,
// which the row-pair slabs of the two-pass path rely on.  The real part may
// fuse one product: a.x b.x + a.y b.y with either product fused is the same
// for (a, b) and (b, a), as the same expression fuses the same position
// (the GPU tests compare row-pair and full-slab results bit for bit).
template <typename C>
__device__ __forceinline__ C cmul_conj_a(C a, C b) {
    C r;
    r.x = a.x * b.x + a.y * b.y;
    {
#pragma clang fp contract(off)
        r.y = a.x * b.y - a.y * b.x;
    }
    return r;
}

template <typename C>
__device__ __forceinline__ double abs4(C w) {  // |w|^4 with the square in FP64
    const auto m = w.x * w.x + w.y * w.y;
    const double md = (double)m;
    return md * md;
}

// Hermitian-pair form: 16 (Re^4 + Im^4) of one half-space transform value
// equals the sum of |W|^4 over the two Pauli strings it stands for.
template <typename C>
__device__ __forceinline__ double abs4h(C w) {
    const double a = (double)(w.x * w.x), b = (double)(w.y * w.y);
    return a * a + b * b;
}

// General reduction of one w = |W|^2 (Spec kinds): the term of the sum in
// FP64, or (histogram) a count in the block's LDS bins.  lnorm2 = log2(n^2).
template <typename Real>
__device__ __forceinline__ double gen_term(Real w, const Spec& sp, Real lnorm2,
                                           unsigned* __restrict__ lh) {
    if (sp.kind == kRedHist) {
        int b = sp.nbins - 1;
        if (w > Real(0)) {  // NaN-safe: every comparison with NaN selects bin 0
            const Real f = floor(lnorm2 - log2(w) + Real(0.5));
            b = !(f >= Real(0)) ? 0 : (f >= Real(sp.nbins - 1) ? sp.nbins - 1 : (int)f);
        }
        atomicAdd(&lh[b], 1u);
        return 0.0;
    }
    if (!(w > Real(0))) return 0.0;
    if (sp.kind == kRedShannon) return (double)(w * log2(w));
    return (double)exp2((Real)sp.alpha * log2(w));
}

// Terms of one transformed value: |W|^2 in the plain form; in the Hermitian
// pair the real and imaginary parts stand for two Pauli strings with
// |W| = 2 |Re| and 2 |Im|.
template <typename Real, bool HERM, typename C>
__device__ __forceinline__ double gen_terms(C v, const Spec& sp, Real lnorm2,
                                            unsigned* __restrict__ lh) {
    if constexpr (HERM)
        return gen_term<Real>(Real(4) * v.x * v.x, sp, lnorm2, lh) +
               gen_term<Real>(Real(4) * v.y * v.y, sp, lnorm2, lh);
    else
        return gen_term<Real>(v.x * v.x + v.y * v.y, sp, lnorm2, lh);
}

// Block-level histogram bins: cleared at kernel start, added to the global
// counters at the end (GEN kernels with a histogram Spec only).
__device__ __forceinline__ void hist_clear(unsigned* lh, const Spec& sp) {
    if (sp.kind == kRedHist) {
        for (int i = threadIdx.x; i < kMaxBins; i += blockDim.x) lh[i] = 0u;
        __syncthreads();
    }
}
__device__ __forceinline__ void hist_flush(unsigned* lh, const Spec& sp) {
    if (sp.kind == kRedHist) {
        __syncthreads();
        for (int i = threadIdx.x; i < sp.nbins; i += blockDim.x)
            if (lh[i]) atomicAdd(&sp.hist[i], (unsigned long long)lh[i]);
    }
}
template <typename Real>
__device__ __forceinline__ Real hist_lnorm2(const Spec& sp) {
    return sp.kind == kRedHist ? (Real)(2.0 * log2(*sp.nrm)) : Real(0);
}

#ifndef SRE2_SPLIT_P1_TAIL
#define SRE2_SPLIT_P1_TAIL 1  // split-form pass 1 ends in a store-layout round
#endif
// Minimum waves per SIMD asked of the compiler (register budget 512 / waves).
// Split-form pass 1 on 2^12 rows keeps its MFMA results in VGPRs at 3 (with
// fewer, the compiler moves them through AGPRs, which costs it about half its
// speed); LDS limits every TB = 12 kernel to 2.5 waves per SIMD anyway, and
// longer rows to 2.  Split-form pass 2 cannot reach 3 without spilling and is
// left alone.
#ifndef SRE2_P1_WAVES
#define SRE2_P1_WAVES 1
#endif
#ifndef SRE2_P1S_WAVES
#define SRE2_P1S_WAVES 3  // split form
#endif
#ifndef SRE2_P2_WAVES
#define SRE2_P2_WAVES 1
#endif
#ifndef SRE2_P2S_WAVES
#define SRE2_P2S_WAVES 1
#endif
#ifndef SRE2_FUSED_WAVES
#define SRE2_FUSED_WAVES 1
#endif
#ifndef SRE2_FUSEDS_WAVES
#define SRE2_FUSEDS_WAVES 2
#endif
// Half-LDS tiles: two workgroups share a CU.  Two-pass tiles ask for the
// waves per SIMD that takes (half_waves: four for 512-thread FP32 tiles, i.e.
// at most 128 registers, two for 256-thread FP64 tiles); the half-LDS fused
// tile (256 threads of 64 values) needs two waves per SIMD.
#ifndef SRE2_FUSEDH_WAVES
#define SRE2_FUSEDH_WAVES 2
#endif
#ifndef SRE2_F32_FUSEDH_WAVES
#define SRE2_F32_FUSEDH_WAVES SRE2_FUSEDH_WAVES
#endif
#ifndef SRE2_HALF_WGS
#define SRE2_HALF_WGS 2  // workgroups per CU that half-LDS two-pass tiles aim for
#endif
// Waves per SIMD that SRE2_HALF_WGS workgroups of 2^(TB - RB) threads need
// (four SIMDs per CU, 64 lanes per wave): the register budget per wave.
__host__ __device__ constexpr int half_waves(int tb, int rb) {
    const int w = SRE2_HALF_WGS * (1 << (tb - rb)) / 256;
    return w < 1 ? 1 : w;
}
// Slab traffic: streamed through the caches (no reuse until the other pass).
#ifndef SRE2_NT_SLAB
#define SRE2_NT_SLAB 1
#endif
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef double f64x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void slab_store(float2* p, float2 v) {
    if constexpr (SRE2_NT_SLAB) {
        f32x2v w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<f32x2v*>(p));
    } else {
        *p = v;
    }
}
__device__ __forceinline__ void slab_store(double2* p, double2 v) {
    if constexpr (SRE2_NT_SLAB) {
        f64x2v w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<f64x2v*>(p));
    } else {
        *p = v;
    }
}
// Reads through a buffer resource (base, size in bytes): an address is the
// resource base + a per-thread vector offset + a scalar offset, so a gather
// whose per-element part is uniform across the wave (the register element's
// part of an index) keeps that part in a scalar register and runs no
// per-element address arithmetic on the VALU.  Offsets are 32-bit: psi and
// one shift's slab hold at most 2^26 complex128 values (1 GiB).  AUX is the
// cache policy; 2 marks a streaming (non-temporal) read.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    // word 3 = 0x00020000: raw (unformatted) 32-bit dword access on gfx9
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                             0x00020000);
}
template <int AUX>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                         float2& v) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, AUX);
    __builtin_memcpy(&v, &w, sizeof(v));
}
template <int AUX>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff,
                                         double2& v) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, AUX);
    __builtin_memcpy(&v, &w, sizeof(v));
}
// Element vidx + sidx of the resource, vidx per thread, sidx uniform.
template <typename C, int AUX = 0>
__device__ __forceinline__ C load_at(__amdgpu_buffer_rsrc_t rs, uint32_t vidx, uint32_t sidx) {
    C v;
    buf_load<AUX>(rs, vidx * (uint32_t)sizeof(C), sidx * (uint32_t)sizeof(C), v);
    return v;
}

// Insert a zero bit at position `hb` of `v`.
__device__ __forceinline__ uint32_t insert0(uint32_t v, uint32_t hb) {
    return ((v >> hb) << (hb + 1)) | (v & ((1u << hb) - 1u));
}

// Remove bit `b` of `v` (the bits above it move down by one): the inverse
// of insert0 on values with that bit clear.  Like insert0 it maps disjoint
// bit sets to disjoint bit sets, so it adds over them.
__host__ __device__ constexpr uint32_t remove_bit(uint32_t v, int b) {
    return ((v >> (b + 1)) << b) | (v & ((1u << b) - 1u));
}

// Row bit left out of a half slab (Hermitian pair, row pairs), for the row
// part xh = x >> L (nonzero) of a shift x: a set bit of xh, the lowest one
// inside `pref` when there is one, else the top one.  Pass 1 then builds
// only the slab rows with that bit clear.
__device__ __forceinline__ int half_row_bit(uint32_t xh, uint32_t pref) {
    const uint32_t p = xh & pref;
    return p ? __builtin_ctz(p) : 31 - __builtin_clz(xh);
}

// Flip the sign bits of a complex value's parts by the masks mx, my (each
// 0 or the sign bit of a float, applied to the high word of a double).
constexpr uint32_t kSign = 0x80000000u;
__device__ __forceinline__ float2 xor_signs(float2 v, uint32_t mx, uint32_t my) {
    v.x = __uint_as_float(__float_as_uint(v.x) ^ mx);
    v.y = __uint_as_float(__float_as_uint(v.y) ^ my);
    return v;
}
__device__ __forceinline__ double2 xor_signs(double2 v, uint32_t mx, uint32_t my) {
    v.x = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v.x) ^ ((uint64_t)mx << 32));
    v.y = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v.y) ^ ((uint64_t)my << 32));
    return v;
}

// Butterflies over the register bits of `bfly` (a subset of `reg`), one tile
// bit at a time (compile-time recursion keeps every register index constant).
template <int RB, uint32_t REG, uint32_t BFLY, int B = 0, typename C>
__device__ __forceinline__ void butterflies(C (&v)[1 << RB]) {
    if constexpr (B < 32) {
        if constexpr (((BFLY >> B) & 1u) != 0) {
            constexpr int rbit = popc(REG & ((1u << B) - 1u));
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                if ((i >> rbit) & 1) continue;
                const int j = i | (1 << rbit);
                const C a = v[i], c = v[j];
                v[i].x = a.x + c.x;
                v[i].y = a.y + c.y;
                v[j].x = a.x - c.x;
                v[j].y = a.y - c.y;
            }
        }
        butterflies<RB, REG, BFLY, B + 1>(v);
    }
}

// Tile bits of this thread's elements outside the registers: lane-id bit i
// goes to tile bit (LPERM >> 5i) & 31, the wave id to the bits of WAVE.
template <uint32_t LPERM, uint32_t WAVE>
__device__ __forceinline__ uint32_t thread_base() {
    const uint32_t t = threadIdx.x;
    uint32_t b = pdep(t >> 6, WAVE);
#pragma unroll
    for (int i = 0; i < 6; ++i) b |= ((t >> i) & 1u) << ((LPERM >> (5 * i)) & 31u);
    return b;
}

// LDS slot of register element i, r = pdep(i, REG), for a thread whose own
// slot offset (bytes) is pb_bytes:
//  padded buffer: pad(base | r) = pad(base) + pad(r) (disjoint bits), so
//    pad(r) becomes the instruction's constant offset;
//  swizzled buffer: the bits of swz(r) at or above SB are tile bits of REG,
//    where swz(base) is zero, so swz(base) ^ swz(r) = (swz(base) ^ lo) + hi
//    with lo, hi the parts of swz(r) below and above bit SB: one XOR per
//    distinct lo, and hi is the constant offset.
template <int SB, bool PADDED>
__device__ __forceinline__ uint32_t thread_slot(uint32_t base) {
    return PADDED ? pad16<SB>(base) : swz<SB>(base);
}
template <int SB, bool PADDED, typename C>
__device__ __forceinline__ C* lds_slot(C* lds, uint32_t pb_bytes, uint32_t r) {
    char* b = reinterpret_cast<char*>(lds);
    if constexpr (PADDED) {
        return reinterpret_cast<C*>(b + pb_bytes + pad<SB>(r) * (uint32_t)sizeof(C));
    } else {
        const uint32_t e = swz<SB>(r);
        const uint32_t lo = e & ((1u << SB) - 1u), hi = e & ~((1u << SB) - 1u);
        return reinterpret_cast<C*>(b + hi * (uint32_t)sizeof(C) +
                                    (pb_bytes ^ (lo * (uint32_t)sizeof(C))));
    }
}

// Registers v[OFF + i], i < 2^RB, hold the elements base | pdep(i, REG).
template <int SB, bool PADDED, int RB, uint32_t REG, uint32_t LPERM, uint32_t WAVE, int OFF = 0,
          typename C, int NV>
__device__ __forceinline__ void lds_put(C* lds, const C (&v)[NV]) {
    static_assert(OFF + (1 << RB) <= NV, "registers");
    const uint32_t pb = thread_slot<SB, PADDED>(thread_base<LPERM, WAVE>()) * (uint32_t)sizeof(C);
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i)
        *lds_slot<SB, PADDED>(lds, pb, pdep((uint32_t)i, REG)) = v[OFF + i];
}

template <int SB, bool PADDED, int RB, uint32_t REG, uint32_t LPERM, uint32_t WAVE, int OFF = 0,
          typename C, int NV>
__device__ __forceinline__ void lds_get(const C* lds, C (&v)[NV]) {
    static_assert(OFF + (1 << RB) <= NV, "registers");
    const uint32_t pb = thread_slot<SB, PADDED>(thread_base<LPERM, WAVE>()) * (uint32_t)sizeof(C);
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i)
        v[OFF + i] = *lds_slot<SB, PADDED>(const_cast<C*>(lds), pb, pdep((uint32_t)i, REG));
}

// Plan selector (PK encodes the kind so that plans stay constexpr):
//   PK = 1000 + N : whole transform over tile bits [0, N)        (fused)
//   PK = 2000     : row transform over all TB tile bits          (pass 1)
//   PK = 3000 + H : column transform over the top H tile bits    (pass 2)
//   PK + 10000 s  : the same transform in split form s (1: FP16, 2: BF16
//                   halves; one plan for both), with H_16 factors on the
//                   matrix cores (pass 1 ends with a round whose lanes run
//                   over the lowest bits, for the stores)
//   tiles above 64 KiB (half_lds) take half-LDS plans (not the fused split
//   form); the fused kernel's then hold 64 values per thread
template <typename Real, int TB, int RB, int PK>
__host__ __device__ constexpr Plan plan_of() {
    constexpr int SB = Prec<Real>::SB;
    constexpr bool H = half_lds<Real>(TB);
    if (PK >= 10000) {
        constexpr int K = PK % 10000;
        if (K >= 3000)
            return H ? make_split_plan_half(TB, RB, SB, TB - (K - 3000), 0)
                     : make_split_plan(TB, RB, SB, TB - (K - 3000), TB, 0);
        if (K >= 2000)
            return H ? make_split_plan_half(TB, RB, SB, 0, SRE2_SPLIT_P1_TAIL)
                     : make_split_plan(TB, RB, SB, 0, TB, SRE2_SPLIT_P1_TAIL);
        return make_split_plan(TB, RB, SB, 0, K - 1000, 2);
    }
    if (PK >= 3000)
        return H ? make_plan_half(TB, RB, SB, TB - (PK - 3000))
                 : make_plan(TB, RB, SB, TB - (PK - 3000), TB);
    if (PK >= 2000) return H ? make_plan_half(TB, RB, SB, 0) : make_plan(TB, RB, SB, 0, TB);
    return fused_half<Real>(PK - 1000) ? make_plan_half(TB, RB, SB, 0)
                                       : make_plan(TB, RB, SB, 0, PK - 1000);
}

template <int TB, int RB, int PK>
__host__ __device__ constexpr bool plan_has_mf() {
    constexpr Plan P = plan_of<float, TB, RB, PK>();
    bool any = false;
    for (int j = 0; j < P.nrounds; ++j) any = any || P.r[j].mf != 0;
    return any;
}

// ---------------------------------------------------------------------------
// Split MFMA forms.  H_16 = H_2^{(x)4} applied along four tile bits is a
// 16x16 matrix of +-1 (exact in FP16 and BF16).  Each FP32 value v (pre-scaled
// by a power of two so that every |v| <= 2^14, which FP16's range needs) is
// split into hi = h(v) and lo = h(v - hi), h = fp16 (SPLIT 1) or bf16
// (SPLIT 2), both rounded to nearest (v - hi is exact in FP32), and one
// v_mfma_f32_16x16x32_{f16,bf16} computes H_16 (hi + lo) with FP32
// accumulation for a 16 x 16 block: K = 32 holds the hi and lo halves of 16
// rows.  The pair carries 22 significant bits with FP16 and 16 with BF16.
// Operand layout (lane l, i = l % 16, g = l / 16):
//   A[i][8g + j], B[8g + j][i] for j = 0..7,  D[4g + r][i] for r = 0..3.
// K order used here: k = 8g + j  ->  row 4g + (j & 3), part j >> 2 (hi, lo),
// so lane l feeds rows 4g..4g+3 and receives the same rows back.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float f32x2c __attribute__((ext_vector_type(2)));
typedef short op8 __attribute__((ext_vector_type(8)));  // 8 halves, as bits

template <int SPLIT>
struct SplitT;
template <>
struct SplitT<1> {
    typedef _Float16 e8 __attribute__((ext_vector_type(8)));
    typedef _Float16 e2 __attribute__((ext_vector_type(2)));
    __device__ __forceinline__ static floatx4 mfma(op8 a, op8 b) {
        const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(e8, a),
                                                      __builtin_bit_cast(e8, b), zero, 0, 0, 0);
    }
};
template <>
struct SplitT<2> {
    typedef __bf16 e8 __attribute__((ext_vector_type(8)));
    typedef __bf16 e2 __attribute__((ext_vector_type(2)));
    __device__ __forceinline__ static floatx4 mfma(op8 a, op8 b) {
        const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(e8, a),
                                                       __builtin_bit_cast(e8, b), zero, 0, 0, 0);
    }
};

template <int SPLIT>
__device__ __forceinline__ op8 h16_operand() {
    using E8 = typename SplitT<SPLIT>::e8;
    using E = decltype(E8{}[0]);
    const int l = threadIdx.x & 63;
    const int i = l & 15, g = l >> 4;
    E8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 4 * g + (j & 3);
        a[j] = (__builtin_popcount(i & k) & 1) ? (E)-1.0f : (E)1.0f;
    }
    return __builtin_bit_cast(op8, a);
}

// Two FP32 values to FP16 / BF16, rounded to nearest (v_cvt_pk_f16_f32,
// v_cvt_pk_bf16_f32).
template <int SPLIT>
__device__ __forceinline__ typename SplitT<SPLIT>::e2 pk_rne(float a, float b) {
    const f32x2c v = {a, b};
    return __builtin_convertvector(v, typename SplitT<SPLIT>::e2);
}

// hi/lo halves of four values in the K order above.  hi = h(v) rounded to
// nearest; v - hi is exact in FP32 (a multiple of v's FP32 ulp below 2^13 of
// them for FP16, 2^16 for BF16), and lo = h(v - hi), also rounded to nearest,
// so the split carries no systematic bias.
template <int SPLIT>
__device__ __forceinline__ op8 split4(float a, float b, float c, float d) {
    const auto hab = pk_rne<SPLIT>(a, b);
    const auto hcd = pk_rne<SPLIT>(c, d);
    const auto lab = pk_rne<SPLIT>(a - (float)hab[0], b - (float)hab[1]);
    const auto lcd = pk_rne<SPLIT>(c - (float)hcd[0], d - (float)hcd[1]);
    const typename SplitT<SPLIT>::e8 r = {hab[0], hab[1], hcd[0], hcd[1],
                                          lab[0], lab[1], lcd[0], lcd[1]};
    return __builtin_bit_cast(op8, r);
}

// One round's H_16 factor in registers.  The factor's tile bits are the
// register-index bits A, A + 1 (j) and the lane-id bits 4, 5 (g): for every
// setting q of the other register-index bits, lane 16g + c holds rows 4g + j
// of column c, which is the B operand layout, and receives rows 4g + r of the
// product in the same registers.
template <int SPLIT, int RB, int A>
__device__ __forceinline__ void mf_apply(float2 (&v)[1 << RB], const op8 amat) {
#pragma unroll
    for (int q = 0; q < (1 << (RB - 2)); ++q) {
        const int b = (q & ((1 << A) - 1)) | ((q >> A) << (A + 2));
        constexpr int s = 1 << A;
        const op8 br = split4<SPLIT>(v[b].x, v[b + s].x, v[b + 2 * s].x, v[b + 3 * s].x);
        const op8 bi = split4<SPLIT>(v[b].y, v[b + s].y, v[b + 2 * s].y, v[b + 3 * s].y);
        const floatx4 dr = SplitT<SPLIT>::mfma(amat, br);
        const floatx4 di = SplitT<SPLIT>::mfma(amat, bi);
#pragma unroll
        for (int r = 0; r < 4; ++r) v[b + r * s] = make_float2(dr[r], di[r]);
    }
}

// The arithmetic of round J: butterflies on its FP32 bits, then its H_16
// factor (split form).
template <typename Real, int TB, int RB, int PK, int J>
__device__ __forceinline__ void round_math(typename CT<Real>::T (&v)[1 << RB], const op8 amat) {
    constexpr Round rd = plan_of<Real, TB, RB, PK>().r[J];
    butterflies<RB, rd.reg, rd.bfly>(v);
    if constexpr (rd.mf != 0) {
        static_assert(sizeof(Real) == 4, "H_16 factors act on FP32 values");
        mf_apply<PK / 10000, RB, mf_reg_index(rd)>(v, amat);
    }
}

// Rounds J .. nrounds-1 of a plan: LDS transpose, then the round's arithmetic.
template <typename Real, int TB, int RB, int PK, int J>
struct RoundRunner {
    using C = typename CT<Real>::T;
    static constexpr Plan P = plan_of<Real, TB, RB, PK>();
    static constexpr int SB = Prec<Real>::SB;
    static constexpr bool PADDED = lds_padded(P);
    static_assert(TB <= 16, "tile slots are formed for elements below 2^16");
    __device__ __forceinline__ static void run(C* lds, C (&v)[1 << RB], const op8 amat) {
        if constexpr (J < P.nrounds) {
            constexpr Round prev = P.r[J - 1];
            constexpr Round cur = P.r[J];
            if constexpr (P.half) {
                // the top tile bit is the top register-index bit of both
                // layouts: move the registers with that bit 0, then 1,
                // through half the tile's LDS (slots drop the top bit)
                constexpr uint32_t low = (1u << (TB - 1)) - 1u;
                constexpr int HR = 1 << (RB - 1);
                static_assert((prev.reg >> (TB - 1)) & (cur.reg >> (TB - 1)) & 1u, "half plan");
                __syncthreads();  // previous readers of the LDS buffer are done
                lds_put<SB, PADDED, RB - 1, prev.reg & low, prev.lperm, prev.wave, 0>(lds, v);
                __syncthreads();
                lds_get<SB, PADDED, RB - 1, cur.reg & low, cur.lperm, cur.wave, 0>(lds, v);
                __syncthreads();
                lds_put<SB, PADDED, RB - 1, prev.reg & low, prev.lperm, prev.wave, HR>(lds, v);
                __syncthreads();
                lds_get<SB, PADDED, RB - 1, cur.reg & low, cur.lperm, cur.wave, HR>(lds, v);
            } else {
                __syncthreads();  // previous readers of the LDS tile are done
                lds_put<SB, PADDED, RB, prev.reg, prev.lperm, prev.wave>(lds, v);
                __syncthreads();
                lds_get<SB, PADDED, RB, cur.reg, cur.lperm, cur.wave>(lds, v);
            }
            round_math<Real, TB, RB, PK, J>(v, amat);
            RoundRunner<Real, TB, RB, PK, J + 1>::run(lds, v, amat);
        }
    }
};

// Whole transform from round 0's register layout to the last round's.
template <typename Real, int TB, int RB, int PK>
__device__ __forceinline__ void run_transform(typename CT<Real>::T* lds,
                                              typename CT<Real>::T (&v)[1 << RB]) {
    op8 amat = {};
    if constexpr (PK >= 10000) amat = h16_operand<PK / 10000>();
    round_math<Real, TB, RB, PK, 0>(v, amat);
    RoundRunner<Real, TB, RB, PK, 1>::run(lds, v, amat);
}

// Sum over a block of NT threads (NT a multiple of 64): a butterfly of
// cross-lane exchanges inside each wave (XOR partners 32, 16, ..., 1, so every
// lane ends with the same wave sum), then the wave sums, added in wave order
// by thread 0 through LDS.  The order is fixed by NT alone.  The result is
// valid in thread 0; `red` needs NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
    static_assert(NT % 64 == 0, "whole waves");
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    constexpr int NW = NT / 64;
    if constexpr (NW == 1) {
        return v;
    } else {
        __syncthreads();  // earlier readers of red are done
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        double t = 0.0;
        if (threadIdx.x == 0)
            for (int w = 0; w < NW; ++w) t += red[w];
        return t;
    }
}

// Fixed-shape tree over T doubles in LDS; segments of `seg` consecutive entries
// are reduced independently (seg divides T, both powers of two).  Result of
// segment j lands in red[j * seg].
template <int T>
__device__ __forceinline__ void seg_tree(double* red, int seg) {
    for (int s = seg >> 1; s >= 1; s >>= 1) {
        __syncthreads();
        const int i = threadIdx.x;
        if ((i & (2 * s - 1)) < s) red[i] += red[i + s];
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Tiny N (N < RB): one thread per shift.
// ---------------------------------------------------------------------------
template <typename Real, int N, bool GEN>
__global__ __launch_bounds__(64) void k_tiny(const typename CT<Real>::T* __restrict__ psi,
                                             int64_t x_begin, int64_t x_count,
                                             double* __restrict__ S_out,
                                             const Pack pk, const Spec sp) {
    using C = typename CT<Real>::T;
    constexpr int D = 1 << N;
    __shared__ unsigned lh[GEN ? kMaxBins : 1];
    if constexpr (GEN) {
        hist_clear(lh, sp);
        const Real lnorm2 = hist_lnorm2<Real>(sp);
        const int64_t idx = (int64_t)blockIdx.x * 64 + threadIdx.x;
        if (idx < x_count) {
            const uint32_t x = (uint32_t)(x_begin + idx);
            C v[D];
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] = cmul_conj_a(psi[k ^ x], psi[k]);
            butterflies<N, (1u << N) - 1u, (1u << N) - 1u>(v);
            double s = 0.0;
#pragma unroll
            for (int z = 0; z < D; ++z) s += gen_terms<Real, false>(v[z], sp, lnorm2, lh);
            S_out[idx] = s;
        }
        hist_flush(lh, sp);
        return;
    }
    if (pk.count) {
        psi = (const C*)pk.psi[blockIdx.y];
        S_out = pk_sx(pk.ws[blockIdx.y], N) + x_begin;
    }
    const int64_t idx = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (idx >= x_count) return;
    const uint32_t x = (uint32_t)(x_begin + idx);
    C v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = cmul_conj_a(psi[k ^ x], psi[k]);
    butterflies<N, (1u << N) - 1u, (1u << N) - 1u>(v);
    double s = 0.0;
#pragma unroll
    for (int z = 0; z < D; ++z) s += abs4(v[z]);
    S_out[idx] = s;
}

// Fused tiles that hold one shift and keep psi[k] in registers (see k_fused).
template <typename Real>
__host__ __device__ constexpr bool fused_keeps_psi(int NT, bool herm) {
    return sizeof(Real) == 4 && !herm && fused_tb<Real>(NT) == NT;
}

// ---------------------------------------------------------------------------
// Fused: whole transforms of NT bits in a 2^TB tile of SPT = 2^(TB-NT) shifts.
//  HERM = false: NT = N, the tile element (slot j, k) is f_x(k), x = x0 + j.
//  HERM = true : NT = N - 1 (Hermitian pair, x >= 1): with hb the top set bit
//                of x, element (j, k') is f_x(k) for k = k' with a 0 inserted
//                at bit hb, i.e. only the half-space k_hb = 0.  Because
//                f_x(k ^ x) = conj f_x(k), W_x(z) over the full space is twice
//                Re or twice i Im of this half transform, so
//                S_x = 16 sum_z' (Re^4 + Im^4).
// ---------------------------------------------------------------------------
template <typename Real, int NT, int TB, int RB, bool HERM, int SPLIT, bool GEN>
__global__ __launch_bounds__(1 << (TB - RB))
__attribute__((amdgpu_waves_per_eu(SPLIT ? SRE2_FUSEDS_WAVES
                                   : (fused_half<Real>(NT)
                                          ? (sizeof(Real) == 4 ? SRE2_F32_FUSEDH_WAVES
                                                               : SRE2_FUSEDH_WAVES)
                                          : SRE2_FUSED_WAVES))))
void k_fused(const typename CT<Real>::T* __restrict__ psi, int64_t x_begin, int64_t x_count,
             double* __restrict__ S_out, const int* __restrict__ scale_exp,
             const Pack pk, const Spec sp) {
    using C = typename CT<Real>::T;
    constexpr int T = 1 << (TB - RB);
    constexpr int PK = 1000 + NT + 10000 * SPLIT;
    constexpr Plan P = plan_of<Real, TB, RB, PK>();
    constexpr Round r0 = P.r[0];
    constexpr Round rl = P.r[P.nrounds - 1];
    constexpr int SPT = 1 << (TB - NT);
    constexpr uint32_t KMASK = (1u << NT) - 1u;
    static_assert((rl.reg & ~KMASK) == 0, "last round: one shift per thread");
    // the buffer also holds the reduction's 2^(TB - RB) doubles
    constexpr int NRED = (1 << (TB - RB)) * (int)sizeof(double) / (int)sizeof(C);
    constexpr int NL = lds_values(P);
    __shared__ C lds[NL > NRED ? NL : NRED];
    __shared__ unsigned lh[GEN ? kMaxBins : 1];
    double* red = reinterpret_cast<double*>(lds);
    if (pk.count) {
        psi = (const C*)pk.psi[blockIdx.y];
        S_out = pk_sx(pk.ws[blockIdx.y], pk.N) + x_begin;
        scale_exp = pk_se(pk.ws[blockIdx.y], pk.N);
    }
    Real lnorm2 = Real(0);
    if constexpr (GEN) {
        hist_clear(lh, sp);
        lnorm2 = hist_lnorm2<Real>(sp);
    }

    const int se = SPLIT ? *scale_exp : 0;
    const Real sc = SPLIT ? ldexpf(1.0f, se) : Real(1);
    const double unscale = SPLIT ? ldexp(1.0, -4 * se) : 1.0;
    const int64_t ntiles = (x_count + SPT - 1) / SPT;
    // one shift per tile: k = e = base | r (disjoint bits) does not depend on
    // the tile, so FP32 tiles read psi[k] once per workgroup and keep it in
    // registers over the tiles the workgroup takes (FP64 tiles have no
    // registers left for it)
    constexpr bool ONE = SPT == 1 && !HERM;
    constexpr bool KEEP = fused_keeps_psi<Real>(NT, HERM);
    const auto rs = buf_rsrc(psi, (uint32_t)sizeof(C) << (NT + (HERM ? 1 : 0)));
    C psik[KEEP ? (1 << RB) : 1];
    if constexpr (KEEP) {
        const uint32_t base = thread_base<r0.lperm, r0.wave>();
#pragma unroll
        for (int i = 0; i < (1 << RB); ++i) psik[i] = load_at<C>(rs, base, pdep((uint32_t)i, r0.reg));
    }
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t x0 = x_begin + tile * SPT;  // first shift of the tile
        C v[1 << RB];
        if constexpr (ONE) {
            // as in pass 1, k ^ x = (base ^ (x outside REG)) + (r ^ (x inside
            // REG)), so the per-element address parts are uniform
            const uint32_t x = (uint32_t)x0;
            const uint32_t base = thread_base<r0.lperm, r0.wave>();
            const uint32_t vb = base ^ (x & ~r0.reg), xr = x & r0.reg;
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                const uint32_t r = pdep((uint32_t)i, r0.reg);
                v[i] = cmul_conj_a(load_at<C>(rs, vb, r ^ xr),
                                   KEEP ? psik[KEEP ? i : 0] : load_at<C>(rs, base, r));
                if constexpr (SPLIT) {
                    v[i].x *= sc;
                    v[i].y *= sc;
                }
            }
        } else if constexpr (SPT == 1 && HERM) {
            // one shift per tile, k = insert0(e, hb), hb the top set bit of x:
            // insert0 maps disjoint bits to disjoint bits, so k = kb + kr with
            // kb = insert0(base, hb) and kr = insert0(r, hb), and k ^ x splits
            // the same way over R = insert0(REG, hb): the per-element parts
            // stay uniform
            const uint32_t x = (uint32_t)x0;
            const uint32_t hb = 31u - __clz(x);
            const uint32_t R = insert0(r0.reg, hb);
            const uint32_t kb = insert0(thread_base<r0.lperm, r0.wave>(), hb);
            const uint32_t vb = kb ^ (x & ~R), xr = x & R;
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                const uint32_t kr = insert0(pdep((uint32_t)i, r0.reg), hb);
                v[i] = cmul_conj_a(load_at<C>(rs, vb, kr ^ xr), load_at<C>(rs, kb, kr));
            }
        } else {
            const uint32_t base = thread_base<r0.lperm, r0.wave>();
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                const uint32_t e = base | pdep((uint32_t)i, r0.reg);
                const int64_t j = e >> NT;  // shift slot in the tile
                if (tile * SPT + j < x_count) {
                    const uint32_t x = (uint32_t)(x0 + j);
                    uint32_t k = e & KMASK;
                    if constexpr (HERM) k = insert0(k, 31u - __clz(x));
                    v[i] = cmul_conj_a(psi[k ^ x], psi[k]);
                    if constexpr (SPLIT) {
                        v[i].x *= sc;
                        v[i].y *= sc;
                    }
                } else {
                    v[i].x = 0;
                    v[i].y = 0;
                }
            }
        }
        run_transform<Real, TB, RB, PK>(lds, v);
        double s = 0.0;
        if constexpr (GEN) {
            // this thread's values belong to one shift slot (the last round's
            // registers lie inside the transform bits); empty slots of the
            // last tile hold zeros that must not enter the histogram
            const int64_t slot = thread_base<rl.lperm, rl.wave>() >> NT;
            if (tile * SPT + slot < x_count) {
#pragma unroll
                for (int i = 0; i < (1 << RB); ++i)
                    s += gen_terms<Real, HERM>(v[i], sp, lnorm2, lh);
            }
        } else {
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) s += HERM ? abs4h(v[i]) : abs4(v[i]);
            if constexpr (HERM) s *= 16.0;
            if constexpr (SPLIT) s *= unscale;
        }
        // thread order index: tile bits outside the last round's registers,
        // compressed; its top TB-NT bits are the shift slot.
        const uint32_t q = pext(thread_base<rl.lperm, rl.wave>(), ((1u << TB) - 1u) & ~rl.reg);
        __syncthreads();
        red[q] = s;
        seg_tree<T>(red, T / SPT);
        if (threadIdx.x < SPT) {
            const int64_t j = threadIdx.x;
            if (tile * SPT + j < x_count) S_out[tile * SPT + j] = red[j * (T / SPT)];
        }
    }
    if constexpr (GEN) hist_flush(lh, sp);
}

// ---------------------------------------------------------------------------
// Two-pass, pass 1: row transform over k_lo (TB = L bits) of f_x for a chunk
// of shifts; the slab of one shift holds 2^NS values.  NS = N, or with HERM
// a half slab of NS = N - 1: only the rows whose bit j = half_row_bit(x >> L,
// pref) is clear (x >= 2^L, so that j is a row bit), for the Hermitian pair
// (pref = 0: j is the top set bit of x) and for the row pairs of the plain
// and split forms (pref = the register row bits of the pass-2 plan, L that
// of the full slab).  Grid
// (cs, rows): block (s, r) takes shift slot s of slab row r; blocks are
// dispatched with x fastest, so neighbouring blocks read the same psi rows.
// ---------------------------------------------------------------------------
template <typename Real, int TB, int RB, bool HERM, int SPLIT>
__global__ __launch_bounds__(1 << (TB - RB))
__attribute__((amdgpu_waves_per_eu(half_lds<Real>(TB) ? half_waves(TB, RB)
                                   : (SPLIT && TB <= 12 ? SRE2_P1S_WAVES : SRE2_P1_WAVES))))
void k_pass1(const typename CT<Real>::T* __restrict__ psi, int NS, int64_t x0, int cs,
             typename CT<Real>::T* __restrict__ scratch, const int* __restrict__ scale_exp,
             uint32_t pref) {
    using C = typename CT<Real>::T;
    constexpr int PK = 2000 + 10000 * SPLIT;
    constexpr Plan P = plan_of<Real, TB, RB, PK>();
    constexpr Round r0 = P.r[0];
    constexpr Round rl = P.r[P.nrounds - 1];
    __shared__ C lds[lds_values(P)];

    (void)cs;
    const uint32_t srow = blockIdx.y;  // row within the slab
    const int64_t s = blockIdx.x;      // shift slot in the chunk
    const uint64_t x = (uint64_t)(x0 + s);
    uint32_t row = srow;
    if constexpr (HERM) row = insert0(srow, half_row_bit((uint32_t)(x >> TB), pref));
    const uint32_t rowbase = row << TB;
    const uint32_t prow = rowbase ^ (uint32_t)(x & ~(uint64_t)((1u << TB) - 1u));  // partner row
    const uint32_t xlo = (uint32_t)(x & ((1u << TB) - 1u));
    const auto rs = buf_rsrc(psi, (uint32_t)sizeof(C) << (NS + (HERM ? 1 : 0)));
    C v[1 << RB];
    {
        // element e = base | r (disjoint bits): psi[rowbase + e] takes the
        // thread part base as vector and rowbase + r as scalar offset, and
        // e ^ xlo = (base ^ (xlo outside REG)) + (r ^ (xlo inside REG)), so
        // the per-element parts are uniform and the per-thread parts are
        // formed once
        const uint32_t base = thread_base<r0.lperm, r0.wave>();
        const uint32_t vb = base ^ (xlo & ~r0.reg), xr = xlo & r0.reg;
#pragma unroll
        for (int i = 0; i < (1 << RB); ++i) {
            const uint32_t r = pdep((uint32_t)i, r0.reg);
            v[i] = cmul_conj_a(load_at<C>(rs, vb, prow + (r ^ xr)), load_at<C>(rs, base, rowbase + r));
        }
        if constexpr (SPLIT) {
            const Real sc = ldexpf(1.0f, *scale_exp);
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                v[i].x *= sc;
                v[i].y *= sc;
            }
        }
    }
    run_transform<Real, TB, RB, PK>(lds, v);
    C* __restrict__ out = scratch + ((uint64_t)s << NS) + ((uint64_t)srow << TB);
    const uint32_t base = thread_base<rl.lperm, rl.wave>();
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) slab_store((out + pdep((uint32_t)i, rl.reg)) + base, v[i]);
}

// ---------------------------------------------------------------------------
// Row pairs (plain and split forms, shifts x >= 2^L).  With xh = x >> L and
// xl = x mod 2^L, f_x(k ^ x) = conj f_x(k) makes slab row r ^ xh of pass 1
// the row r transformed with its input XOR-permuted by xl and conjugated, so
//   row(r ^ xh)[z] = (-1)^popcount(z & xl) conj(row(r)[z]).
// That holds bit for bit: the products are exactly conjugate (cmul_conj_a),
// and a butterfly network fed an XOR-permuted input computes the same sums
// and differences, some of them negated (u + v = v + u, v - u = -(u - v)).
// So pass 1 stores only the rows with bit j = half_row_bit(xh, register row
// bits of the pass-2 tile) clear, and pass 2 rebuilds a row with bit j set
// from its partner: conjugate and sign are sign-bit flips, and the column
// transform then runs on exactly the values of the full slab.  (The split
// forms' H_16 products on the matrix cores sum in an order the permutation
// does not preserve: there the rebuilt rows are the exact images of the
// computed stored rows, equal to the full slab's up to rounding.)  A launch
// covers shifts of one row part xh (its chunk stays inside one block of 2^L
// shifts), so j is one value per launch and the kernel runs a tile loop
// specialised on it: j is taken among the register row bits when xh has one,
// so that which elements are rebuilt is fixed per register index
// (pair_load_reg); otherwise xh has only thread row bits and whole threads
// hold rebuilt rows (pair_load_thr; not in the plain half-LDS tiles, whose
// row pairs start where xh has a register row bit, pair_first_shift, and
// which form the thread's address parts per tile to stay within their
// registers).  Stored values are read twice (as
// themselves and as a partner) inside one tile, the second time from the
// caches.
// ---------------------------------------------------------------------------
template <typename C, int RB, uint32_t REG, int CB, int J>
__device__ __forceinline__ void pair_load_reg(C (&v)[1 << RB], __amdgpu_buffer_rsrc_t rs, int L,
                                              uint32_t vb0, uint32_t vb1, uint32_t xh,
                                              uint32_t xl, uint32_t cto, uint32_t mT) {
    constexpr uint32_t CMASK = (1u << CB) - 1u;
    const uint32_t xhr = xh & (REG >> CB);  // xh on the register row bits
    // conjugate: the imaginary part flips; the empty asm keeps the compiler
    // from splitting y ^ mTy back into two XORs per element
    uint32_t mTy = mT ^ kSign;
    asm volatile("" : "+v"(mTy));
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        const uint32_t r = pdep((uint32_t)i, REG);
        const uint32_t R = r >> CB, cr = r & CMASK;
        if ((R >> J) & 1u) {  // a rebuilt row: partner row ^ xh, stored
            const uint32_t sr = cr ? ((__builtin_popcount(cr & xl) & 1u) ? kSign : 0u) : 0u;
            const C t = load_at<C>(rs, vb1, (remove_bit(R ^ xhr, J) << L) + cto + cr);
            v[i] = xor_signs(t, mT ^ sr, mTy ^ sr);
        } else {
            v[i] = load_at<C>(rs, vb0, (remove_bit(R, J) << L) + cto + cr);
        }
    }
}

// Calls f(std::integral_constant<int, j>) for the register row bit j.
template <uint32_t RROW, int JJ = 0, typename F>
__device__ __forceinline__ void with_reg_row_bit(int j, F&& f) {
    if constexpr (JJ < 32) {
        if constexpr ((RROW >> JJ) & 1u) {
            if (j == JJ) {
                f(std::integral_constant<int, JJ>{});
                return;
            }
        }
        with_reg_row_bit<RROW, JJ + 1>(j, f);
    }
}

// j a thread row bit (xh has no register row bit): a thread's rows are all
// stored (fm = 0) or all rebuilt (fm = ~0); vb already points at the stored rows.
template <typename C, int RB, uint32_t REG, int CB>
__device__ __forceinline__ void pair_load_thr(int j, C (&v)[1 << RB], __amdgpu_buffer_rsrc_t rs,
                                              int L, uint32_t vb, uint32_t fm, uint32_t xl,
                                              uint32_t cto, uint32_t mT) {
    constexpr uint32_t CMASK = (1u << CB) - 1u;
#pragma unroll
    for (int i = 0; i < (1 << RB); ++i) {
        const uint32_t r = pdep((uint32_t)i, REG);
        const uint32_t R = r >> CB, cr = r & CMASK;
        const uint32_t m = fm & (mT ^ ((__builtin_popcount(cr & xl) & 1u) ? kSign : 0u));
        const C t = load_at<C>(rs, vb, (remove_bit(R, j) << L) + cto + cr);
        v[i] = xor_signs(t, m, m ^ (fm & kSign));
    }
}

// ---------------------------------------------------------------------------
// Two-pass, pass 2: column transform over the HT slab-row bits of one shift's
// slab (2^NS values = 2^HT rows of 2^L; with PAIR the slab holds the 2^(HT-1)
// stored rows of the row pairs, and x0 is the chunk's first shift).  A tile
// is 2^HT rows x 2^(TB-HT) columns.  Block b -> shift slot b / P, column
// group b % P; the group loops over its column tiles and writes one FP64
// partial of S_x.
// ---------------------------------------------------------------------------
template <typename Real, int HT, int TB, int RB, bool HERM, int SPLIT, bool GEN, bool PAIR>
__global__ __launch_bounds__(1 << (TB - RB))
__attribute__((amdgpu_waves_per_eu(half_lds<Real>(TB) ? half_waves(TB, RB)
                                   : (SPLIT ? SRE2_P2S_WAVES : SRE2_P2_WAVES))))
void k_pass2(const typename CT<Real>::T* __restrict__ scratch, int NS, int P,
             double* __restrict__ part, const int* __restrict__ scale_exp, const Spec sp,
             int64_t x0) {
    static_assert(!PAIR || (!HERM && !GEN), "row pairs: plain and split M2 forms only");
    using C = typename CT<Real>::T;
    constexpr int T = 1 << (TB - RB);
    constexpr int PK = 3000 + HT + 10000 * SPLIT;
    constexpr Plan PL = plan_of<Real, TB, RB, PK>();
    constexpr Round r0 = PL.r[0];
    constexpr int CB = TB - HT;  // column bits per tile
    constexpr uint32_t CMASK = (1u << CB) - 1u;
    // streaming loads only when a tile reads whole 128-byte lines of a row
    constexpr bool NT = SRE2_NT_SLAB && ((int)sizeof(C) << CB) >= 128;
    __shared__ C lds[lds_values(PL)];
    __shared__ double red[T];
    __shared__ unsigned lh[GEN ? kMaxBins : 1];
    Real lnorm2 = Real(0);
    if constexpr (GEN) {
        hist_clear(lh, sp);
        lnorm2 = hist_lnorm2<Real>(sp);
    }

    const int64_t b = blockIdx.x;
    const int64_t s = b / P;
    const int g = (int)(b % P);
    const int L = NS - HT;  // row bits of pass 1
    const int ntile = 1 << (L - CB);  // column tiles per shift
    const int per = ntile / P;
    const int SH = PAIR ? NS - 1 : NS;  // slab bits of one shift
    const auto rs = buf_rsrc(scratch + ((uint64_t)s << SH), (uint32_t)sizeof(C) << SH);
    // tile element e -> slab offset (e >> CB) * 2^L + (e & CMASK), which adds
    // over disjoint bits: the thread's part once, the register element's part
    // (and the column tile's) as a uniform offset
    const uint32_t base = thread_base<r0.lperm, r0.wave>();
    const uint32_t vb = ((base >> CB) << L) + (base & CMASK);
    // row pairs: the shift's row and column parts, the left-out row bit j,
    // the thread's stored-row (vb0) and partner-row (vb1) address parts and
    // the sign (-1)^popcount(z & xl) of its column bits
    constexpr uint32_t RROW = r0.reg >> CB;
    // the thread-row variant is left out of the plain half-LDS tiles (their
    // registers are full); their row pairs start where x >> L has a register
    // row bit, which for their plans (the top row bits in registers) is
    // x >= 2^(L + lowest register row bit), pair_first_shift
    constexpr bool THR = !half_lds<Real>(TB) || SPLIT;
    static_assert(!PAIR || THR || RROW + (RROW & (0u - RROW)) == (1u << HT),
                  "half-LDS row pairs need the top row bits in registers");
    uint32_t xh = 0, xl = 0, vb0 = 0, vb1 = 0, sT = 0, fm = 0;
    int j = 0;
    if constexpr (PAIR) {
        const uint64_t x = (uint64_t)(x0 + s);
        xh = (uint32_t)(x >> L);
        xl = (uint32_t)x & ((1u << L) - 1u);
        j = half_row_bit(xh, RROW);
        const uint32_t rowT = base >> CB, colT = base & CMASK;
        if constexpr (THR) {
            vb0 = (remove_bit(rowT, j) << L) + colT;
            vb1 = (remove_bit(rowT ^ (xh & ~RROW), j) << L) + colT;
            sT = __builtin_popcount(colT & xl) & 1u;
            fm = 0u - ((rowT >> j) & 1u);
        }
    }
    double acc = 0.0;
    // column transform of one tile and its terms, tiles in ascending order
    auto consume = [&](C (&v)[1 << RB]) {
        run_transform<Real, TB, RB, PK>(lds, v);
        if constexpr (GEN) {
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) acc += gen_terms<Real, HERM>(v[i], sp, lnorm2, lh);
        } else {
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) acc += HERM ? abs4h(v[i]) : abs4(v[i]);
        }
    };
    const int c0 = g * per, c1 = (g + 1) * per;
    // Plain, Hermitian and row-pair tiles that fit the LDS whole load the
    // next tile while transforming this one (two register sets; these
    // kernels are held to two waves per SIMD by their LDS tiles, which leaves
    // the registers; the full-slab split kernel and split tiles above 2^12
    // values have none to spare);
    // barriers wait on LDS only, so the loads stay in flight across the
    // transform.  load_tile(v, ct) fills v with column tile ct.
    constexpr bool PREFETCH = !half_lds<Real>(TB) && (!SPLIT || (PAIR && TB <= 12)) && !GEN;
    auto tiles = [&](auto&& load_tile) {
        if constexpr (PREFETCH) {
            C va[1 << RB], vn[1 << RB];
            load_tile(va, c0);
            for (int ct = c0; ct < c1; ct += 2) {
                if (ct + 1 < c1) load_tile(vn, ct + 1);
                consume(va);
                if (ct + 1 < c1) {
                    if (ct + 2 < c1) load_tile(va, ct + 2);
                    consume(vn);
                }
            }
        } else {
            for (int ct = c0; ct < c1; ++ct) {
                C v[1 << RB];
                load_tile(v, ct);
                consume(v);
            }
        }
    };
    if constexpr (PAIR) {
        if ((RROW >> j) & 1u) {
            with_reg_row_bit<RROW>(j, [&](auto J) {
                tiles([&](C (&v)[1 << RB], int ct) {
                    constexpr int JJ = decltype(J)::value;
                    const uint32_t cto = (uint32_t)ct << CB;
                    uint32_t v0 = vb0, v1 = vb1, st = sT;
                    if constexpr (!THR) {
                        // large tiles: the thread's parts formed per tile from
                        // its id (the empty asm statements keep them there),
                        // so that no register holds them across the
                        // transform; remove_bit is linear over XOR, so the
                        // partner part is the stored part XOR a uniform term
                        uint32_t tb = thread_base<r0.lperm, r0.wave>();
                        uint32_t xt = remove_bit(xh & ~RROW, JJ) << L;
                        asm volatile("" : "+v"(tb), "+s"(xt));
                        v0 = (remove_bit(tb >> CB, JJ) << L) + (tb & CMASK);
                        v1 = v0 ^ xt;
                        st = __builtin_popcount(tb & CMASK & xl) & 1u;
                    }
                    const uint32_t mT = ((st ^ __builtin_popcount(cto & xl)) & 1u) ? kSign : 0u;
                    pair_load_reg<C, RB, r0.reg, CB, JJ>(v, rs, L, v0, v1, xh, xl, cto, mT);
                });
            });
        } else if constexpr (THR) {
            const uint32_t vbt = fm ? vb1 : vb0;
            tiles([&](C (&v)[1 << RB], int ct) {
                const uint32_t cto = (uint32_t)ct << CB;
                const uint32_t mT = ((sT ^ __builtin_popcount(cto & xl)) & 1u) ? kSign : 0u;
                pair_load_thr<C, RB, r0.reg, CB>(j, v, rs, L, vbt, fm, xl, cto, mT);
            });
        } else {
            // half-LDS tiles take row pairs only for shifts whose row part
            // has a register row bit (pair_first_shift); a launch outside
            // that range reports NaN rather than a wrong sum
            acc = __builtin_nan("");
        }
    } else {
        tiles([&](C (&v)[1 << RB], int ct) {
            const uint32_t cto = (uint32_t)ct << CB;
#pragma unroll
            for (int i = 0; i < (1 << RB); ++i) {
                const uint32_t r = pdep((uint32_t)i, r0.reg);
                v[i] = load_at<C, NT ? 2 : 0>(rs, vb, cto + ((r >> CB) << L) + (r & CMASK));
            }
        });
    }
    if constexpr (!GEN) {
        if constexpr (HERM) acc *= 16.0;
        if constexpr (SPLIT) acc *= ldexp(1.0, -4 * *scale_exp);
    }
    const double tot = block_sum<T>(acc, red);
    if (threadIdx.x == 0) part[b] = tot;
    if constexpr (GEN) hist_flush(lh, sp);
}

// ---------------------------------------------------------------------------
// Staging and reductions.
// ---------------------------------------------------------------------------
template <typename Src, typename Dst>
__global__ void k_convert(const Src* __restrict__ in, Dst* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        Dst d;
        d.x = in[i].x;
        d.y = in[i].y;
        out[i] = d;
    }
}

constexpr int kRedThreads = 256;
static_assert(kRedThreads <= kMaxRed, "reduction blocks");

// part[b] = sum of |psi|^2 over block b's fixed range; flag[b] = non-finite seen.
template <typename C>
__global__ __launch_bounds__(kRedThreads) void k_norm_part(const C* __restrict__ psi, int64_t n,
                                                           int64_t per_block,
                                                           double* __restrict__ part,
                                                           double* __restrict__ flag,
                                                           const Pack pk) {
    __shared__ double red[kRedThreads];
    if (pk.count) {
        psi = (const C*)pk.psi[blockIdx.y];
        part = pk_npart(pk.ws[blockIdx.y], pk.N);
        flag = pk_nflag(pk.ws[blockIdx.y], pk.N);
    }
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = lo + per_block < n ? lo + per_block : n;
    double s = 0.0;
    int bad = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRedThreads) {
        const double re = (double)psi[i].x, im = (double)psi[i].y;
        if (!isfinite(re) || !isfinite(im)) bad = 1;
        s += re * re + im * im;
    }
    const double tot = block_sum<kRedThreads>(s, red);
    const double nbad = block_sum<kRedThreads>(bad ? 1.0 : 0.0, red);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = tot;
        flag[blockIdx.x] = nbad;
    }
}

// Moments of the input as given, per block over the same fixed ranges as
// k_norm_part: m[b] = sum |psi|^2, m[K + b] = sum |psi|^4 (the inverse
// participation ratio's numerator), m[2K + b] = count of non-finite
// amplitudes, K = kMaxRed; all in FP64.
template <typename C>
__global__ __launch_bounds__(kRedThreads) void k_moment_part(const C* __restrict__ psi, int64_t n,
                                                             int64_t per_block,
                                                             double* __restrict__ m) {
    __shared__ double red[kRedThreads];
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = lo + per_block < n ? lo + per_block : n;
    double s2 = 0.0, s4 = 0.0, bad = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRedThreads) {
        const double re = (double)psi[i].x, im = (double)psi[i].y;
        if (!isfinite(re) || !isfinite(im)) bad += 1.0;
        const double q = re * re + im * im;
        s2 += q;
        s4 += q * q;
    }
    const double t2 = block_sum<kRedThreads>(s2, red);
    const double t4 = block_sum<kRedThreads>(s4, red);
    const double tb = block_sum<kRedThreads>(bad, red);
    if (threadIdx.x == 0) {
        m[blockIdx.x] = t2;
        m[kMaxRed + blockIdx.x] = t4;
        m[2 * kMaxRed + blockIdx.x] = tb;
    }
}

// out[j] = sum over b < nb of m[j K + b] in b order, j = 0, 1, 2.
__global__ void k_moment_final(const double* __restrict__ m, int nb, double* __restrict__ out) {
    const int j = threadIdx.x;
    if (j >= 3) return;
    double a = 0.0;
    for (int b = 0; b < nb; ++b) a += m[j * kMaxRed + b];
    out[j] = a;
}

// part[b] = sum of v over block b's fixed range (optionally with stride-P
// grouping: entry x*P+p belongs to shift x; Sx, when non-null, receives
// sum_p v[x*P+p] in p order).
__global__ __launch_bounds__(kRedThreads) void k_sum_part(const double* __restrict__ v,
                                                          int64_t nshift, int P,
                                                          int64_t per_block,
                                                          double* __restrict__ part,
                                                          double* __restrict__ Sx,
                                                          const Pack pk) {
    __shared__ double red[kRedThreads];
    if (pk.count) {
        v = pk_sx(pk.ws[blockIdx.y], pk.N);
        part = pk_spart(pk.ws[blockIdx.y], pk.N);
        Sx = nullptr;
    }
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = lo + per_block < nshift ? lo + per_block : nshift;
    double s = 0.0;
    for (int64_t x = lo + threadIdx.x; x < hi; x += kRedThreads) {
        double sx = 0.0;
        for (int p = 0; p < P; ++p) sx += v[x * P + p];
        if (Sx) Sx[x] = sx;
        s += sx;
    }
    const double tot = block_sum<kRedThreads>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Sx[s] = sum_p part[s*P + p] in p order (one thread per shift).
__global__ __launch_bounds__(256) void k_group_sum(const double* __restrict__ part, int64_t ns,
                                                   int P, double* __restrict__ Sx) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= ns) return;
    double a = 0.0;
    for (int p = 0; p < P; ++p) a += part[s * P + p];
    Sx[s] = a;
}

// out[0] = M2, out[1] = S, out[2] = n, out[3] = status (0 ok, 1 bad input).
__global__ __launch_bounds__(kRedThreads) void k_final(const double* __restrict__ spart, int ns,
                                                       const double* __restrict__ npart,
                                                       const double* __restrict__ nflag, int nn,
                                                       int N, double* __restrict__ out,
                                                       const Pack pk, int kind, double alpha) {
    __shared__ double red[kRedThreads];
    if (pk.count) {
        spart = pk_spart(pk.ws[blockIdx.y], pk.N);
        npart = pk_npart(pk.ws[blockIdx.y], pk.N);
        nflag = pk_nflag(pk.ws[blockIdx.y], pk.N);
        out = pk.out[blockIdx.y];
    }
    double a = 0.0, b = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < ns; i += kRedThreads) a += spart[i];
    for (int i = threadIdx.x; i < nn; i += kRedThreads) {
        b += npart[i];
        c += nflag[i];
    }
    const double S = block_sum<kRedThreads>(a, red);
    const double n = block_sum<kRedThreads>(b, red);
    const double bad = block_sum<kRedThreads>(c, red);
    if (threadIdx.x == 0) {
        const bool ok = bad == 0.0 && n > 0.0 && isfinite(n) && isfinite(S);
        const double n2 = n * n;
        double m = NAN;
        if (kind == kRedQuartic)
            m = -log2(S / (ldexp(1.0, N) * n2 * n2));
        else if (kind == kRedPow)  // Eq. 1: log2(S / (2^N n^(2 alpha))) / (1 - alpha)
            m = (log2(S) - (double)N - alpha * log2(n2)) / (1.0 - alpha);
        else if (kind == kRedShannon)  // alpha -> 1, with sum_P w = 2^N n^2
            m = log2(n2) - S / (ldexp(1.0, N) * n2);
        out[0] = ok ? m : NAN;
        out[1] = S;
        out[2] = n;
        out[3] = ok ? 0.0 : 1.0;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from sre2_api.hip).
// ---------------------------------------------------------------------------
namespace {

// Workgroups of `threads` threads of `kernel` the current device holds at
// once (CUs x occupancy); 32768 if the runtime cannot say.
int64_t resident_workgroups(const void* kernel, int threads) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
        cus < 1 || per < 1)
        return 32768;
    return (int64_t)cus * per;
}

template <typename Real, int N, bool GEN>
hipError_t launch_tiny_n(const void* psi, int64_t x0, int64_t xc, double* S,
                         const Pack& pk, const Spec& sp, hipStream_t st) {
    using C = typename CT<Real>::T;
    const int64_t blocks = (xc + 63) / 64;
    hipLaunchKernelGGL((k_tiny<Real, N, GEN>), dim3((unsigned)blocks, (unsigned)(pk.count ? pk.count : 1)), dim3(64), 0, st,
                       (const C*)psi, x0, xc, S, pk, sp);
    return hipGetLastError();
}

template <typename Real, int NT, bool HERM, int SPLIT, bool GEN>
hipError_t launch_fused_nt(const void* psi, int64_t x0, int64_t xc, double* S, const int* se,
                           const Pack& pk, const Spec& sp, hipStream_t st) {
    using C = typename CT<Real>::T;
    constexpr int TB = fused_tb<Real>(NT), RB = fused_rb<Real>(NT, SPLIT != 0);
    constexpr int SPT = 1 << (TB - NT);
    const int64_t ntiles = (xc + SPT - 1) / SPT;
    // Tiles that keep psi[k] in registers amortise its reads over the tiles a
    // workgroup takes: their grid is twice the workgroups the GPU holds at
    // once (queried once per kernel; measured at N = 14, 0.58 -> 0.44 ms),
    // the others take one tile per workgroup up to 65536 workgroups.
    int64_t cap = 65536;
    if constexpr (fused_keeps_psi<Real>(NT, HERM)) {
        static const int64_t resident = resident_workgroups(
            reinterpret_cast<const void*>(&k_fused<Real, NT, TB, RB, HERM, SPLIT, GEN>), 1 << (TB - RB));
        cap = 2 * resident;
    }
    const int64_t grid = ntiles < cap ? ntiles : cap;
    hipLaunchKernelGGL((k_fused<Real, NT, TB, RB, HERM, SPLIT, GEN>), dim3((unsigned)grid, (unsigned)(pk.count ? pk.count : 1)),
                       dim3(1 << (TB - RB)), 0, st, (const C*)psi, x0, xc, S, se, pk, sp);
    return hipGetLastError();
}

template <typename Real, int HT, bool HERM, int SPLIT, bool GEN, bool PAIR>
hipError_t launch_pass2_ht(const void* scratch, int NS, int cs, int P, double* part, const int* se,
                           const Spec& sp, int64_t x0, hipStream_t st) {
    using C = typename CT<Real>::T;
    constexpr int TB = pass2_tb<Real>(HT), RB = Tune<Real>::RB2;
    hipLaunchKernelGGL((k_pass2<Real, HT, TB, RB, HERM, SPLIT, GEN, PAIR>),
                       dim3((unsigned)((int64_t)cs * P)), dim3(1 << (TB - RB)), 0, st,
                       (const C*)scratch, NS, P, part, se, sp, x0);
    return hipGetLastError();
}

// Register row bits of the first round of the pass-2 tile of HT rows (split
// form s: its matrix-core plan): the preferred left-out row bits of the row
// pairs, so that pass 1 leaves out the rows pass 2 rebuilds.
template <typename Real, int HT, int SPLIT>
constexpr uint32_t pass2_reg_rows() {
    constexpr int TB = pass2_tb<Real>(HT), RB = Tune<Real>::RB2;
    return plan_of<Real, TB, RB, 3000 + HT + 10000 * SPLIT>().r[0].reg >> (TB - HT);
}
template <typename Real, int... Hs>
uint32_t pair_pref_of(int HT, int split, std::integer_sequence<int, Hs...>) {
    uint32_t m = 0;
    ((HT == Hs + 1 ? (m = split == 0 ? pass2_reg_rows<Real, Hs + 1, 0>()
                        : split == 1 ? pass2_reg_rows<Real, Hs + 1, 1>()
                                     : pass2_reg_rows<Real, Hs + 1, 2>(),
                      0)
                   : 0),
     ...);
    return m;
}

template <typename Real, bool GEN, int... Ns>
hipError_t dispatch_tiny(int N, const void* psi, int64_t x0, int64_t xc, double* S,
                         const Pack& pk, const Spec& sp, hipStream_t st,
                         std::integer_sequence<int, Ns...>) {
    hipError_t e = hipErrorInvalidValue;
    ((N == Ns + 1 ? (e = launch_tiny_n<Real, Ns + 1, GEN>(psi, x0, xc, S, pk, sp, st), 0) : 0),
     ...);
    return e;
}

template <typename Real, bool HERM, int SPLIT, bool GEN, int... Ns>
hipError_t dispatch_fused(int NT, const void* psi, int64_t x0, int64_t xc, double* S,
                          const int* se, const Pack& pk, const Spec& sp, hipStream_t st,
                          std::integer_sequence<int, Ns...>) {
    constexpr int RB = Tune<Real>::RBF;
    hipError_t e = hipErrorInvalidValue;
    ((NT == Ns + RB
          ? (e = launch_fused_nt<Real, Ns + RB, HERM, SPLIT, GEN>(psi, x0, xc, S, se, pk, sp, st),
             0)
          : 0),
     ...);
    return e;
}

template <typename Real, bool HERM, int SPLIT, bool GEN, bool PAIR = false, int... Hs>
hipError_t dispatch_pass2(int HT, const void* scratch, int NS, int cs, int P, double* part,
                          const int* se, const Spec& sp, int64_t x0, hipStream_t st,
                          std::integer_sequence<int, Hs...>) {
    hipError_t e = hipErrorInvalidValue;
    ((HT == Hs + 1
          ? (e = launch_pass2_ht<Real, Hs + 1, HERM, SPLIT, GEN, PAIR>(scratch, NS, cs, P, part,
                                                                       se, sp, x0, st),
             0)
          : 0),
     ...);
    return e;
}


}  // namespace

template <typename Real, bool GEN>
hipError_t shift_kernel_gen(const void* psi, int N, bool herm, int split, int64_t x0,
                            int64_t xc, double* S, const int* se, const Pack& pk, const Spec& sp,
                            hipStream_t st) {
    constexpr int RB = Tune<Real>::RBF, FMAX = Tune<Real>::FMAX;
    if (herm) {
        if (x0 < 1 || N - 1 < RB) return hipErrorInvalidValue;
        return dispatch_fused<Real, true, 0, GEN>(N - 1, psi, x0, xc, S, se, pk, sp, st,
                                                      std::make_integer_sequence<int, FMAX - RB>{});
    }
    if (N < RB)
        return dispatch_tiny<Real, GEN>(N, psi, x0, xc, S, pk, sp, st,
                                        std::make_integer_sequence<int, RB - 1>{});
    if constexpr (sizeof(Real) == 4 && !GEN) {
        if (split == 1)
            return dispatch_fused<Real, false, 1, false>(
                N, psi, x0, xc, S, se, pk, sp, st, std::make_integer_sequence<int, FMAX - RB + 1>{});
        if (split == 2)
            return dispatch_fused<Real, false, 2, false>(
                N, psi, x0, xc, S, se, pk, sp, st, std::make_integer_sequence<int, FMAX - RB + 1>{});
    }
    return dispatch_fused<Real, false, 0, GEN>(N, psi, x0, xc, S, se, pk, sp, st,
                                                   std::make_integer_sequence<int, FMAX - RB + 1>{});
}

template <typename Real>
hipError_t launch_shift_kernel(const void* psi, int N, bool herm, int split, int64_t x0,
                               int64_t xc, double* S, const int* se, const Pack& pk,
                               const Spec* sp, hipStream_t st) {
    constexpr int FMAX = Tune<Real>::FMAX;
    if (N > FMAX || split < 0 || split > 2 || (split && (herm || sizeof(Real) != 4)) ||
        pk.count > kMaxPack)
        return hipErrorInvalidValue;
    if (sp) {
        if (split || pk.count || sp->kind < kRedPow || sp->kind > kRedHist ||
            (sp->kind == kRedHist && (!sp->hist || !sp->nrm || sp->nbins < 2 ||
                                      sp->nbins > kMaxBins)))
            return hipErrorInvalidValue;
        return shift_kernel_gen<Real, true>(psi, N, herm, split, x0, xc, S, se, pk, *sp, st);
    }
    return shift_kernel_gen<Real, false>(psi, N, herm, split, x0, xc, S, se, pk, Spec{}, st);
}

template <typename Real, int... Hs>
int64_t pair_first_shift_of(int N, int split, std::integer_sequence<int, Hs...> hs) {
    const int L = row_bits_of<Real>(N), HT = N - L;
    int64_t first = (int64_t)1 << L;
    if (split == 0 && half_lds<Real>(pass2_tb<Real>(HT))) {
        const uint32_t rrow = pair_pref_of<Real>(HT, split, hs);
        first = (int64_t)1 << (L + __builtin_ctz(rrow));
    }
    return first;
}

// First shift of the row-pair range of an N-qubit evaluation (split form
// `split`): 2^L, or for the plain half-LDS pass-2 tiles 2^(L + r) with r the
// lowest register row bit of the pass-2 plan, so that x >> L has one.
template <typename Real>
int64_t pair_first_shift(int N, int split) {
    if (N <= Tune<Real>::FMAX || N > max_n_of<Real>()) return (int64_t)1 << N;
    constexpr int HMAX = pass2_max_rows<Real>();
    return pair_first_shift_of<Real>(N, split, std::make_integer_sequence<int, HMAX>{});
}
template int64_t pair_first_shift<float>(int, int);
template int64_t pair_first_shift<double>(int, int);

template <typename Real, int TB>
hipError_t launch_pass1_tb(const void* psi, int NS, bool half, int split, int64_t x0, int cs,
                           void* scratch, const int* se, uint32_t pref, hipStream_t st) {
    using C = typename CT<Real>::T;
    constexpr int RB = pass1_rb<Real>(TB, false), RBS = pass1_rb<Real>(TB, true);
    const int64_t rows = (int64_t)1 << (NS - TB);
    if (cs < 1 || rows > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)cs, (unsigned)rows), block(1 << (TB - RB)), blocks(1 << (TB - RBS));
    if (split) {
        if constexpr (sizeof(Real) == 4) {
            if (split == 1 && half)
                hipLaunchKernelGGL((k_pass1<Real, TB, RBS, true, 1>), grid, blocks, 0, st,
                                   (const C*)psi, NS, x0, cs, (C*)scratch, se, pref);
            else if (split == 1)
                hipLaunchKernelGGL((k_pass1<Real, TB, RBS, false, 1>), grid, blocks, 0, st,
                                   (const C*)psi, NS, x0, cs, (C*)scratch, se, pref);
            else if (half)
                hipLaunchKernelGGL((k_pass1<Real, TB, RBS, true, 2>), grid, blocks, 0, st,
                                   (const C*)psi, NS, x0, cs, (C*)scratch, se, pref);
            else
                hipLaunchKernelGGL((k_pass1<Real, TB, RBS, false, 2>), grid, blocks, 0, st,
                                   (const C*)psi, NS, x0, cs, (C*)scratch, se, pref);
        }
    } else if (half)
        hipLaunchKernelGGL((k_pass1<Real, TB, RB, true, 0>), grid, block, 0, st, (const C*)psi,
                           NS, x0, cs, (C*)scratch, se, pref);
    else
        hipLaunchKernelGGL((k_pass1<Real, TB, RB, false, 0>), grid, block, 0, st,
                           (const C*)psi, NS, x0, cs, (C*)scratch, se, pref);
    return hipGetLastError();
}

template <typename Real, int... Ls>
hipError_t dispatch_pass1(int L, const void* psi, int NS, bool half, int split, int64_t x0,
                          int cs, void* scratch, const int* se, uint32_t pref, hipStream_t st,
                          std::integer_sequence<int, Ls...>) {
    hipError_t e = hipErrorInvalidValue;
    ((L == Tune<Real>::ROW + Ls
          ? (e = launch_pass1_tb<Real, Tune<Real>::ROW + Ls>(psi, NS, half, split, x0, cs,
                                                             scratch, se, pref, st),
             0)
          : 0),
     ...);
    return e;
}

// Slab geometry of a two-pass slab kind: slab bits NS of one shift and
// pass-1 row bits L (the row pairs keep the rows and columns of the full
// slab and store half its rows).
template <typename Real>
void slab_geometry(int N, int slab, int* NS, int* L) {
    *NS = N - (slab == kSlabFull ? 0 : 1);
    *L = row_bits_of<Real>(slab == kSlabHerm ? N - 1 : N);
}

template <typename Real>
hipError_t launch_pass1(const void* psi, int N, int slab, int split, int64_t x0, int cs,
                        void* scratch, const int* se, hipStream_t st) {
    if (N <= Tune<Real>::FMAX || N > max_n_of<Real>()) return hipErrorInvalidValue;
    if (slab < kSlabFull || slab > kSlabPairs || split < 0 || split > 2 ||
        (split && (slab == kSlabHerm || sizeof(Real) != 4)))
        return hipErrorInvalidValue;
    int NS, L;
    slab_geometry<Real>(N, slab, &NS, &L);
    if (slab != kSlabFull && x0 < ((int64_t)1 << L)) return hipErrorInvalidValue;
    if (slab == kSlabPairs && x0 < pair_first_shift<Real>(N, split)) return hipErrorInvalidValue;
    constexpr int HMAX = pass2_max_rows<Real>();
    const uint32_t pref =
        slab == kSlabPairs
            ? pair_pref_of<Real>(N - L, split, std::make_integer_sequence<int, HMAX>{})
            : 0u;
    return dispatch_pass1<Real>(
        L, psi, NS, slab != kSlabFull, split, x0, cs, scratch, se, pref, st,
        std::make_integer_sequence<int, Prec<Real>::MAXTB - Tune<Real>::ROW + 1>{});
}

template <typename Real>
hipError_t launch_pass2(const void* scratch, int N, int slab, int split, int64_t x0, int cs,
                        int P, double* part, const int* se, const Spec* sp, hipStream_t st) {
    if (N <= Tune<Real>::FMAX || N > max_n_of<Real>()) return hipErrorInvalidValue;
    if (slab < kSlabFull || slab > kSlabPairs || split < 0 || split > 2 ||
        (split && (slab == kSlabHerm || sizeof(Real) != 4)) || (sp && slab == kSlabPairs))
        return hipErrorInvalidValue;
    int NS, L;
    slab_geometry<Real>(N, slab, &NS, &L);
    if (slab == kSlabPairs && x0 < pair_first_shift<Real>(N, split)) return hipErrorInvalidValue;
    const bool herm = slab == kSlabHerm;
    if (slab == kSlabPairs) NS = N;  // the kernel takes the full slab's bits
    const int HT = NS - L;
    constexpr int HMAX = pass2_max_rows<Real>();
    constexpr auto hs = std::make_integer_sequence<int, HMAX>{};
    if (sp) {
        if (split || sp->kind < kRedPow || sp->kind > kRedHist ||
            (sp->kind == kRedHist && (!sp->hist || !sp->nrm || sp->nbins < 2 ||
                                      sp->nbins > kMaxBins)))
            return hipErrorInvalidValue;
        if (herm)
            return dispatch_pass2<Real, true, 0, true>(HT, scratch, NS, cs, P, part, se, *sp, x0,
                                                       st, hs);
        return dispatch_pass2<Real, false, 0, true>(HT, scratch, NS, cs, P, part, se, *sp, x0,
                                                    st, hs);
    }
    const Spec none{};
    if (herm)
        return dispatch_pass2<Real, true, 0, false>(HT, scratch, NS, cs, P, part, se, none, x0,
                                                    st, hs);
    if (slab == kSlabPairs) {
        if constexpr (sizeof(Real) == 4) {
            if (split == 1)
                return dispatch_pass2<Real, false, 1, false, true>(HT, scratch, NS, cs, P, part,
                                                                   se, none, x0, st, hs);
            if (split == 2)
                return dispatch_pass2<Real, false, 2, false, true>(HT, scratch, NS, cs, P, part,
                                                                   se, none, x0, st, hs);
        }
        return dispatch_pass2<Real, false, 0, false, true>(HT, scratch, NS, cs, P, part, se, none,
                                                           x0, st, hs);
    }
    if constexpr (sizeof(Real) == 4) {
        if (split == 1)
            return dispatch_pass2<Real, false, 1, false>(HT, scratch, NS, cs, P, part, se, none,
                                                         x0, st, hs);
        if (split == 2)
            return dispatch_pass2<Real, false, 2, false>(HT, scratch, NS, cs, P, part, se, none,
                                                         x0, st, hs);
    }
    return dispatch_pass2<Real, false, 0, false>(HT, scratch, NS, cs, P, part, se, none, x0, st,
                                                 hs);
}

template hipError_t launch_shift_kernel<float>(const void*, int, bool, int, int64_t, int64_t,
                                               double*, const int*, const Pack&, const Spec*,
                                               hipStream_t);
template hipError_t launch_shift_kernel<double>(const void*, int, bool, int, int64_t, int64_t,
                                                double*, const int*, const Pack&, const Spec*,
                                                hipStream_t);
template hipError_t launch_pass1<float>(const void*, int, int, int, int64_t, int, void*,
                                        const int*, hipStream_t);
template hipError_t launch_pass1<double>(const void*, int, int, int, int64_t, int, void*,
                                         const int*, hipStream_t);
template hipError_t launch_pass2<float>(const void*, int, int, int, int64_t, int, int, double*,
                                        const int*, const Spec*, hipStream_t);
template hipError_t launch_pass2<double>(const void*, int, int, int, int64_t, int, int, double*,
                                         const int*, const Spec*, hipStream_t);

// s = 14 - ceil(log2 n) from the norm partials (0 when n is not positive and
// finite): with every |value| of a transform bounded by n, the scaled values
// of the split form stay below 2^14, inside FP16's range.
__global__ void k_split_scale(const double* __restrict__ npart, int nb, int* __restrict__ se,
                              const Pack pk) {
    if (threadIdx.x != 0) return;
    if (pk.count) {
        npart = pk_npart(pk.ws[blockIdx.y], pk.N);
        se = pk_se(pk.ws[blockIdx.y], pk.N);
    }
    double n = 0.0;
    for (int i = 0; i < nb; ++i) n += npart[i];
    int s = 0;
    if (n > 0.0 && isfinite(n)) {
        s = 14 - (int)ceil(log2(n));
        s = s < -100 ? -100 : (s > 100 ? 100 : s);
    }
    *se = s;
}

hipError_t launch_split_scale(const double* npart, int nb, int* se, const Pack& pk, hipStream_t st) {
    hipLaunchKernelGGL(k_split_scale, dim3(1, (unsigned)(pk.count ? pk.count : 1)), dim3(64), 0, st, npart, nb, se,
                       pk);
    return hipGetLastError();
}

hipError_t launch_convert(const void* in, int in_dtype, void* out, int out_dtype, int64_t n,
                          hipStream_t st) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (in_dtype == kC128 && out_dtype == kC64)
        hipLaunchKernelGGL((k_convert<double2, float2>), dim3(blocks), dim3(256), 0, st,
                           (const double2*)in, (float2*)out, n);
    else if (in_dtype == kC64 && out_dtype == kC128)
        hipLaunchKernelGGL((k_convert<float2, double2>), dim3(blocks), dim3(256), 0, st,
                           (const float2*)in, (double2*)out, n);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_norm(const void* psi, int dtype, int64_t n, int nblocks, double* part,
                       double* flag, const Pack& pk, hipStream_t st) {
    const int64_t per = (n + nblocks - 1) / nblocks;
    const dim3 grid(nblocks, pk.count ? pk.count : 1);
    if (dtype == kC64)
        hipLaunchKernelGGL((k_norm_part<float2>), grid, dim3(kRedThreads), 0, st,
                           (const float2*)psi, n, per, part, flag, pk);
    else
        hipLaunchKernelGGL((k_norm_part<double2>), grid, dim3(kRedThreads), 0, st,
                           (const double2*)psi, n, per, part, flag, pk);
    return hipGetLastError();
}

hipError_t launch_moments(const void* psi, int dtype, int64_t n, int nblocks, double* m,
                          double* out, hipStream_t st) {
    if (nblocks < 1 || nblocks > kMaxRed) return hipErrorInvalidValue;
    const int64_t per = (n + nblocks - 1) / nblocks;
    if (dtype == kC64)
        hipLaunchKernelGGL((k_moment_part<float2>), dim3(nblocks), dim3(kRedThreads), 0, st,
                           (const float2*)psi, n, per, m);
    else
        hipLaunchKernelGGL((k_moment_part<double2>), dim3(nblocks), dim3(kRedThreads), 0, st,
                           (const double2*)psi, n, per, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_moment_final, dim3(1), dim3(64), 0, st, m, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_sum(const double* v, int64_t nshift, int P, int nblocks, double* part,
                      double* Sx, const Pack& pk, hipStream_t st) {
    const int64_t per = (nshift + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_sum_part, dim3(nblocks, pk.count ? pk.count : 1), dim3(kRedThreads), 0, st, v, nshift, P,
                       per, part, Sx, pk);
    return hipGetLastError();
}

hipError_t launch_group_sum(const double* part, int64_t ns, int P, double* Sx, hipStream_t st) {
    hipLaunchKernelGGL(k_group_sum, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, part, ns,
                       P, Sx);
    return hipGetLastError();
}

hipError_t launch_final(const double* spart, int ns, const double* npart, const double* nflag,
                        int nn, int N, double* out, const Pack& pk, int kind, double alpha,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_final, dim3(1, pk.count ? pk.count : 1), dim3(kRedThreads), 0, st, spart, ns, npart, nflag,
                       nn, N, out, pk, kind, alpha);
    return hipGetLastError();
}

__global__ void k_norm_total(const double* __restrict__ npart, int nb, double* __restrict__ nrm) {
    if (threadIdx.x != 0) return;
    double n = 0.0;
    for (int i = 0; i < nb; ++i) n += npart[i];
    *nrm = n;
}

hipError_t launch_norm_total(const double* npart, int nb, double* nrm, hipStream_t st) {
    hipLaunchKernelGGL(k_norm_total, dim3(1), dim3(64), 0, st, npart, nb, nrm);
    return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0ull;
}

hipError_t launch_zero_u64(unsigned long long* p, int count, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3((count + 63) / 64), dim3(64), 0, st, p, count);
    return hipGetLastError();
}

}  // namespace sre2
