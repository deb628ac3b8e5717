// sre2_sim.hip - complex128 state-vector simulator for the quench-dynamics
// workloads (C ABI in include/sre2.h, sre2_sim_*), and the pipeline that
// streams its snapshots into the serving loop.
//
// The simulator owns one device state psi (2^N complex128) and a stream of
// its own.  Operations, all as HIP kernels on that stream:
//   * random product state  prod_i (cos(t_i/2)|0> + e^{i p_i} sin(t_i/2)|1>)
//     (the initial state of the Hamiltonian-quench example);
//   * two-qubit gates       4x4 unitaries on qubit pairs, index
//     j = bit(q0) + 2 bit(q1) (the brickwork random-circuit example);
//   * TFIM step             psi <- exp(-i H dt) psi for
//     H = -J sum_{i=0}^{N-2} Z_i Z_{i+1} - hx sum_i X_i - hz sum_i Z_i (open
//     chain), by a Chebyshev expansion of the propagator: with a >= ||H||,
//     exp(-i H dt) = sum_k (2 - [k = 0]) (-i)^k J_k(a dt) T_k(H / a), the T_k
//     from the three-term recurrence T_{k+1} = 2 (H/a) T_k - T_{k-1}; the
//     series is cut where |J_k(a dt)| < 1e-17 beyond k > a dt.
// The pipeline evolves step by step and, after every step, copies the state
// into one of a ring of snapshot buffers and submits it to a server as a
// device input; a ring buffer is reused only once its request is done, so the
// evolution of step t + 1 overlaps the evaluation of the earlier snapshots.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

#include "../../include/sre2.h"
#include "sre2_internal.h"

using namespace sre2;

namespace {

constexpr int kSimMaxN = 26;
constexpr int kRing = 4;  // snapshot buffers of the pipeline

struct ProductArgs {
    double c0[kSimMaxN];   // cos(theta_i / 2)
    double c1r[kSimMaxN];  // Re e^{i phi_i} sin(theta_i / 2)
    double c1i[kSimMaxN];  // Im
};

struct Gate {
    double re[16], im[16];  // row-major U[i][j]
};

__global__ void k_product(double2* __restrict__ psi, int N, const ProductArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ((int64_t)1 << N)) return;
    double re = 1.0, im = 0.0;
    for (int i = 0; i < N; ++i) {
        if ((k >> i) & 1) {
            const double r = re * a.c1r[i] - im * a.c1i[i];
            im = re * a.c1i[i] + im * a.c1r[i];
            re = r;
        } else {
            re *= a.c0[i];
            im *= a.c0[i];
        }
    }
    psi[k] = make_double2(re, im);
}

// One thread per group of four amplitudes that differ in bits q0, q1.
__global__ void k_gate2(double2* __restrict__ psi, int N, int q0, int q1, const Gate g) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= ((int64_t)1 << (N - 2))) return;
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    // insert zero bits at lo, then hi
    uint64_t b = (uint64_t)m;
    b = ((b >> lo) << (lo + 1)) | (b & ((1ull << lo) - 1));
    b = ((b >> hi) << (hi + 1)) | (b & ((1ull << hi) - 1));
    uint64_t idx[4];
    double2 a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        idx[j] = b | ((uint64_t)(j & 1) << q0) | ((uint64_t)(j >> 1) << q1);
        a[j] = psi[idx[j]];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            re += g.re[4 * i + j] * a[j].x - g.im[4 * i + j] * a[j].y;
            im += g.re[4 * i + j] * a[j].y + g.im[4 * i + j] * a[j].x;
        }
        psi[idx[i]] = make_double2(re, im);
    }
}

// acc = c * v
__global__ void k_scale_into(const double2* __restrict__ v, double2* __restrict__ acc, int64_t n,
                             double cr, double ci) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double2 x = v[k];
    acc[k] = make_double2(cr * x.x - ci * x.y, cr * x.y + ci * x.x);
}

// One Chebyshev term: h = (H / a) cur; next = h (first) or 2 h - prev,
// written over prev; acc += c * next.  H is applied as its diagonal
// (Ising and longitudinal-field energies of basis state k, Z|0> = |0>) plus
// -hx times the N single-bit flips.
__global__ void k_cheb(const double2* __restrict__ cur, double2* __restrict__ prev,
                       double2* __restrict__ acc, int N, double J, double hx, double hz,
                       double inv_a, double cr, double ci, int first) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ((int64_t)1 << N)) return;
    const uint64_t u = (uint64_t)k;
    const int bonds_flipped = __popcll((u ^ (u >> 1)) & ((1ull << (N - 1)) - 1));
    const int ones = __popcll(u);
    const double diag = -J * (double)((N - 1) - 2 * bonds_flipped) - hz * (double)(N - 2 * ones);
    const double2 c = cur[k];
    double hr = diag * c.x, hi = diag * c.y;
    for (int i = 0; i < N; ++i) {
        const double2 f = cur[u ^ (1ull << i)];
        hr -= hx * f.x;
        hi -= hx * f.y;
    }
    hr *= inv_a;
    hi *= inv_a;
    double2 nx;
    if (first) {
        nx = make_double2(hr, hi);
    } else {
        const double2 p = prev[k];
        nx = make_double2(2.0 * hr - p.x, 2.0 * hi - p.y);
    }
    prev[k] = nx;
    double2 s = acc[k];
    s.x += cr * nx.x - ci * nx.y;
    s.y += cr * nx.y + ci * nx.x;
    acc[k] = s;
}

// Bessel functions J_0..J_M(x), x > 0, by Miller's backward recurrence
// J_{k-1} = (2k / x) J_k - J_{k+1} from a start far above x, normalised with
// J_0 + 2 sum_{k>=1} J_{2k} = 1 (Abramowitz & Stegun 9.1.27 and 9.1.46).
std::vector<double> bessel_j(double x, int M) {
    const int start = M + 20 + (int)(10.0 + x);
    std::vector<double> j(start + 2, 0.0);
    j[start + 1] = 0.0;
    j[start] = 1e-300;
    for (int k = start; k >= 1; --k) {
        j[k - 1] = (2.0 * k / x) * j[k] - j[k + 1];
        if (std::fabs(j[k - 1]) > 1e250) {  // rescale to stay in range
            for (int q = k - 1; q <= start; ++q) j[q] *= 1e-250;
        }
    }
    double norm = j[0];
    for (int k = 2; k <= start; k += 2) norm += 2.0 * j[k];
    std::vector<double> out(M + 1);
    for (int k = 0; k <= M; ++k) out[k] = j[k] / norm;
    return out;
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct sre2_sim {
    int device = 0;
    int N = 0;
    hipStream_t st = nullptr;
    double2* psi = nullptr;
    double2* wb = nullptr;   // Chebyshev T_k
    double2* acc = nullptr;  // Chebyshev sum
    void* ring[kRing] = {};
    size_t ring_bytes = 0;
};

namespace {

struct Guard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit Guard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess) err = hipSetDevice(dev);
    }
    ~Guard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int launched() { return hipGetLastError() == hipSuccess ? SRE2_OK : SRE2_EHIP; }

int tfim_step(sre2_sim* s, double J, double hx, double hz, double dt) {
    const int N = s->N;
    const int64_t n = int64_t(1) << N;
    // ||H|| <= |J| (N - 1) + (|hx| + |hz|) N
    const double a = std::fabs(J) * (N - 1) + (std::fabs(hx) + std::fabs(hz)) * N;
    if (!(a > 0.0) || dt == 0.0) return SRE2_OK;  // H = 0 or no time: identity
    const double x = a * std::fabs(dt);
    int M = (int)(x + 30.0 + 5.0 * std::cbrt(x));
    const std::vector<double> jb = bessel_j(x, M);
    int K = M;
    while (K > (int)x + 1 && std::fabs(jb[K]) < 1e-17) --K;
    // coefficient of T_k: (2 - [k = 0]) (-i sgn(dt))^k J_k(x)
    auto coef = [&](int k, double* cr, double* ci) {
        const double m = (k == 0 ? 1.0 : 2.0) * jb[k];
        const int r = k & 3;
        const double sg = dt > 0 ? 1.0 : -1.0;
        // (-i sg)^k: r = 0 -> 1, 1 -> -i sg, 2 -> -1, 3 -> i sg
        *cr = r == 0 ? m : (r == 2 ? -m : 0.0);
        *ci = r == 1 ? -sg * m : (r == 3 ? sg * m : 0.0);
    };
    const unsigned nb = blocks_for(n);
    double cr, ci;
    coef(0, &cr, &ci);
    hipLaunchKernelGGL(k_scale_into, dim3(nb), dim3(256), 0, s->st, s->psi, s->acc, n, cr, ci);
    // buffers: psi holds T_0, wb receives T_1; then the newer overwrites the older
    double2* older = s->wb;  // T_{k-1} slot that receives T_{k+1}
    double2* newer = s->psi;
    for (int k = 1; k <= K; ++k) {
        coef(k, &cr, &ci);
        hipLaunchKernelGGL(k_cheb, dim3(nb), dim3(256), 0, s->st, newer, older, s->acc, N, J, hx,
                           hz, 1.0 / a, cr, ci, k == 1 ? 1 : 0);
        double2* t = older;
        older = newer;
        newer = t;
    }
    // the sum is the new state; keep the buffers distinct
    double2* t = s->psi;
    s->psi = s->acc;
    s->acc = t;
    return launched();
}

int apply_gates(sre2_sim* s, const double* gates, const int* pairs, int count) {
    const int64_t groups = int64_t(1) << (s->N - 2);
    for (int g = 0; g < count; ++g) {
        Gate G;
        for (int e = 0; e < 16; ++e) {
            G.re[e] = gates[32 * g + 2 * e];
            G.im[e] = gates[32 * g + 2 * e + 1];
        }
        hipLaunchKernelGGL(k_gate2, dim3(blocks_for(groups)), dim3(256), 0, s->st, s->psi, s->N,
                           pairs[2 * g], pairs[2 * g + 1], G);
    }
    return launched();
}

int check_pairs(int N, const int* pairs, int count) {
    for (int g = 0; g < count; ++g) {
        const int a = pairs[2 * g], b = pairs[2 * g + 1];
        if (a < 0 || b < 0 || a >= N || b >= N || a == b) return SRE2_EINVAL;
    }
    return SRE2_OK;
}

int copy_state(sre2_sim* s, int dtype, void* dst) {
    const int64_t n = int64_t(1) << s->N;
    if (dtype == SRE2_C128) {
        return hipMemcpyAsync(dst, s->psi, (size_t)n * 16, hipMemcpyDeviceToDevice, s->st) ==
                       hipSuccess
                   ? SRE2_OK
                   : SRE2_EHIP;
    }
    return launch_convert(s->psi, kC128, dst, kC64, n, s->st) == hipSuccess ? SRE2_OK : SRE2_EHIP;
}

// Evolution callback of the pipeline: step t (1-based) of the dynamics.
template <typename Step>
int run_pipeline(sre2_sim* s, sre2_server* srv, int steps, int dtype, double* results, Step step) {
    const size_t bytes = (size_t(1) << s->N) * (dtype == SRE2_C64 ? 8 : 16);
    if (s->ring_bytes < bytes) {
        for (void*& r : s->ring) {
            if (r) (void)hipFree(r);
            r = nullptr;
        }
        s->ring_bytes = 0;
        for (void*& r : s->ring)
            if (hipMalloc(&r, bytes) != hipSuccess) {
                (void)hipGetLastError();
                return SRE2_ENOMEM;
            }
        s->ring_bytes = bytes;
    }
    std::vector<uint64_t> tickets(steps + 1, 0);
    auto wait_done = [&](int t) -> int {
        for (;;) {
            int state = 0;
            double lat = 0.0;
            const int rc = sre2_server_poll(srv, tickets[t], &state, results + SRE2_OUT_LEN * t, &lat);
            if (rc) return rc;
            if (state == SRE2_REQ_DONE) return SRE2_OK;
            if (state == SRE2_REQ_CANCELLED) return SRE2_ECANCELLED;
            if (state == SRE2_REQ_FAILED) return SRE2_EHIP;
            std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    };
    for (int t = 0; t <= steps; ++t) {
        int rc = SRE2_OK;
        if (t > 0) rc = step(t);
        if (!rc && t >= kRing) rc = wait_done(t - kRing);  // ring slot free again
        void* slot = s->ring[t % kRing];
        if (!rc) rc = copy_state(s, dtype, slot);
        if (!rc && hipStreamSynchronize(s->st) != hipSuccess) rc = SRE2_EHIP;
        if (!rc) rc = sre2_server_submit(srv, slot, s->N, dtype, 1, &tickets[t]);
        if (rc) {
            // let submitted requests finish before the ring may be reused
            for (int q = t - kRing + 1; q < t; ++q)
                if (q >= 0) (void)wait_done(q);
            return rc;
        }
    }
    for (int t = steps - kRing + 1; t <= steps; ++t) {
        if (t < 0) continue;
        const int rc = wait_done(t);
        if (rc) return rc;
    }
    return SRE2_OK;
}

}  // namespace

extern "C" {

int sre2_sim_create(sre2_sim** out, int hip_device, int N) {
    if (!out || hip_device < 0 || N < 2 || N > kSimMaxN) return SRE2_EINVAL;
    Guard g(hip_device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    sre2_sim* s = new (std::nothrow) sre2_sim();
    if (!s) return SRE2_ENOMEM;
    s->device = hip_device;
    s->N = N;
    const size_t bytes = (size_t(1) << N) * sizeof(double2);
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void**)&s->psi, bytes) != hipSuccess ||
        hipMalloc((void**)&s->wb, bytes) != hipSuccess ||
        hipMalloc((void**)&s->acc, bytes) != hipSuccess) {
        (void)hipGetLastError();
        sre2_sim_destroy(s);
        return SRE2_ENOMEM;
    }
    // start in |0...0> (the product state with every theta_i = 0)
    ProductArgs a{};
    for (int i = 0; i < N; ++i) a.c0[i] = 1.0;
    hipLaunchKernelGGL(k_product, dim3(blocks_for(int64_t(1) << N)), dim3(256), 0, s->st, s->psi,
                       N, a);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->st) != hipSuccess) {
        sre2_sim_destroy(s);
        return SRE2_EHIP;
    }
    *out = s;
    return SRE2_OK;
}

int sre2_sim_destroy(sre2_sim* s) {
    if (!s) return SRE2_OK;
    Guard g(s->device);
    int rc = g.err == hipSuccess ? SRE2_OK : SRE2_EHIP;
    if (s->st) (void)hipStreamSynchronize(s->st);
    void* bufs[] = {s->psi, s->wb, s->acc, s->ring[0], s->ring[1], s->ring[2], s->ring[3]};
    for (void* b : bufs)
        if (b && hipFree(b) != hipSuccess) rc = SRE2_EHIP;
    if (s->st && hipStreamDestroy(s->st) != hipSuccess) rc = SRE2_EHIP;
    delete s;
    return rc;
}

int sre2_sim_product_state(sre2_sim* s, const double* theta, const double* phi) {
    if (!s || !theta || !phi) return SRE2_EINVAL;
    for (int i = 0; i < s->N; ++i)
        if (!std::isfinite(theta[i]) || !std::isfinite(phi[i])) return SRE2_EINVAL;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    ProductArgs a{};
    for (int i = 0; i < s->N; ++i) {
        const double c = std::cos(0.5 * theta[i]), sn = std::sin(0.5 * theta[i]);
        a.c0[i] = c;
        a.c1r[i] = std::cos(phi[i]) * sn;
        a.c1i[i] = std::sin(phi[i]) * sn;
    }
    const int64_t n = int64_t(1) << s->N;
    hipLaunchKernelGGL(k_product, dim3(blocks_for(n)), dim3(256), 0, s->st, s->psi, s->N, a);
    return launched();
}

int sre2_sim_apply_gates(sre2_sim* s, const double* gates, const int* pairs, int count) {
    if (!s || count < 0 || (count > 0 && (!gates || !pairs))) return SRE2_EINVAL;
    int rc = check_pairs(s->N, pairs, count);
    if (rc) return rc;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    return apply_gates(s, gates, pairs, count);
}

int sre2_sim_tfim_step(sre2_sim* s, double J, double hx, double hz, double dt) {
    if (!s || !std::isfinite(J) || !std::isfinite(hx) || !std::isfinite(hz) || !std::isfinite(dt))
        return SRE2_EINVAL;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    return tfim_step(s, J, hx, hz, dt);
}

int sre2_sim_state(sre2_sim* s, int dtype, void* dst) {
    if (!s || !dst || (dtype != SRE2_C64 && dtype != SRE2_C128)) return SRE2_EINVAL;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    int rc = copy_state(s, dtype, dst);
    if (!rc && hipStreamSynchronize(s->st) != hipSuccess) rc = SRE2_EHIP;
    return rc;
}

int sre2_sim_run_tfim(sre2_sim* s, sre2_server* srv, double J, double hx, double hz, double dt,
                      int steps, int dtype, double* results) {
    if (!s || !srv || !results || steps < 0 || (dtype != SRE2_C64 && dtype != SRE2_C128) ||
        !std::isfinite(J) || !std::isfinite(hx) || !std::isfinite(hz) || !std::isfinite(dt))
        return SRE2_EINVAL;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    return run_pipeline(s, srv, steps, dtype, results,
                        [&](int) { return tfim_step(s, J, hx, hz, dt); });
}

int sre2_sim_run_circuit(sre2_sim* s, sre2_server* srv, const double* gates, const int* pairs,
                         int gates_per_step, int steps, int dtype, double* results) {
    if (!s || !srv || !results || steps < 0 || gates_per_step < 0 ||
        (steps > 0 && gates_per_step > 0 && (!gates || !pairs)) ||
        (dtype != SRE2_C64 && dtype != SRE2_C128))
        return SRE2_EINVAL;
    int rc = check_pairs(s->N, pairs, gates_per_step);
    if (rc) return rc;
    Guard g(s->device);
    if (g.err != hipSuccess) return SRE2_EHIP;
    return run_pipeline(s, srv, steps, dtype, results, [&](int t) {
        return apply_gates(s, gates + (size_t)32 * gates_per_step * (t - 1), pairs,
                           gates_per_step);
    });
}

}  // extern "C"
