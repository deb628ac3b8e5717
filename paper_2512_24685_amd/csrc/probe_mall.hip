// probe_mall.hip - memory-hierarchy probe behind the two-pass design (run by
// `python bench.py --mall-probe`; not part of libsre2).
//
// Each workgroup copies its own slice of buffer A into buffer B and back,
// `iters` times, so the footprint is 2 S bytes spread evenly over the XCDs.
// Footprints up to 4 MiB per XCD stay in that XCD's L2, up to the 256 MiB
// MALL in the MALL, beyond that in HBM.  Three access modes: ordinary loads
// and stores, non-temporal ones, and ordinary ones followed by a device-scope
// release (the fence a producer needs before it signals a consumer on
// another XCD) plus an atomic flag per iteration.  Also prints which XCD
// runs each workgroup (HW_REG_XCC_ID).  Every index stays inside its buffer
// (checked on the host before each launch); there are no waits.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#define CHECK(x)                                                             \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) {                                              \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                         \
        }                                                                    \
    } while (0)

typedef float f4 __attribute__((ext_vector_type(4)));

template <int MODE>  // 0 ordinary, 1 non-temporal, 2 ordinary + release per iteration
__global__ __launch_bounds__(256) void k_pingpong(f4* a, f4* b, size_t per_wg, int iters,
                                                  unsigned* flag) {
    const size_t base = (size_t)blockIdx.x * per_wg;
    for (int it = 0; it < iters; ++it) {
        const f4* src = (it & 1) ? b : a;
        f4* dst = (it & 1) ? a : b;
        for (size_t i = threadIdx.x; i < per_wg; i += 256) {
            f4 v = MODE == 1 ? __builtin_nontemporal_load(src + base + i) : src[base + i];
            v.x += 1.0f;
            if (MODE == 1)
                __builtin_nontemporal_store(v, dst + base + i);
            else
                dst[base + i] = v;
        }
        if (MODE == 2) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(flag + blockIdx.x, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ void k_xcc(unsigned* out) {
    if (threadIdx.x == 0)
        out[blockIdx.x] = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((16 - 1) << 11));
}

int main() {
    const size_t max_bytes = size_t(4) << 30;
    const int G = 2048;  // workgroups: 8 per CU
    f4 *a, *b;
    unsigned *flag, *xcc;
    CHECK(hipMalloc(&a, max_bytes));
    CHECK(hipMalloc(&b, max_bytes));
    CHECK(hipMemset(a, 0, max_bytes));
    CHECK(hipMemset(b, 0, max_bytes));
    CHECK(hipMalloc(&flag, G * sizeof(unsigned)));
    CHECK(hipMemset(flag, 0, G * sizeof(unsigned)));
    const int NX = 4096;
    CHECK(hipMalloc(&xcc, NX * sizeof(unsigned)));
    hipLaunchKernelGGL(k_xcc, dim3(NX), dim3(64), 0, 0, xcc);
    CHECK(hipDeviceSynchronize());
    std::vector<unsigned> hx(NX);
    CHECK(hipMemcpy(hx.data(), xcc, NX * sizeof(unsigned), hipMemcpyDeviceToHost));
    int rr = 0;
    for (int i = 0; i < NX; ++i) rr += (int)((hx[i] & 7u) == (unsigned)(i % 8));
    printf("workgroups whose XCD is (id mod 8): %d of %d\n", rr, NX);
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    const size_t sizes_mib[] = {16, 32, 64, 128, 192, 256, 1024, 4096};
    const char* names[] = {"ordinary", "non-temporal", "ordinary+release"};
    for (size_t mib : sizes_mib) {
        const size_t S = mib << 20;
        const size_t per_wg = S / sizeof(f4) / G;
        if (S > max_bytes || per_wg * G * sizeof(f4) > S) {
            printf("bad size\n");
            return 1;
        }
        int iters = (int)((size_t(40) << 30) / (2 * S));
        iters = iters < 4 ? 4 : iters & ~1;
        for (int mode = 0; mode < 3; ++mode) {
            for (int pass = 0; pass < 2; ++pass) {  // pass 0 warms up
                const int it = pass ? iters : 2;
                if (pass) CHECK(hipEventRecord(e0, 0));
                if (mode == 0)
                    hipLaunchKernelGGL(k_pingpong<0>, dim3(G), dim3(256), 0, 0, a, b, per_wg, it, flag);
                else if (mode == 1)
                    hipLaunchKernelGGL(k_pingpong<1>, dim3(G), dim3(256), 0, 0, a, b, per_wg, it, flag);
                else
                    hipLaunchKernelGGL(k_pingpong<2>, dim3(G), dim3(256), 0, 0, a, b, per_wg, it, flag);
                CHECK(hipGetLastError());
                if (pass) CHECK(hipEventRecord(e1, 0));
                CHECK(hipDeviceSynchronize());
            }
            float ms = 0.f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            printf("footprint %5zu MiB  %-16s %5d iterations  %8.3f ms  %6.2f TB/s read+write\n",
                   2 * mib, names[mode], iters, ms, 2.0 * S * iters / (ms * 1e-3) / 1e12);
            fflush(stdout);
        }
    }
    return 0;
}
