// probe_store.hip - HBM store-rate probe behind the two-pass slab layout (run
// as `paper_2512_24685_amd/probe_store`; not part of libsre2).
//
// Writes 4 GiB with 256-thread workgroups of 32 KiB each (one pass-1 row of
// 2^12 complex64 values per workgroup), five times per pattern, and prints
// the rate of each:
//   A  pass 1's lane order: 8-byte non-temporal stores, lanes 0-3 on value
//      bits 0-3, the 16 registers on bits 4-7, lanes 4-5 on bits 8-9, the
//      wave on bits 10-11 (each instruction writes four 128-byte runs);
//   B  the same values as 16-byte stores (adjacent pairs per lane);
//   C  A with ordinary (cached) stores;
//   D  16-byte stores, 64 lanes contiguous per instruction;
//   E4, E8, E16  A's order inside the workgroup, but the 32 KiB row cut into
//      8 pieces of 4 KiB interleaved with those of the G - 1 neighbouring
//      workgroups in dispatch order (G = 4, 8, 16).
// Arguments: [patterns [rounds]], e.g. `probe_store A 1` (default: all
// patterns, three rounds).  Every store stays inside the buffer (the
// workgroup count is a multiple of every G; checked on the host before the
// launches); the kernels have no waits.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define CHECK(x)                                                                  \
    do {                                                                          \
        hipError_t e_ = (x);                                                      \
        if (e_ != hipSuccess) {                                                   \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr size_t kBytes = 4ull << 30;
constexpr unsigned kRowValues = 4096;  // complex64 values per workgroup (32 KiB)

// value index inside the row of thread t, register i (pattern A's order)
__device__ __forceinline__ unsigned row_value(unsigned t, int i) {
    const unsigned l = t & 63, w = t >> 6;
    return (l & 15) | ((l >> 4) << 8) | (w << 10) | ((unsigned)i << 4);
}

template <bool NT>
__global__ __launch_bounds__(256) void k_rowA(f2* out) {
    f2* o = out + (size_t)blockIdx.x * kRowValues;
    f2 v = {(float)threadIdx.x, 1.0f};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (NT)
            __builtin_nontemporal_store(v, o + row_value(threadIdx.x, i));
        else
            o[row_value(threadIdx.x, i)] = v;
        v.y += 1.0f;
    }
}

__global__ __launch_bounds__(256) void k_rowB(f4* out) {
    // pairs: lanes 0-3 on pair bits 0-3, registers on bits 4-6, lanes 4-5 on
    // bits 7-8, the wave on bits 9-10
    const unsigned t = threadIdx.x, l = t & 63, w = t >> 6;
    const unsigned base = (l & 15) | ((l >> 4) << 7) | (w << 9);
    f4* o = out + (size_t)blockIdx.x * (kRowValues / 2);
    f4 v = {(float)t, 1.0f, 2.0f, 3.0f};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        __builtin_nontemporal_store(v, o + base + (i << 4));
        v.y += 1.0f;
    }
}

__global__ __launch_bounds__(256) void k_rowD(f4* out) {
    f4* o = out + (size_t)blockIdx.x * (kRowValues / 2);
    f4 v = {(float)threadIdx.x, 1.0f, 2.0f, 3.0f};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        __builtin_nontemporal_store(v, o + threadIdx.x + i * 256);
        v.y += 1.0f;
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_rowE(f2* out) {
    const size_t b = blockIdx.x;
    f2 v = {(float)threadIdx.x, 1.0f};
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const unsigned e = row_value(threadIdx.x, i);
        const size_t piece = ((b / G) * 8 + (e >> 9)) * G + (b % G);
        __builtin_nontemporal_store(v, out + piece * 512 + (e & 511));
        v.y += 1.0f;
    }
}

int main(int argc, char** argv) {
    const char* only = argc > 1 ? argv[1] : nullptr;  // comma-separated pattern names
    const int rounds = argc > 2 ? atoi(argv[2]) : 3;
    if (rounds < 1 || rounds > 100) {
        printf("rounds must be in [1, 100]\n");
        return 1;
    }
    void* buf = nullptr;
    CHECK(hipMalloc(&buf, kBytes));
    const unsigned wgs = (unsigned)(kBytes / (kRowValues * sizeof(f2)));
    if (wgs % 16 != 0) {
        printf("workgroup count %u is not a multiple of 16\n", wgs);
        return 1;
    }
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    const char* names[] = {"A", "B", "C", "D", "E4", "E8", "E16"};
    for (int rep = 0; rep < rounds; ++rep) {
        for (int k = 0; k < 7; ++k) {
            if (only) {
                bool want = false;
                const size_t n = strlen(names[k]);
                for (const char* p = only; *p;) {
                    const char* q = strchr(p, ',');
                    const size_t len = q ? (size_t)(q - p) : strlen(p);
                    want = want || (len == n && strncmp(p, names[k], n) == 0);
                    p = q ? q + 1 : p + len;
                }
                if (!want) continue;
            }
            for (int timed = 0; timed < 2; ++timed) {  // one untimed round first
                CHECK(hipEventRecord(a));
                for (int it = 0; it < 5; ++it) {
                    switch (k) {
                        case 0: hipLaunchKernelGGL(k_rowA<true>, dim3(wgs), dim3(256), 0, 0, (f2*)buf); break;
                        case 1: hipLaunchKernelGGL(k_rowB, dim3(wgs), dim3(256), 0, 0, (f4*)buf); break;
                        case 2: hipLaunchKernelGGL(k_rowA<false>, dim3(wgs), dim3(256), 0, 0, (f2*)buf); break;
                        case 3: hipLaunchKernelGGL(k_rowD, dim3(wgs), dim3(256), 0, 0, (f4*)buf); break;
                        case 4: hipLaunchKernelGGL(k_rowE<4>, dim3(wgs), dim3(256), 0, 0, (f2*)buf); break;
                        case 5: hipLaunchKernelGGL(k_rowE<8>, dim3(wgs), dim3(256), 0, 0, (f2*)buf); break;
                        default: hipLaunchKernelGGL(k_rowE<16>, dim3(wgs), dim3(256), 0, 0, (f2*)buf); break;
                    }
                    CHECK(hipGetLastError());
                }
                CHECK(hipEventRecord(b));
                CHECK(hipEventSynchronize(b));
                float ms = 0.0f;
                CHECK(hipEventElapsedTime(&ms, a, b));
                if (timed)
                    printf("round %d pattern %-3s %.3f ms per 4 GiB, %.2f TB/s\n", rep, names[k], ms / 5,
                           (double)kBytes / (ms / 5 * 1e-3) / 1e12);
            }
        }
    }
    fflush(stdout);
    CHECK(hipFree(buf));
    return 0;
}
