// Host-side driver of the C ABI for the sanitizer build: every call takes a
// path that is decided on the host (argument checks, sizing queries,
// context bookkeeping), as tests/test_abi.py exercises them.  Fake device
// pointers are never dereferenced.  Exit status 0 when every return code is
// the expected one.
#include <stdio.h>
#include <stdint.h>

#include "../../include/sre2.h"

static int failures = 0;
#define EXPECT(call, want)                                                          \
    do {                                                                            \
        const long long got_ = (long long)(call);                                  \
        if (got_ != (long long)(want)) {                                           \
            printf("FAIL %s = %lld, expected %lld\n", #call, got_, (long long)(want)); \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

int main() {
    void* fake = (void*)0x10000;
    double* fout = (double*)0x20000;
    EXPECT(sre2_version() >= 100, 1);
    for (int c = 1; c >= -12; --c) EXPECT(sre2_strerror(c) != NULL, 1);
    sre2_ctx* ctx = NULL;
    EXPECT(sre2_create(NULL, 0), SRE2_EINVAL);
    EXPECT(sre2_create(&ctx, -1), SRE2_EINVAL);
    EXPECT(sre2_create(&ctx, 0), SRE2_OK);
    EXPECT(sre2_set_scratch_limit(ctx, size_t(1) << 20), SRE2_OK);
    EXPECT(sre2_set_scratch_limit(ctx, size_t(32) << 30), SRE2_OK);
    EXPECT(sre2_set_row_pairs(ctx, 0), SRE2_OK);
    EXPECT(sre2_set_row_pairs(ctx, 1), SRE2_OK);
    EXPECT(sre2_set_row_pairs(nullptr, 1), SRE2_EINVAL);
    EXPECT(sre2_set_timing(ctx, 1), SRE2_OK);
    double ms[SRE2_KIND_COUNT];
    int64_t launches[SRE2_KIND_COUNT];
    EXPECT(sre2_timing_read(ctx, ms, launches), SRE2_OK);
    EXPECT(sre2_timing_read(ctx, NULL, launches), SRE2_EINVAL);
    // argument checks of every entry point
    EXPECT(sre2_m2(NULL, fake, 10, 0, 0, NULL, fout, NULL), SRE2_EINVAL);
    EXPECT(sre2_m2(ctx, NULL, 10, 0, 0, NULL, fout, NULL), SRE2_EINVAL);
    EXPECT(sre2_m2(ctx, fake, 0, 0, 0, NULL, fout, NULL), SRE2_EINVAL);
    EXPECT(sre2_m2(ctx, fake, 27, 0, 0, NULL, fout, NULL), SRE2_EINVAL);
    EXPECT(sre2_m2(ctx, fake, 10, 7, 0, NULL, fout, NULL), SRE2_EDTYPE);
    EXPECT(sre2_m2(ctx, fake, 10, 0, 99, NULL, fout, NULL), SRE2_EFORM);
    EXPECT(sre2_m2(ctx, fake, 25, 0, SRE2_FORM_FP64, NULL, fout, NULL), SRE2_EFORM);
    EXPECT(sre2_m2(ctx, fake, 10, 0, 0, NULL, NULL, NULL), SRE2_EINVAL);
    EXPECT(sre2_sre(ctx, fake, 10, 0, 0, -1.0, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_sre(ctx, fake, 10, 0, SRE2_FORM_SPLIT_F16, 3.0, NULL, fout), SRE2_EFORM);
    EXPECT(sre2_pauli_spectrum(ctx, fake, 10, 0, 0, 1, NULL, (uint64_t*)fake, fout), SRE2_EINVAL);
    EXPECT(sre2_pauli_spectrum(ctx, fake, 10, 0, 0, 65, NULL, (uint64_t*)fake, fout), SRE2_EINVAL);
    EXPECT(sre2_partials(ctx, fake, 4, 0, 0, 0, 17, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_partials(ctx, fake, 4, 0, 0, -1, 2, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_partials(ctx, fake, 4, 0, 0, 15, 2, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_moments(ctx, fake, 27, 0, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_moments(ctx, fake, 4, 2, NULL, fout), SRE2_EDTYPE);
    const void* ptrs[2] = {fake, fake};
    int Ns[2] = {8, 40};
    EXPECT(sre2_m2_batched(ctx, ptrs, Ns, 0, 0, 0, NULL, fout), SRE2_EINVAL);
    EXPECT(sre2_m2_batched(ctx, ptrs, Ns, 2, 0, 0, NULL, fout), SRE2_EINVAL);
    // sizing queries over every shape
    for (int form = -1; form <= 6; ++form)
        for (int N = 0; N <= 27; ++N) {
            for (int dt = -1; dt <= 2; ++dt) (void)sre2_workspace_bytes(N, dt, form);
            (void)sre2_row_bits(N, form);
            int64_t cs = 0;
            int P = 0;
            (void)sre2_chunking(ctx, N, form, &cs, &P);
            // the allocation-free call lays out its array for every shape and
            // rejects what it cannot hold; the rest reaches the (absent) device
            for (int dt = 0; dt <= 1; ++dt) {
                const int rc = sre2_m2_noalloc(0, fake, N, dt, form, NULL, fout, NULL);
                EXPECT(rc == SRE2_EINVAL || rc == SRE2_EFORM || rc == SRE2_ESCRATCH ||
                           rc == SRE2_EHIP,
                       1);
            }
        }
    EXPECT(sre2_m2_noalloc(0, fake, 21, SRE2_C64, SRE2_FORM_FP32, NULL, fout, NULL),
           SRE2_ESCRATCH);
    EXPECT(sre2_m2_noalloc(0, fake, 26, SRE2_C128, SRE2_FORM_FP32_HERM, NULL, fout, NULL),
           SRE2_ESCRATCH);
    EXPECT(sre2_m2_noalloc(-1, fake, 10, SRE2_C64, SRE2_FORM_FP32, NULL, fout, NULL),
           SRE2_EINVAL);
    EXPECT(sre2_workspace_bytes(20, SRE2_C64, SRE2_FORM_FP32) > (size_t(32) << 30), 1);
    EXPECT(sre2_destroy(ctx), SRE2_OK);
    EXPECT(sre2_destroy(NULL), SRE2_OK);
    // serving and simulator argument checks (no device is touched)
    sre2_server* srv = NULL;
    EXPECT(sre2_server_create(NULL, 0, 0, size_t(1) << 30, 8), SRE2_EINVAL);
    EXPECT(sre2_server_create(&srv, 0, 0, 1024, 8), SRE2_EINVAL);
    EXPECT(sre2_server_create(&srv, 0, 99, size_t(1) << 30, 8), SRE2_EFORM);
    EXPECT(sre2_server_destroy(NULL), SRE2_OK);
    sre2_sim* sim = NULL;
    EXPECT(sre2_sim_create(&sim, 0, 1), SRE2_EINVAL);
    EXPECT(sre2_sim_create(&sim, 0, 27), SRE2_EINVAL);
    EXPECT(sre2_sim_destroy(NULL), SRE2_OK);
    printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
