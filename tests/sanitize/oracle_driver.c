/* Driver of the FP64 oracle for the sanitizer build: every entry point on
 * small seeded states (N <= 6), plus its argument checks.  Exit status 0 when
 * every call returns as expected and the brute force agrees with the XOR-FWHT
 * sums (Eq. 1 against Algorithm 1). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int sre2o_pauli_expect(const double *, int, uint64_t, uint64_t, double *, double *);
int sre2o_brute_sum(const double *, int, int, double *);
int sre2o_fwht(double *, int);
int sre2o_shift_transform(const double *, int, uint64_t, double *);
int sre2o_shift_partials(const double *, int, const int64_t *, int64_t, int, double *);
int sre2o_all_partials(const double *, int, int, double *);
int sre2o_sum_ascending(const double *, int64_t, double *);
int sre2o_norm2(const double *, int, double *);
int sre2o_ipr(const double *, int, double *);
int sre2o_m2(const double *, int, int, double *, double *, double *);
int sre2o_alpha_sum(const double *, int, double, int, int, double *);
int sre2o_brute_alpha_sum(const double *, int, double, int, int, double *);
int sre2o_spectrum(const double *, int, int, double, int, int64_t *, int64_t *);

static int failures = 0;
#define EXPECT(c)                                  \
    do {                                           \
        if (!(c)) {                                \
            printf("FAIL line %d: %s\n", __LINE__, #c); \
            ++failures;                            \
        }                                          \
    } while (0)

int main(void)
{
    uint64_t s = 0x9e3779b97f4a7c15ull;
    for (int N = 1; N <= 6; ++N) {
        const int d = 1 << N;
        double *psi = malloc(sizeof(double) * 2 * d);
        double *W = malloc(sizeof(double) * 2 * d);
        double *S = malloc(sizeof(double) * d);
        for (int i = 0; i < 2 * d; ++i) {
            s = s * 6364136223846793005ull + 1442695040888963407ull;
            psi[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
        }
        double m2, tot, n, brute, ipr, re, im, a, b, sum;
        EXPECT(sre2o_m2(psi, N, 2, &m2, &tot, &n) == 0);
        EXPECT(sre2o_brute_sum(psi, N, 2, &brute) == 0);
        EXPECT(fabs(brute - tot) <= 1e-12 * tot);
        EXPECT(sre2o_norm2(psi, N, &n) == 0 && sre2o_ipr(psi, N, &ipr) == 0);
        EXPECT(sre2o_pauli_expect(psi, N, (uint64_t)(d - 1), 1, &re, &im) == 0);
        EXPECT(sre2o_shift_transform(psi, N, 1, W) == 0);
        EXPECT(sre2o_all_partials(psi, N, 2, S) == 0);
        int64_t xs[2] = {0, d - 1};
        double S2[2];
        EXPECT(sre2o_shift_partials(psi, N, xs, 2, 2, S2) == 0);
        EXPECT(S2[0] == S[0] && S2[1] == S[d - 1]);
        EXPECT(sre2o_sum_ascending(S, d, &sum) == 0 && fabs(sum - tot) <= 1e-13 * tot);
        EXPECT(sre2o_alpha_sum(psi, N, 1.5, 1, 2, &a) == 0);
        EXPECT(sre2o_brute_alpha_sum(psi, N, 1.5, 1, 2, &b) == 0 && fabs(a - b) <= 1e-12 * b);
        EXPECT(sre2o_alpha_sum(psi, N, 1.0, 2, 2, &a) == 0);
        int64_t counts[16], near;
        EXPECT(sre2o_spectrum(psi, N, 16, 1e-3, 2, counts, &near) == 0);
        int64_t tsum = 0;
        for (int i = 0; i < 16; ++i) tsum += counts[i];
        EXPECT(tsum == (int64_t)d * d);
        EXPECT(sre2o_fwht(W, N) == 0);
        free(psi);
        free(W);
        free(S);
    }
    double v = 0.0, x[2] = {1.0, 0.0};
    int64_t c[4], nr;
    EXPECT(sre2o_m2(NULL, 3, 1, &v, NULL, NULL) == -1);
    EXPECT(sre2o_m2(x, 31, 1, &v, NULL, NULL) == -1);
    EXPECT(sre2o_pauli_expect(x, 0, 1, 0, &v, &v) == -1);
    EXPECT(sre2o_brute_sum(x, 13, 1, &v) == -1);
    EXPECT(sre2o_spectrum(x, 0, 1, 0.0, 1, c, &nr) == -1);
    EXPECT(sre2o_alpha_sum(x, 0, -1.0, 1, 1, &v) == -1);
    printf("%s: %d failures\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
