/*
 * sre2_oracle.c - plain FP64 CPU oracle for the second-order stabilizer
 * Renyi entropy M2 (Huang, Li, Lee, Zhong, arXiv:2512.24685).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is computed in IEEE double precision with plain scalar loops,
 * no blocking, no fusion and no reordering beyond what each definition says.
 * Build with plain -O2 (no -ffast-math).
 *
 * Quantities (qubit j = bit j of the basis index, LSB = qubit 0):
 *   Pauli string      P = X^x Z^z, x,z in Z_2^N           (main text, bit-string
 *                                                           encoding of Paulis)
 *   expectation       <psi|X^x Z^z|psi>: by the brute force, psi with the
 *                       one-qubit factors of X^x Z^z applied, then an inner
 *                       product; by the transform, Eq. Pauli_expect,
 *                       sum_t (-1)^{z.t} conj(psi[t^x]) psi[t]
 *   SRE, alpha = 2    M2 = -log2( (1/d) sum_{x,z} |<X^x Z^z>|^4 ), d = 2^N  (Eq. 1)
 *   XOR-FWHT form     sum_{x,z} |<X^x Z^z>|^4 = sum_x sum_z |FWHT_k(G_x)(z)|^4,
 *                     G_x[k] = conj(psi[k^x]) psi[k]        (Eq. final1, Algorithm 1)
 *   FWHT              unnormalised Walsh-Hadamard transform, H_2 on every
 *                     qubit in turn, (a,b) -> (a+b, a-b)     (SI, fast WHT section)
 *
 * Reading adopted for unnormalised input: with n = sum_t |psi[t]|^2 the
 * oracle returns M2 = -log2( S / (2^N n^4) ), which is the paper's value when
 * n = 1 and is invariant under psi -> c psi.
 *
 * General Renyi index (Eq. 1), w = |<X^x Z^z>|^2 before normalisation:
 *   alpha != 1        M_alpha = log2( sum w^alpha / (2^N n^(2 alpha)) ) / (1 - alpha)
 *   alpha -> 1        M_1 = -sum_P Xi_P log2 Xi_P - N,  Xi_P = w / (2^N n^2);
 *                     with sum_P w = 2^N n^2 (purity of a pure state) this is
 *                     M_1 = log2(n^2) - (sum w log2 w) / (2^N n^2)
 *   Pauli spectrum    counts of q = w / n^2 in bins b = round(-log2 q), the
 *                     last bin also taking q = 0 and everything beyond it.
 *
 * Arrays are interleaved (re, im) doubles of length 2 * 2^N.  Every function
 * returns 0 on success and a negative value on a bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_N 30

/* Neumaier-compensated running sum, ascending index order. */
static double compensated_sum(const double *v, int64_t n)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = s + v[i];
        if (fabs(s) >= fabs(v[i]))
            c += (s - t) + v[i];
        else
            c += (v[i] - t) + s;
        s = t;
    }
    return s + c;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int sre2o_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* phi = X^x Z^z psi, built one single-qubit factor at a time from the
 * action of the Pauli matrices on the computational basis (main text: a
 * Pauli string is a tensor product of one-qubit Paulis; P = X^x Z^z with
 * x, z in Z_2^N): Z on qubit j flips the sign of every amplitude whose bit j
 * is 1, then X on qubit j exchanges the two amplitudes of every pair that
 * differs only in bit j.  Z^z acts first (it is the right factor). */
static void apply_pauli(const double *psi, int N, uint64_t x, uint64_t z, double *phi)
{
    const uint64_t d = (uint64_t)1 << N;
    memcpy(phi, psi, sizeof(double) * 2 * (size_t)d);
    for (int j = 0; j < N; ++j) {
        const uint64_t m = (uint64_t)1 << j;
        if (!(z & m))
            continue;
        for (uint64_t t = 0; t < d; ++t)
            if (t & m) {
                phi[2 * t] = -phi[2 * t];
                phi[2 * t + 1] = -phi[2 * t + 1];
            }
    }
    for (int j = 0; j < N; ++j) {
        const uint64_t m = (uint64_t)1 << j;
        if (!(x & m))
            continue;
        for (uint64_t t = 0; t < d; ++t)
            if (!(t & m)) {
                const uint64_t u = t | m;
                const double r = phi[2 * t], i = phi[2 * t + 1];
                phi[2 * t] = phi[2 * u];
                phi[2 * t + 1] = phi[2 * u + 1];
                phi[2 * u] = r;
                phi[2 * u + 1] = i;
            }
    }
}

/* <psi|phi> = sum_t conj(psi[t]) phi[t], ascending t. */
static void inner(const double *psi, const double *phi, uint64_t d, double *re, double *im)
{
    double sr = 0.0, si = 0.0;
    for (uint64_t t = 0; t < d; ++t) {
        sr += psi[2 * t] * phi[2 * t] + psi[2 * t + 1] * phi[2 * t + 1];
        si += psi[2 * t] * phi[2 * t + 1] - psi[2 * t + 1] * phi[2 * t];
    }
    *re = sr;
    *im = si;
}

/* <psi| X^x Z^z |psi> of Eq. 1 by applying the Pauli string to psi (not by
 * the index formula of Eq. Pauli_expect, which the transform path uses). */
int sre2o_pauli_expect(const double *psi, int N, uint64_t x, uint64_t z,
                       double *out_re, double *out_im)
{
    if (!psi || !out_re || !out_im || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const uint64_t d = (uint64_t)1 << N;
    if (x >= d || z >= d)
        return -1;
    double *phi = (double *)malloc(sizeof(double) * 2 * (size_t)d);
    if (!phi)
        return -2;
    apply_pauli(psi, N, x, z, phi);
    inner(psi, phi, d, out_re, out_im);
    free(phi);
    return 0;
}

/* Brute force: sum over all 4^N Pauli strings of |<P>|^4 (Eq. 1), each
 * expectation from the Pauli string applied to psi, O(N 8^N).  Per-shift sums
 * are kept and added in ascending shift order. */
int sre2o_brute_sum(const double *psi, int N, int nthreads, double *out_sum)
{
    if (!psi || !out_sum || N < 0 || N > 12)
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *per_x = (double *)malloc(sizeof(double) * (size_t)d);
    if (!per_x)
        return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t x = 0; x < d; ++x) {
        double *q = (double *)malloc(sizeof(double) * (size_t)d);
        double *phi = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        if (!q || !phi) {
#pragma omp atomic write
            err = -2;
        } else {
            for (int64_t z = 0; z < d; ++z) {
                double re, im;
                apply_pauli(psi, N, (uint64_t)x, (uint64_t)z, phi);
                inner(psi, phi, (uint64_t)d, &re, &im);
                const double m = re * re + im * im;
                q[z] = m * m;
            }
            per_x[x] = compensated_sum(q, d);
        }
        free(q);
        free(phi);
    }
    if (!err)
        *out_sum = compensated_sum(per_x, d);
    free(per_x);
    return err;
}

/* In-place unnormalised Walsh-Hadamard transform of an interleaved complex
 * array of length 2^N.  H_{2^N} is the Kronecker product of N copies of the
 * one-qubit H_2 = [[1, 1], [1, -1]] (SI, fast WHT section), so it is applied
 * as H_2 on qubit j for j = 0 .. N-1: the entries t and t + 2^j of every index
 * t with bit j clear, (a, b), become (a + b, a - b). */
int sre2o_fwht(double *a, int N)
{
    if (!a || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const uint64_t d = (uint64_t)1 << N;
    for (int j = 0; j < N; ++j) {
        const uint64_t m = (uint64_t)1 << j;
        for (uint64_t t = 0; t < d; ++t) {
            if (t & m)
                continue;
            const uint64_t u = t | m;
            const double ar = a[2 * t], ai = a[2 * t + 1];
            const double br = a[2 * u], bi = a[2 * u + 1];
            a[2 * t] = ar + br;
            a[2 * t + 1] = ai + bi;
            a[2 * u] = ar - br;
            a[2 * u + 1] = ai - bi;
        }
    }
    return 0;
}

/* W_x = FWHT_k( conj(psi[k^x]) psi[k] ), one shift (Algorithm 1, loop body). */
int sre2o_shift_transform(const double *psi, int N, uint64_t x, double *W)
{
    if (!psi || !W || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const uint64_t d = (uint64_t)1 << N;
    if (x >= d)
        return -1;
    for (uint64_t k = 0; k < d; ++k) {
        const uint64_t u = k ^ x;
        const double ar = psi[2 * u], ai = -psi[2 * u + 1];
        const double br = psi[2 * k], bi = psi[2 * k + 1];
        W[2 * k] = ar * br - ai * bi;
        W[2 * k + 1] = ar * bi + ai * br;
    }
    return sre2o_fwht(W, N);
}

static double shift_partial(const double *psi, int N, uint64_t x, double *W, double *q)
{
    const int64_t d = (int64_t)1 << N;
    sre2o_shift_transform(psi, N, x, W);
    for (int64_t z = 0; z < d; ++z) {
        const double m = W[2 * z] * W[2 * z] + W[2 * z + 1] * W[2 * z + 1];
        q[z] = m * m;
    }
    return compensated_sum(q, d);
}

/* S_x = sum_z |W_x(z)|^4 for each shift in xs[0..nx). */
int sre2o_shift_partials(const double *psi, int N, const int64_t *xs, int64_t nx,
                         int nthreads, double *S)
{
    if (!psi || !S || (!xs && nx > 0) || nx < 0 || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const int64_t d = (int64_t)1 << N;
    for (int64_t i = 0; i < nx; ++i)
        if (xs[i] < 0 || xs[i] >= d)
            return -1;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        double *q = (double *)malloc(sizeof(double) * (size_t)d);
        if (!W || !q) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < nx; ++i)
                S[i] = shift_partial(psi, N, (uint64_t)xs[i], W, q);
        }
        free(W);
        free(q);
    }
    return err;
}

/* S_x for every shift x = 0 .. 2^N - 1. */
int sre2o_all_partials(const double *psi, int N, int nthreads, double *S)
{
    if (!psi || !S || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const int64_t d = (int64_t)1 << N;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        double *q = (double *)malloc(sizeof(double) * (size_t)d);
        if (!W || !q) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t x = 0; x < d; ++x)
                S[x] = shift_partial(psi, N, (uint64_t)x, W, q);
        }
        free(W);
        free(q);
    }
    return err;
}

int sre2o_sum_ascending(const double *v, int64_t n, double *out)
{
    if ((!v && n > 0) || !out || n < 0)
        return -1;
    *out = compensated_sum(v, n);
    return 0;
}

/* n = sum_t |psi[t]|^2 (ascending t, compensated). */
int sre2o_norm2(const double *psi, int N, double *out)
{
    if (!psi || !out || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *q = (double *)malloc(sizeof(double) * (size_t)d);
    if (!q)
        return -2;
    for (int64_t t = 0; t < d; ++t)
        q[t] = psi[2 * t] * psi[2 * t] + psi[2 * t + 1] * psi[2 * t + 1];
    *out = compensated_sum(q, d);
    free(q);
    return 0;
}

/* Inverse participation ratio sum_t |psi(t)|^4 of the state as given (no
 * normalisation), ascending compensated FP64 sum.  By Parseval applied to the
 * x = 0 transform (f_0 = |psi|^2), sum_z |W_0(z)|^2 = 2^N times this value. */
int sre2o_ipr(const double *psi, int N, double *out)
{
    if (!psi || !out || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *q = (double *)malloc(sizeof(double) * (size_t)d);
    if (!q)
        return -2;
    for (int64_t t = 0; t < d; ++t) {
        const double m = psi[2 * t] * psi[2 * t] + psi[2 * t + 1] * psi[2 * t + 1];
        q[t] = m * m;
    }
    *out = compensated_sum(q, d);
    free(q);
    return 0;
}

/* M2 by Algorithm 1: all shifts, FWHT per shift, ascending compensated sum,
 * then M2 = -log2( S / (2^N n^4) ).  Optionally returns S and n. */
int sre2o_m2(const double *psi, int N, int nthreads, double *m2, double *total,
             double *norm2)
{
    if (!psi || !m2 || N < 0 || N > ORACLE_MAX_N)
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *S = (double *)malloc(sizeof(double) * (size_t)d);
    if (!S)
        return -2;
    int rc = sre2o_all_partials(psi, N, nthreads, S);
    if (rc) {
        free(S);
        return rc;
    }
    double s = compensated_sum(S, d);
    free(S);
    double n;
    rc = sre2o_norm2(psi, N, &n);
    if (rc)
        return rc;
    if (!(n > 0.0) || !isfinite(n))
        return -3;
    *m2 = -log2(s / (ldexp(1.0, N) * n * n * n * n));
    if (total)
        *total = s;
    if (norm2)
        *norm2 = n;
    return 0;
}

/* Term of the generalised Pauli sum for one w = |W|^2: kind 1 -> w^alpha,
 * kind 2 -> w log2 w (0 at w = 0). */
static double alpha_term(double w, double alpha, int kind)
{
    if (!(w > 0.0))
        return 0.0;
    return kind == 1 ? pow(w, alpha) : w * log2(w);
}

/* Generalised sums of Eq. 1 by the per-shift FWHT of Algorithm 1, with the
 * quartic replaced by alpha_term: per-shift compensated sums over z, then a
 * compensated sum over x in ascending order. */
int sre2o_alpha_sum(const double *psi, int N, double alpha, int kind, int nthreads,
                    double *out)
{
    if (!psi || !out || N < 0 || N > ORACLE_MAX_N || (kind != 1 && kind != 2) ||
        !(alpha > 0.0))
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *per_x = (double *)malloc(sizeof(double) * (size_t)d);
    if (!per_x)
        return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        double *q = (double *)malloc(sizeof(double) * (size_t)d);
        if (!W || !q) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t x = 0; x < d; ++x) {
                sre2o_shift_transform(psi, N, (uint64_t)x, W);
                for (int64_t z = 0; z < d; ++z)
                    q[z] = alpha_term(W[2 * z] * W[2 * z] + W[2 * z + 1] * W[2 * z + 1], alpha,
                                      kind);
                per_x[x] = compensated_sum(q, d);
            }
        }
        free(W);
        free(q);
    }
    if (!err)
        *out = compensated_sum(per_x, d);
    free(per_x);
    return err;
}

/* The same sums over all 4^N Pauli strings with every expectation value from
 * the Pauli string applied to psi, O(N 8^N), N <= 12. */
int sre2o_brute_alpha_sum(const double *psi, int N, double alpha, int kind, int nthreads,
                          double *out)
{
    if (!psi || !out || N < 0 || N > 12 || (kind != 1 && kind != 2) || !(alpha > 0.0))
        return -1;
    const int64_t d = (int64_t)1 << N;
    double *per_x = (double *)malloc(sizeof(double) * (size_t)d);
    if (!per_x)
        return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t x = 0; x < d; ++x) {
        double *q = (double *)malloc(sizeof(double) * (size_t)d);
        double *phi = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        if (!q || !phi) {
#pragma omp atomic write
            err = -2;
        } else {
            for (int64_t z = 0; z < d; ++z) {
                double re, im;
                apply_pauli(psi, N, (uint64_t)x, (uint64_t)z, phi);
                inner(psi, phi, (uint64_t)d, &re, &im);
                q[z] = alpha_term(re * re + im * im, alpha, kind);
            }
            per_x[x] = compensated_sum(q, d);
        }
        free(q);
        free(phi);
    }
    if (!err)
        *out = compensated_sum(per_x, d);
    free(per_x);
    return err;
}

/* Pauli-spectrum histogram: for every Pauli string, q = |W|^2 / n^2 goes to
 * bin round(-log2 q) (clamped to [0, nbins - 1]; q = 0 to the last bin).
 * near_edge counts the strings whose -log2 q lies within eps of an edge
 * between two bins (b + 1/2, b = 0 .. nbins - 2), where a rounding of the
 * expectation value can change the bin. */
int sre2o_spectrum(const double *psi, int N, int nbins, double eps, int nthreads,
                   int64_t *counts, int64_t *near_edge)
{
    if (!psi || !counts || !near_edge || N < 0 || N > ORACLE_MAX_N || nbins < 2 ||
        nbins > 64 || !(eps >= 0.0))
        return -1;
    const int64_t d = (int64_t)1 << N;
    double n;
    int rc = sre2o_norm2(psi, N, &n);
    if (rc)
        return rc;
    if (!(n > 0.0) || !isfinite(n))
        return -3;
    int64_t total[64] = {0};
    int64_t near = 0;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel
    {
        int64_t mine[64] = {0};
        int64_t mnear = 0;
        double *W = (double *)malloc(sizeof(double) * 2 * (size_t)d);
        if (!W) {
#pragma omp atomic write
            err = -2;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t x = 0; x < d; ++x) {
                sre2o_shift_transform(psi, N, (uint64_t)x, W);
                for (int64_t z = 0; z < d; ++z) {
                    const double q = (W[2 * z] * W[2 * z] + W[2 * z + 1] * W[2 * z + 1]) / (n * n);
                    int b = nbins - 1;
                    if (q > 0.0) {
                        const double t = -log2(q);
                        const double f = floor(t + 0.5);
                        b = f < 0.0 ? 0 : (f > nbins - 1 ? nbins - 1 : (int)f);
                        /* nearest edge e + 1/2 between bins e and e + 1 */
                        const double r = t - 0.5;
                        const double e = floor(r + 0.5);
                        if (e >= 0.0 && e <= nbins - 2 && fabs(r - e) <= eps)
                            ++mnear;
                    }
                    ++mine[b];
                }
            }
        }
        free(W);
#pragma omp critical
        {
            for (int b = 0; b < nbins; ++b)
                total[b] += mine[b];
            near += mnear;
        }
    }
    if (err)
        return err;
    for (int b = 0; b < nbins; ++b)
        counts[b] = total[b];
    *near_edge = near;
    return 0;
}
