/*
 * Driver that runs every FP64 oracle function on small seeded inputs, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py (test infrastructure: it checks the oracle's
 * memory accesses and arithmetic for undefined behaviour, not its values,
 * which the pin tests cover).  Exit status 0 when every call returned the
 * expected status and every result is finite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

double oracle_sqdist(const double *u, const double *v, int d);
double oracle_phi(double D, int kernel, double nu, double rho, double amp);
int oracle_neighborhood(const double *X, int64_t n, int d, int64_t i, int k, int mode,
                        int32_t *nb);
int64_t oracle_nearest(const double *X, int64_t n, int d, const double *z, double *dmin);
int64_t oracle_build(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                     int kernel, double nu, double rho, double noise, double amp, int mode,
                     const int64_t *rows, int64_t nrows, int32_t *nb_out, double *C_out,
                     int32_t *status_out, int nthreads);
void oracle_nearest_batch(const double *X, int64_t n, int d, const double *Z, int64_t m,
                          int64_t *nn_out, double *dmin_out, int nthreads);
void oracle_mean_batch(const double *X, int d, int ell, int k, int kernel, double nu, double rho,
                       double amp, const double *Z, int64_t m, const int32_t *nb,
                       const double *C, double *out, int nthreads);
void oracle_muygps_batch(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                         int kernel, double nu, double rho, double noise, double amp,
                         const double *Z, int64_t m, int32_t *nb_out, double *out,
                         int32_t *status_out, int nthreads);
double oracle_dphi_drho(double D, int kernel, double nu, double rho, double amp);
int64_t oracle_loo_loss_grad(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                             int kernel, double nu, double rho, double noise, double amp,
                             const int64_t *rows, int64_t nrows, double *terms,
                             int32_t *status_out, int nthreads);

static uint64_t state = 0x9e3779b97f4a7c15ull;

static double uniform(void) /* xorshift64*, top 53 bits */
{
    state ^= state >> 12;
    state ^= state << 25;
    state ^= state >> 27;
    return (double)((state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;

static void expect(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static int all_finite(const double *a, int64_t cnt)
{
    for (int64_t i = 0; i < cnt; ++i)
        if (!isfinite(a[i]))
            return 0;
    return 1;
}

static void run(int64_t n, int d, int ell, int k, int kernel, double nu, int mode, int dups)
{
    const int64_t m = 13;
    double *X = malloc(sizeof(double) * n * d), *Y = malloc(sizeof(double) * n * ell);
    double *Z = malloc(sizeof(double) * m * d);
    for (int64_t i = 0; i < n * d; ++i)
        X[i] = uniform();
    if (dups) /* the second half repeats the first: exact distance ties */
        for (int64_t i = n / 2; i < n; ++i)
            for (int c = 0; c < d; ++c)
                X[i * d + c] = X[(i - n / 2) * d + c];
    for (int64_t i = 0; i < n * ell; ++i)
        Y[i] = uniform() - 0.5;
    for (int64_t i = 0; i < m * d; ++i)
        Z[i] = uniform();
    int32_t *nb = malloc(sizeof(int32_t) * n * k);
    double *C = malloc(sizeof(double) * n * k * ell);
    int32_t *st = malloc(sizeof(int32_t) * n);
    const double rho = 0.4, noise = 1e-2, amp = 1.0;
    int64_t bad = oracle_build(X, Y, n, d, ell, k, kernel, nu, rho, noise, amp, mode, NULL, 0, nb,
                               C, st, 1);
    expect(bad == 0, "build status");
    expect(all_finite(C, n * k * ell), "finite coefficients");
    int64_t rows[3] = {0, n / 2, n - 1};
    int32_t nb3[3 * 256];
    double C3[3 * 256 * 4];
    int32_t st3[3];
    expect(oracle_build(X, Y, n, d, ell, k, kernel, nu, rho, noise, amp, mode, rows, 3, nb3, C3,
                        st3, 1) == 0, "build of sampled rows");
    int64_t nn[13];
    double dmin[13], mu[13 * 4];
    oracle_nearest_batch(X, n, d, Z, m, nn, dmin, 1);
    for (int64_t t = 0; t < m; ++t)
        expect(nn[t] >= 0 && nn[t] < n, "nearest index");
    /* each query's neighbourhood and coefficient row: those of its nearest point */
    int32_t *nbj = malloc(sizeof(int32_t) * m * k);
    double *Cj = malloc(sizeof(double) * m * k * ell);
    for (int64_t t = 0; t < m; ++t) {
        for (int s = 0; s < k; ++s)
            nbj[t * k + s] = nb[nn[t] * k + s];
        for (int64_t e = 0; e < (int64_t)k * ell; ++e)
            Cj[t * k * ell + e] = C[nn[t] * k * ell + e];
    }
    oracle_mean_batch(X, d, ell, k, kernel, nu, rho, amp, Z, m, nbj, Cj, mu, 1);
    free(nbj);
    free(Cj);
    expect(all_finite(mu, m * ell), "finite means");
    int32_t nbq[13 * 256], stq[13];
    double muq[13 * 4];
    oracle_muygps_batch(X, Y, n, d, ell, k, kernel, nu, rho, noise, amp, Z, m, nbq, muq, stq, 1);
    for (int64_t t = 0; t < m; ++t)
        expect(stq[t] == 0, "MuyGPs status");
    if (mode == 0) {
        double terms[3 * 3];
        int32_t stl[3];
        expect(oracle_loo_loss_grad(X, Y, n, d, ell, k, kernel, nu, rho, noise, amp, rows, 3,
                                    terms, stl, 1) == 0,
               "loss gradient status");
        expect(all_finite(terms, 9), "finite loss terms");
    }
    expect(isfinite(oracle_dphi_drho(oracle_sqdist(X, X + d, d), kernel, nu, rho, amp)),
           "finite dphi/drho");
    expect(oracle_phi(0.0, kernel, nu, rho, amp) == amp, "phi(0) = a");
    free(X);
    free(Y);
    free(Z);
    free(nb);
    free(C);
    free(st);
}

int main(void)
{
    /* every kernel, both neighbourhood modes, k = 1, k = n - 1 (leave one
     * out) and k = n (self-inclusive), duplicated points, several responses */
    run(200, 3, 2, 20, 1, 0.5, 0, 0);
    run(150, 2, 1, 30, 1, 1.5, 0, 1);
    run(120, 4, 3, 16, 1, 2.5, 1, 0);
    run(90, 5, 4, 25, 0, 0.0, 0, 0);
    run(60, 2, 1, 1, 1, 1.5, 0, 0);
    run(40, 3, 2, 39, 0, 0.0, 0, 0);
    run(40, 3, 2, 40, 1, 2.5, 1, 0);
    run(300, 8, 1, 150, 1, 1.5, 0, 0);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle driver: all calls clean\n");
    return 0;
}
