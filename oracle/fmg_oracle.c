/*
 * FastMuyGPs FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, sequential, obviously
 * correct statement of what the FastMuyGPs posterior-mean path computes.  It
 * shares no code with the HIP library under paper_2205_10879_amd/: no header,
 * no helper, no table.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load it.  The product path never does.
 *
 * Everything is IEEE double, built with -O2 -ffp-contract=off and without
 * fast-math, so every product, difference and sum is rounded on its own, in
 * the order written.  Item loops (training rows, queries) may run on several
 * OpenMP threads; the arithmetic of one item is sequential, so results do not
 * depend on the thread count.
 *
 * Paper: Dunton, Priest, Muyskens, "Fast Gaussian Process Posterior Mean
 * Prediction via Local Cross Validation and Precomputation" (arXiv 2205.10879).
 *
 * Readings taken where the paper is silent or ambiguous (each also listed in
 * the design notes):
 *   - neighbourhoods are leave-one-out by default: N(i) is the k nearest
 *     training points other than i.  MODE_SELF gives the paper-literal set
 *     S_i = [i ; k-1 nearest others] of Algorithm 2;
 *   - ranking uses the squared Euclidean distance, ties go to the smaller
 *     index;
 *   - the nugget sigma^2 is added by index on the training diagonal only,
 *     never to a cross-covariance, with unit amplitude a;
 *   - RBF is exp(-r^2 / (2 rho^2)), the nu -> infinity limit of the Matern
 *     form (Section 2, Matern kernel paragraph);
 *   - C_{N*} in the prediction formula is the coefficient row C_j of the
 *     query's nearest training point j (Section 3, prediction paragraph).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_RBF = 0, ORACLE_MATERN = 1 };
enum { ORACLE_MODE_LOO = 0, ORACLE_MODE_SELF = 1 };

/* Squared Euclidean distance, summed over coordinates left to right, each
 * difference, square and partial sum rounded separately.  Section 2: the
 * kernels are stationary and isotropic, functions of ||x - x'|| only. */
double oracle_sqdist(const double *u, const double *v, int d)
{
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
        double t = u[c] - v[c];
        double t2 = t * t;
        s = s + t2;
    }
    return s;
}

/* Kernel value phi from the squared distance D.
 * Matern (Section 2, Matern equation) at the half-integer smoothness values,
 * where the Bessel-function form reduces to a polynomial times an
 * exponential in s = sqrt(2 nu) r / rho:
 *   nu = 1/2 : a exp(-s)                      (the exponential kernel)
 *   nu = 3/2 : a (1 + s) exp(-s)
 *   nu = 5/2 : a (1 + s + s^2/3) exp(-s)
 * RBF, the nu -> infinity limit: a exp(-D / (2 rho^2)).
 * Returns NaN for an unsupported nu. */
double oracle_phi(double D, int kernel, double nu, double rho, double amp)
{
    if (kernel == ORACLE_RBF)
        return amp * exp(-D / (2.0 * rho * rho));
    double r = sqrt(D);
    if (nu == 0.5) {
        double s = r / rho;
        return amp * exp(-s);
    }
    if (nu == 1.5) {
        double s = sqrt(3.0) * r / rho;
        return amp * (1.0 + s) * exp(-s);
    }
    if (nu == 2.5) {
        double s = sqrt(5.0) * r / rho;
        return amp * (1.0 + s + s * s / 3.0) * exp(-s);
    }
    return NAN;
}

/* (D, p) < (D', p') lexicographically: smaller distance first, ties to the
 * smaller index. */
static int key_less(double da, int64_t pa, double db, int64_t pb)
{
    return da < db || (da == db && pa < pb);
}

/* The `want` smallest keys (D(x_i, x_p), p) over training points p != skip
 * (skip < 0: no exclusion), ascending.  Brute force over p = 0 .. n-1 in
 * order, keeping a sorted list by insertion.  Returns how many were found
 * (min(want, candidates)). */
static int64_t smallest_keys(const double *X, int64_t n, int d, const double *q,
                             int64_t skip, int64_t want, int64_t *idx, double *dist)
{
    int64_t cnt = 0;
    for (int64_t p = 0; p < n; ++p) {
        if (p == skip)
            continue;
        double D = oracle_sqdist(q, X + p * d, d);
        if (cnt == want && !key_less(D, p, dist[cnt - 1], idx[cnt - 1]))
            continue;
        int64_t pos = (cnt < want) ? cnt : want - 1;
        while (pos > 0 && key_less(D, p, dist[pos - 1], idx[pos - 1])) {
            dist[pos] = dist[pos - 1];
            idx[pos] = idx[pos - 1];
            --pos;
        }
        dist[pos] = D;
        idx[pos] = p;
        if (cnt < want)
            ++cnt;
    }
    return cnt;
}

/* Neighbourhood of training point i (Algorithm 2, offline loop).
 * LOO: the k nearest training points other than i.
 * SELF: i itself followed by its k-1 nearest other points.
 * Writes k indices; returns 0, or -1 when there are too few points. */
int oracle_neighborhood(const double *X, int64_t n, int d, int64_t i, int k,
                        int mode, int32_t *out)
{
    int64_t want = (mode == ORACLE_MODE_SELF) ? k - 1 : k;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (want > 0 ? want : 1));
    double *dist = (double *)malloc(sizeof(double) * (want > 0 ? want : 1));
    int64_t got = want > 0 ? smallest_keys(X, n, d, X + i * d, i, want, idx, dist) : 0;
    int rc = (got == want) ? 0 : -1;
    int o = 0;
    if (mode == ORACLE_MODE_SELF)
        out[o++] = (int32_t)i;
    for (int64_t s = 0; s < got; ++s)
        out[o++] = (int32_t)idx[s];
    free(idx);
    free(dist);
    return rc;
}

/* Nearest training point of z: argmin over all p of (D(z, x_p), p)
 * (Algorithm 2, online loop: the query's nearest training point). */
int64_t oracle_nearest(const double *X, int64_t n, int d, const double *z, double *dmin)
{
    int64_t best = -1;
    double bd = 0.0;
    for (int64_t p = 0; p < n; ++p) {
        double D = oracle_sqdist(z, X + p * d, d);
        if (best < 0 || key_less(D, p, bd, best)) {
            best = p;
            bd = D;
        }
    }
    if (dmin)
        *dmin = bd;
    return best;
}

/* Cholesky factorisation K = L L^T, column by column (the classical
 * Cholesky-Crout order: column j is formed from the already finished columns
 * 0..j-1, inner sums in increasing index).  L overwrites the lower triangle
 * of the row-major k x k array K.  Returns 0, or -1 when a pivot is not
 * positive and finite (the matrix is not numerically positive definite). */
int oracle_cholesky(double *K, int k)
{
    for (int j = 0; j < k; ++j) {
        double s = K[j * k + j];
        for (int p = 0; p < j; ++p)
            s = s - K[j * k + p] * K[j * k + p];
        if (!(s > 0.0) || !isfinite(s))
            return -1;
        double ljj = sqrt(s);
        K[j * k + j] = ljj;
        for (int a = j + 1; a < k; ++a) {
            double t = K[a * k + j];
            for (int p = 0; p < j; ++p)
                t = t - K[a * k + p] * K[j * k + p];
            K[a * k + j] = t / ljj;
        }
    }
    return 0;
}

/* Solve L L^T c = y for one right-hand side (stride `stride` between the k
 * entries of y and c).  Forward substitution L w = y, then back substitution
 * L^T c = w, sums in increasing index. */
void oracle_cholesky_solve(const double *L, int k, const double *y, double *c, int stride)
{
    double *w = (double *)malloc(sizeof(double) * k);
    for (int a = 0; a < k; ++a) {
        double t = y[a * stride];
        for (int b = 0; b < a; ++b)
            t = t - L[a * k + b] * w[b];
        w[a] = t / L[a * k + a];
    }
    for (int a = k - 1; a >= 0; --a) {
        double t = w[a];
        for (int b = a + 1; b < k; ++b)
            t = t - L[b * k + a] * c[b * stride];
        c[a * stride] = t / L[a * k + a];
    }
    free(w);
}

/* Kernel matrix of a neighbourhood (Section 3, coefficient equation):
 * K_ab = phi(||x_a - x_b||) for a != b and K_aa = a + sigma^2, the nugget
 * keyed by index, never by a zero distance. */
void oracle_assemble(const double *X, int d, const int32_t *nb, int k, int kernel,
                     double nu, double rho, double noise, double amp, double *K)
{
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            if (a == b) {
                K[a * k + b] = amp + noise;
            } else {
                double D = oracle_sqdist(X + (int64_t)nb[a] * d, X + (int64_t)nb[b] * d, d);
                K[a * k + b] = oracle_phi(D, kernel, nu, rho, amp);
            }
        }
}

/* Offline training of FastMuyGPs (Algorithm 2; Section 3, coefficient
 * equation) for the training rows `rows[0..nrows-1]` (all rows when rows is
 * NULL, then nrows = n):
 *   N(i)  = neighbourhood of row i (LOO or SELF);
 *   C[i]  = K(X_N, X_N)^{-1} Y(X_N), one column per response.
 * Outputs: nb_out [nrows, k], C_out [nrows, k, ell], status_out [nrows]
 * (0 = ok, 1 = not positive definite: that C row is NaN, 2 = too few points).
 * Returns the number of rows with a non-zero status. */
int64_t oracle_build(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                     int kernel, double nu, double rho, double noise, double amp, int mode,
                     const int64_t *rows, int64_t nrows, int32_t *nb_out, double *C_out,
                     int32_t *status_out, int nthreads)
{
    int64_t bad = 0;
    if (!rows)
        nrows = n;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : bad)
#endif
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows ? rows[t] : t;
        int32_t *nb = nb_out + t * k;
        double *C = C_out + t * (int64_t)k * ell;
        double *K = (double *)malloc(sizeof(double) * k * k);
        double *yN = (double *)malloc(sizeof(double) * k * ell);
        int st = 0;
        if (oracle_neighborhood(X, n, d, i, k, mode, nb) != 0) {
            st = 2;
        } else {
            oracle_assemble(X, d, nb, k, kernel, nu, rho, noise, amp, K);
            if (oracle_cholesky(K, k) != 0) {
                st = 1;
            } else {
                for (int a = 0; a < k; ++a)
                    for (int c = 0; c < ell; ++c)
                        yN[a * ell + c] = Y[(int64_t)nb[a] * ell + c];
                for (int c = 0; c < ell; ++c)
                    oracle_cholesky_solve(K, k, yN + c, C + c, ell);
            }
        }
        if (st != 0) {
            for (int64_t e = 0; e < (int64_t)k * ell; ++e)
                C[e] = NAN;
            ++bad;
        }
        status_out[t] = st;
        free(K);
        free(yN);
    }
    return bad;
}

/* Nearest training point of every query (Algorithm 2, online loop). */
void oracle_nearest_batch(const double *X, int64_t n, int d, const double *Z, int64_t m,
                          int64_t *nn_out, double *dmin_out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t t = 0; t < m; ++t)
        nn_out[t] = oracle_nearest(X, n, d, Z + t * d, dmin_out ? dmin_out + t : NULL);
}

/* Posterior mean of query t (Section 3, prediction equation):
 *   mu(z)[c] = sum_s phi(||z - x_{N(j)_s}||) * C[j][s][c],
 * accumulated in s order, with the neighbourhood nb_j [k] and the
 * coefficient row C_j [k, ell] of the query's nearest training point j.
 * The cross-covariance carries no nugget. */
void oracle_mean(const double *X, int d, int ell, int k, int kernel, double nu, double rho,
                 double amp, const double *z, const int32_t *nb_j, const double *C_j,
                 double *out)
{
    for (int c = 0; c < ell; ++c)
        out[c] = 0.0;
    for (int s = 0; s < k; ++s) {
        double D = oracle_sqdist(z, X + (int64_t)nb_j[s] * d, d);
        double w = oracle_phi(D, kernel, nu, rho, amp);
        for (int c = 0; c < ell; ++c)
            out[c] = out[c] + w * C_j[s * ell + c];
    }
}

/* Means of m queries: query t uses neighbourhood row nb [t, k] and
 * coefficient row C [t, k, ell] (those of its nearest training point). */
void oracle_mean_batch(const double *X, int d, int ell, int k, int kernel, double nu, double rho,
                       double amp, const double *Z, int64_t m, const int32_t *nb,
                       const double *C, double *out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t t = 0; t < m; ++t)
        oracle_mean(X, d, ell, k, kernel, nu, rho, amp, Z + t * d, nb + t * k,
                    C + t * (int64_t)k * ell, out + t * ell);
}

/* MuyGPs prediction of a novel point (Section 2.1, MuyGPs prediction
 * equation):
 *   N*(z) = the k nearest training points of z, ties to the smaller index
 *           (z is not a training point, so nothing is excluded);
 *   mu(z) = K(z, X_N*) K(X_N*, X_N*)^{-1} Y(X_N*),
 * with the nugget on the diagonal of K(X_N*, X_N*) only (by index) and none on
 * the cross-covariance.  The solve is the same Cholesky as the training
 * loop's; the dot product is the same accumulation as oracle_mean.
 * Writes nb_out [k] and out [ell]; returns 0, 1 (not positive definite: out
 * is NaN) or 2 (fewer than k training points). */
int oracle_muygps_mean(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                       int kernel, double nu, double rho, double noise, double amp,
                       const double *z, int32_t *nb_out, double *out)
{
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * k);
    double *dist = (double *)malloc(sizeof(double) * k);
    double *K = (double *)malloc(sizeof(double) * k * k);
    double *yN = (double *)malloc(sizeof(double) * k * ell);
    double *w = (double *)malloc(sizeof(double) * k * ell);
    int st = 0;
    int64_t got = smallest_keys(X, n, d, z, -1, k, idx, dist);
    if (got != k) {
        st = 2;
    } else {
        for (int s = 0; s < k; ++s)
            nb_out[s] = (int32_t)idx[s];
        oracle_assemble(X, d, nb_out, k, kernel, nu, rho, noise, amp, K);
        if (oracle_cholesky(K, k) != 0) {
            st = 1;
        } else {
            for (int a = 0; a < k; ++a)
                for (int c = 0; c < ell; ++c)
                    yN[a * ell + c] = Y[(int64_t)nb_out[a] * ell + c];
            for (int c = 0; c < ell; ++c)
                oracle_cholesky_solve(K, k, yN + c, w + c, ell);
            oracle_mean(X, d, ell, k, kernel, nu, rho, amp, z, nb_out, w, out);
        }
    }
    if (st != 0)
        for (int c = 0; c < ell; ++c)
            out[c] = NAN;
    free(idx);
    free(dist);
    free(K);
    free(yN);
    free(w);
    return st;
}

/* MuyGPs predictions of m queries: nb_out [m, k], out [m, ell], status [m]. */
void oracle_muygps_batch(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                         int kernel, double nu, double rho, double noise, double amp,
                         const double *Z, int64_t m, int32_t *nb_out, double *out,
                         int32_t *status_out, int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
#endif
    for (int64_t t = 0; t < m; ++t)
        status_out[t] = oracle_muygps_mean(X, Y, n, d, ell, k, kernel, nu, rho, noise, amp,
                                           Z + t * d, nb_out + t * k, out + t * ell);
}

/* Derivative of the kernel value with respect to the length scale rho,
 * from the squared distance D (Section 2, Matern equation, half-integer
 * closed forms; RBF limit).  With s the scaled distance of oracle_phi:
 *   nu = 1/2 : dphi/drho = a s exp(-s) / rho            (s = r / rho)
 *   nu = 3/2 : dphi/drho = a s^2 exp(-s) / rho          (s = sqrt(3) r / rho)
 *   nu = 5/2 : dphi/drho = a s^2 (1 + s) exp(-s) / (3 rho)  (s = sqrt(5) r / rho)
 *   RBF      : dphi/drho = a exp(-D / (2 rho^2)) D / rho^3
 * (each is d/ds of the closed form times ds/drho = -s / rho).  NaN for an
 * unsupported nu. */
double oracle_dphi_drho(double D, int kernel, double nu, double rho, double amp)
{
    if (kernel == ORACLE_RBF)
        return amp * exp(-D / (2.0 * rho * rho)) * D / (rho * rho * rho);
    double r = sqrt(D);
    if (nu == 0.5) {
        double s = r / rho;
        return amp * s * exp(-s) / rho;
    }
    if (nu == 1.5) {
        double s = sqrt(3.0) * r / rho;
        return amp * s * s * exp(-s) / rho;
    }
    if (nu == 2.5) {
        double s = sqrt(5.0) * r / rho;
        return amp * s * s * (1.0 + s) * exp(-s) / (3.0 * rho);
    }
    return NAN;
}

/* Leave-one-out loss of MuyGPs hyperparameter training and its gradient
 * (Algorithm 1; Section 2.1, leave-one-out prediction and loss Q(theta)).
 * For batch row t (training point i = rows[t], leave-one-out neighbourhood
 * N(i) of the k nearest other points):
 *   K      = K(X_N, X_N) + sigma^2 I,   kz = K(x_i, X_N)  (no nugget),
 *   mu_c   = kz K^{-1} Y_N[:, c],       e_c = mu_c - y_{i,c},
 *   loss_t = sum_c e_c^2,
 * and, for theta in {rho, sigma^2}, with dK^{-1} = -K^{-1} dK K^{-1},
 *   dmu_c  = dkz K^{-1} Y_N[:, c] - kz K^{-1} dK K^{-1} Y_N[:, c],
 *   g_t    = sum_c 2 e_c dmu_c,
 * where dK/drho holds dphi/drho off the diagonal (the diagonal a + sigma^2
 * does not depend on rho), dK/dsigma^2 = I, dkz/drho = dphi/drho and
 * dkz/dsigma^2 = 0.  Writes terms [nrows, 3] = (loss_t, g_rho, g_sigma2),
 * unnormalised (Q = sum loss_t / (nrows ell), likewise its gradient), and
 * status [nrows] (0 ok, 1 not positive definite: terms NaN, 2 too few
 * points).  Returns the number of rows with a non-zero status. */
int64_t oracle_loo_loss_grad(const double *X, const double *Y, int64_t n, int d, int ell, int k,
                             int kernel, double nu, double rho, double noise, double amp,
                             const int64_t *rows, int64_t nrows, double *terms,
                             int32_t *status_out, int nthreads)
{
    int64_t bad = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : bad)
#endif
    for (int64_t t = 0; t < nrows; ++t) {
        int64_t i = rows[t];
        int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * k);
        double *K = (double *)malloc(sizeof(double) * k * k);
        double *dK = (double *)malloc(sizeof(double) * k * k);
        double *kz = (double *)malloc(sizeof(double) * k);
        double *dkz = (double *)malloc(sizeof(double) * k);
        double *yN = (double *)malloc(sizeof(double) * k);
        double *alpha = (double *)malloc(sizeof(double) * k);
        double *w = (double *)malloc(sizeof(double) * k);
        double *u = (double *)malloc(sizeof(double) * k);
        int st = 0;
        double loss = 0.0, g_rho = 0.0, g_s2 = 0.0;
        if (oracle_neighborhood(X, n, d, i, k, ORACLE_MODE_LOO, nb) != 0) {
            st = 2;
        } else {
            oracle_assemble(X, d, nb, k, kernel, nu, rho, noise, amp, K);
            for (int a = 0; a < k; ++a) {
                for (int b = 0; b < k; ++b) {
                    double D = oracle_sqdist(X + (int64_t)nb[a] * d, X + (int64_t)nb[b] * d, d);
                    dK[a * k + b] = (a == b) ? 0.0 : oracle_dphi_drho(D, kernel, nu, rho, amp);
                }
                double Dz = oracle_sqdist(X + i * d, X + (int64_t)nb[a] * d, d);
                kz[a] = oracle_phi(Dz, kernel, nu, rho, amp);
                dkz[a] = oracle_dphi_drho(Dz, kernel, nu, rho, amp);
            }
            if (oracle_cholesky(K, k) != 0) {
                st = 1;
            } else {
                for (int c = 0; c < ell; ++c) {
                    for (int a = 0; a < k; ++a)
                        yN[a] = Y[(int64_t)nb[a] * ell + c];
                    oracle_cholesky_solve(K, k, yN, alpha, 1);
                    double mu = 0.0;
                    for (int a = 0; a < k; ++a)
                        mu = mu + kz[a] * alpha[a];
                    double e = mu - Y[i * ell + c];
                    loss = loss + e * e;
                    /* rho: dkz alpha - kz K^{-1} (dK alpha) */
                    for (int a = 0; a < k; ++a) {
                        double s = 0.0;
                        for (int b = 0; b < k; ++b)
                            s = s + dK[a * k + b] * alpha[b];
                        w[a] = s;
                    }
                    oracle_cholesky_solve(K, k, w, u, 1);
                    double dmu = 0.0;
                    for (int a = 0; a < k; ++a)
                        dmu = dmu + dkz[a] * alpha[a] - kz[a] * u[a];
                    g_rho = g_rho + 2.0 * e * dmu;
                    /* sigma^2: dK = I, so dmu = -kz K^{-1} alpha */
                    oracle_cholesky_solve(K, k, alpha, u, 1);
                    double dmu_s = 0.0;
                    for (int a = 0; a < k; ++a)
                        dmu_s = dmu_s - kz[a] * u[a];
                    g_s2 = g_s2 + 2.0 * e * dmu_s;
                }
            }
        }
        if (st != 0) {
            loss = NAN;
            g_rho = NAN;
            g_s2 = NAN;
            ++bad;
        }
        terms[t * 3 + 0] = loss;
        terms[t * 3 + 1] = g_rho;
        terms[t * 3 + 2] = g_s2;
        status_out[t] = st;
        free(nb);
        free(K);
        free(dK);
        free(kz);
        free(dkz);
        free(yN);
        free(alpha);
        free(w);
        free(u);
    }
    return bad;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
