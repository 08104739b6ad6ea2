// Gradient of the leave-one-out loss of MuyGPs hyperparameter training
// (Algorithm 1; Section 2.1, loss Q(theta)) with respect to the length scale
// rho and the noise variance sigma^2.  It runs in FP64 whatever the model
// precision (FP32 inputs are widened exactly), so that an optimiser sees a
// smooth objective.
//
// For batch point i with the model's leave-one-out neighbourhood N:
//   K = K(X_N, X_N) + sigma^2 I,   kz = K(x_i, X_N)  (no nugget),
//   alpha = K^{-1} Y_N,  mu_c = kz . alpha_c,  e_c = mu_c - y_{i,c}.
// Since dK^{-1} = -K^{-1} dK K^{-1} and K is symmetric,
//   d mu_c = dkz . alpha_c - beta^T dK alpha_c,   beta = K^{-1} kz,
// so with v = sum_c e_c alpha_c (one value per neighbour)
//   d(sum_c e_c^2)/drho     = 2 (dkz . v - beta . (dK v)),
//   d(sum_c e_c^2)/dsigma^2 = -2 beta . v            (dK/dsigma^2 = I),
// where dK/drho holds dphi/drho off the diagonal.
//
// One wavefront per batch point; lane a owns neighbour a (k <= 64):
//   1. the k neighbour rows and x_i are staged in LDS;
//   2. lane a forms row a of K, and its entries of kz and dkz;
//   3. right-looking Cholesky in registers (pivot j from lane j, column j
//      broadcast through LDS); the factor is stored packed in LDS;
//   4. forward and back substitution for the ell columns of Y_N and for kz
//      together;
//   5. predictions and errors from wave sums, then the two contractions
//      (dK v re-formed from the staged rows).
// Per-point terms (sum_c e_c^2, d/drho, d/dsigma^2) go to `terms`; a
// deterministic two-pass column sum follows.  A non-positive or non-finite
// pivot makes the point's terms NaN.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

// Kernel value phi and its derivative in rho, from the squared distance D;
// the value uses the same closed forms as phi64.  With s the scaled
// distance, d/drho = d/ds * ds/drho and ds/drho = -s / rho.
__device__ __forceinline__ double phi_drho64(double D, int kc, double inv_rho, double amp,
                                             double &dphi) {
    if (kc == KC_RBF) {
        const double v = amp * exp(-0.5 * D * inv_rho * inv_rho);
        dphi = v * D * inv_rho * inv_rho * inv_rho;
        return v;
    }
    const double r = sqrt(D);
    if (kc == KC_M12) {
        const double s = r * inv_rho, e = exp(-s);
        dphi = amp * s * e * inv_rho;
        return amp * e;
    }
    if (kc == KC_M32) {
        const double s = 1.7320508075688772 * r * inv_rho, e = exp(-s);
        dphi = amp * s * s * e * inv_rho;
        return amp * (1.0 + s) * e;
    }
    const double s = 2.2360679774997896 * r * inv_rho, e = exp(-s);
    dphi = amp * s * s * (1.0 + s) * e * inv_rho * (1.0 / 3.0);
    return amp * (1.0 + s + s * s * (1.0 / 3.0)) * e;
}

__device__ __forceinline__ double lds_sqdist(const double *__restrict__ u,
                                             const double *__restrict__ w, int d) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
        const double t = u[c] - w[c];
        s = fma(t, t, s);
    }
    return s;
}

__host__ __device__ __forceinline__ size_t grad_lds_doubles(int k, int d) {
    return (size_t)(k + 1) * (d + 1) + (size_t)k * (k + 1) / 2 + 128;
}

template <typename TI, int KMAX, int ELLMAX>
__global__ __launch_bounds__(64) void loo_grad_kernel(GradArgs P) {
    extern __shared__ __align__(16) char smem[];
    const int64_t t = blockIdx.x;
    if (t >= P.b) return;
    const int a = threadIdx.x;
    const int k = P.k, d = P.d, ell = P.ell;
    const int xs_ld = d + 1;
    double *xs = (double *)smem;          // [k + 1, d + 1]; row k is x_i
    double *Lp = xs + (k + 1) * xs_ld;    // packed factor: row a at a (a + 1) / 2
    double *cb = Lp + k * (k + 1) / 2;    // [64] column broadcast
    double *vs = cb + 64;                 // [64] v broadcast
    const TI *__restrict__ X = (const TI *)P.X;
    const TI *__restrict__ Y = (const TI *)P.Y;

    const int64_t i = P.rows[t];
    if (i < 0 || i >= P.n) {
        if (a == 0) {
            atomicOr(P.bad, 1);
            P.terms[t * 3 + 0] = NAN;
            P.terms[t * 3 + 1] = NAN;
            P.terms[t * 3 + 2] = NAN;
        }
        return;
    }
    const int64_t p = (a < k) ? (int64_t)P.N[i * k + a] : 0;
    if (a < k)
        for (int c = 0; c < d; ++c) xs[a * xs_ld + c] = (double)X[p * d + c];
    for (int c = a; c < d; c += 64) xs[k * xs_ld + c] = (double)X[i * d + c];
    __syncthreads();

    const double *xa = xs + (a < k ? a : 0) * xs_ld;
    double kz = 0.0, dkz = 0.0;
    if (a < k) kz = phi_drho64(lds_sqdist(xa, xs + k * xs_ld, d), P.kc, P.inv_rho, P.amp, dkz);
    const double diag = P.amp + P.noise;
    double K[KMAX];
#pragma unroll
    for (int b = 0; b < KMAX; ++b) {
        double v = (a == b) ? 1.0 : 0.0;
        if (a < k && b < k)
            v = (a == b) ? diag : phi64(lds_sqdist(xa, xs + b * xs_ld, d), P.kc, P.inv_rho, P.amp);
        K[b] = v;
    }

    // Cholesky: after step j lane a > j holds L_aj in K[j]; lane j holds
    // L_jj.  Lanes at or past k carry identity rows and stay untouched.
    bool bad = false;
    double inv_own = 1.0;  // 1 / L_aa of this lane
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
            double piv = readlane_f64(K[j], j);
            if (!(piv > 0.0) || !isfinite(piv)) {
                bad = true;
                piv = 1.0;
            }
            const double ljj = sqrt(piv);
            const double inv = 1.0 / ljj;
            const double lj = (a == j) ? ljj : K[j] * inv;
            if (a == j) inv_own = inv;
            K[j] = lj;
            cb[a] = lj;
            __syncthreads();
#pragma unroll
            for (int b = j + 1; b < KMAX; ++b)
                if (b < k) K[b] -= lj * cb[b];
            __syncthreads();
        }
    }
    if (a < k) {
        const int row = a * (a + 1) / 2;
#pragma unroll
        for (int b = 0; b < KMAX; ++b)
            if (b <= a) Lp[row + b] = K[b];
    }
    __syncthreads();

    // Right-hand sides: the ell columns of Y_N, and kz (for beta).
    double y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? (double)Y[p * ell + c] : 0.0;
    double yb = kz;
    const double *Lrow = Lp + (a < k ? a * (a + 1) / 2 : 0);
    for (int j = 0; j < k; ++j) {  // L w = y
        const double ij = readlane_f64(inv_own, j);
        const double laj = (a > j && a < k) ? Lrow[j] : 0.0;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c < ell) {
                const double wj = readlane_f64(y[c], j) * ij;
                y[c] = (a == j) ? wj : y[c] - laj * wj;
            }
        }
        const double wj = readlane_f64(yb, j) * ij;
        yb = (a == j) ? wj : yb - laj * wj;
    }
    for (int j = k - 1; j >= 0; --j) {  // L^T x = w
        const double ij = readlane_f64(inv_own, j);
        const double lja = (a < j) ? Lp[j * (j + 1) / 2 + a] : 0.0;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c < ell) {
                const double xj = readlane_f64(y[c], j) * ij;
                y[c] = (a == j) ? xj : y[c] - lja * xj;
            }
        }
        const double xj = readlane_f64(yb, j) * ij;
        yb = (a == j) ? xj : yb - lja * xj;
    }
    // Lanes at or past k hold zeros in y and yb: their right-hand sides are
    // zero and no update reaches them (their factor entries are zero).

    double loss = 0.0, v = 0.0;
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) {
        if (c < ell) {
            const double mu = wave_sum_f64(kz * y[c]);
            const double e = mu - (double)Y[i * ell + c];
            loss += e * e;
            v += e * y[c];
        }
    }
    const double g_s2 = -2.0 * wave_sum_f64(yb * v);
    vs[a] = v;
    __syncthreads();
    double w = 0.0;  // (dK v)_a
    if (a < k) {
        for (int b = 0; b < k; ++b) {
            if (b == a) continue;
            double dk;
            phi_drho64(lds_sqdist(xa, xs + b * xs_ld, d), P.kc, P.inv_rho, P.amp, dk);
            w = fma(dk, vs[b], w);
        }
    }
    const double g_rho = 2.0 * wave_sum_f64(dkz * v - yb * w);
    if (a == 0) {
        P.terms[t * 3 + 0] = bad ? NAN : loss;
        P.terms[t * 3 + 1] = bad ? NAN : g_rho;
        P.terms[t * 3 + 2] = bad ? NAN : g_s2;
    }
}

// Column sums of terms [b, 3]: fixed-order per-block partials, then one
// block adds the partials in a fixed order (deterministic).
__global__ __launch_bounds__(256) void terms_partial_kernel(const double *__restrict__ terms,
                                                            int64_t b, double *__restrict__ part) {
    __shared__ double sh[3][256];
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + t; r < b; r += (int64_t)gridDim.x * 256) {
        s0 += terms[r * 3 + 0];
        s1 += terms[r * 3 + 1];
        s2 += terms[r * 3 + 2];
    }
    sh[0][t] = s0;
    sh[1][t] = s1;
    sh[2][t] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
            sh[2][t] += sh[2][t + w];
        }
        __syncthreads();
    }
    if (t < 3) part[blockIdx.x * 3 + t] = sh[t][0];
}

__global__ __launch_bounds__(256) void terms_final_kernel(const double *__restrict__ part, int nb,
                                                          double *__restrict__ out) {
    __shared__ double sh[3][256];
    const int t = threadIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = t; q < nb; q += 256) {
        s0 += part[q * 3 + 0];
        s1 += part[q * 3 + 1];
        s2 += part[q * 3 + 2];
    }
    sh[0][t] = s0;
    sh[1][t] = s1;
    sh[2][t] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
            sh[2][t] += sh[2][t + w];
        }
        __syncthreads();
    }
    if (t < 3) out[t] = sh[t][0];
}

template <typename TI, int KMAX, int ELLMAX>
hipError_t launch_grad_t(const GradArgs &a, hipStream_t s) {
    const size_t shm = grad_lds_doubles(a.k, a.d) * sizeof(double);
    hipLaunchKernelGGL((loo_grad_kernel<TI, KMAX, ELLMAX>), dim3((unsigned)a.b), dim3(64), shm, s,
                       a);
    return hipGetLastError();
}

template <typename TI>
hipError_t launch_grad_k(const GradArgs &a, hipStream_t s) {
    if (a.k <= 32) {
        if (a.ell <= 4) return launch_grad_t<TI, 32, 4>(a, s);
        return launch_grad_t<TI, 32, 16>(a, s);
    }
    if (a.ell <= 4) return launch_grad_t<TI, 64, 4>(a, s);
    return launch_grad_t<TI, 64, 16>(a, s);
}

}  // namespace

size_t loo_grad_lds_bytes(int k, int d) { return grad_lds_doubles(k, d) * sizeof(double); }

int loo_grad_blocks(int64_t b) {
    const int64_t nb = (b + 255) / 256;
    return (int)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb));
}

hipError_t launch_loo_grad(bool f64, const GradArgs &a, double *part, double *out,
                           hipStream_t s) {
    if (a.b <= 0) return hipSuccess;
    if (a.k < 1 || a.k > 64 || a.ell < 1 || a.ell > 16 || a.d < 1 ||
        loo_grad_lds_bytes(a.k, a.d) > 65536)
        return hipErrorInvalidValue;
    const hipError_t e = f64 ? launch_grad_k<double>(a, s) : launch_grad_k<float>(a, s);
    if (e != hipSuccess) return e;
    const int nb = loo_grad_blocks(a.b);
    hipLaunchKernelGGL(terms_partial_kernel, dim3(nb), dim3(256), 0, s, (const double *)a.terms,
                       a.b, part);
    hipLaunchKernelGGL(terms_final_kernel, dim3(1), dim3(256), 0, s, (const double *)part, nb,
                       out);
    return hipGetLastError();
}

}  // namespace fmg
