// Leave-one-out loss of MuyGPs hyperparameter training (Algorithm 1; Section
// 2.1, loss Q(theta)): helpers that gather a batch of training rows and
// reduce the squared errors of their leave-one-out predictions.  The
// neighbour lists do not depend on theta (the kernels are isotropic, so the
// ranking is by distance alone); the coefficient rows are solved again by
// the precompute kernel and the predictions formed by the gather kernel.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

// Batch row t: X row, neighbour list and response row of training point
// rows[t]; an index outside [0, n) sets *bad and yields zero rows.
template <typename T>
__global__ __launch_bounds__(256) void batch_rows_kernel(const T *__restrict__ X,
                                                         const int32_t *__restrict__ N,
                                                         const T *__restrict__ Y,
                                                         const int32_t *__restrict__ rows,
                                                         int64_t b, int64_t n, int d, int k,
                                                         int ell, T *__restrict__ Xb,
                                                         int32_t *__restrict__ Nb,
                                                         T *__restrict__ Yb, int *bad) {
    const int64_t t = (int64_t)blockIdx.x;
    if (t >= b) return;
    const int64_t i = rows[t];
    const bool ok = i >= 0 && i < n;
    if (!ok && threadIdx.x == 0) atomicOr(bad, 1);
    for (int c = threadIdx.x; c < d; c += blockDim.x) Xb[t * d + c] = ok ? X[i * d + c] : T(0);
    for (int s = threadIdx.x; s < k; s += blockDim.x) Nb[t * k + s] = ok ? N[i * k + s] : 0;
    for (int c = threadIdx.x; c < ell; c += blockDim.x) Yb[t * ell + c] = ok ? Y[i * ell + c] : T(0);
}

// Sum of (Y - mu)^2 over `count` values: fixed-order per-block partials,
// then one block adds the partials in a fixed order (deterministic).
template <typename T>
__global__ __launch_bounds__(256) void sq_err_partial_kernel(const T *__restrict__ Y,
                                                             const T *__restrict__ mu,
                                                             int64_t count,
                                                             double *__restrict__ part) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + t; e < count; e += (int64_t)gridDim.x * 256) {
        const double r = (double)Y[e] - (double)mu[e];
        s += r * r;
    }
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void sum_kernel(const double *__restrict__ part, int nb,
                                                  double *__restrict__ out) {
    __shared__ double sh[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int b = t; b < nb; b += 256) s += part[b];
    sh[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) *out = sh[0];
}

}  // namespace

hipError_t launch_batch_rows(bool f64, const void *X, const int32_t *N, const void *Y,
                             const int32_t *rows, int64_t b, int64_t n, int d, int k, int ell,
                             void *Xb, int32_t *Nb, void *Yb, int *bad, hipStream_t s) {
    if (b <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(batch_rows_kernel<double>, dim3((unsigned)b), dim3(64), 0, s,
                           (const double *)X, N, (const double *)Y, rows, b, n, d, k, ell,
                           (double *)Xb, Nb, (double *)Yb, bad);
    else
        hipLaunchKernelGGL(batch_rows_kernel<float>, dim3((unsigned)b), dim3(64), 0, s,
                           (const float *)X, N, (const float *)Y, rows, b, n, d, k, ell,
                           (float *)Xb, Nb, (float *)Yb, bad);
    return hipGetLastError();
}

int sq_err_blocks(int64_t count) {
    const int64_t nb = (count + 255) / 256;
    return (int)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb));
}

hipError_t launch_sq_err(bool f64, const void *Y, const void *mu, int64_t count, double *part,
                         double *out, hipStream_t s) {
    const int nb = sq_err_blocks(count);
    if (f64)
        hipLaunchKernelGGL(sq_err_partial_kernel<double>, dim3(nb), dim3(256), 0, s,
                           (const double *)Y, (const double *)mu, count, part);
    else
        hipLaunchKernelGGL(sq_err_partial_kernel<float>, dim3(nb), dim3(256), 0, s,
                           (const float *)Y, (const float *)mu, count, part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, (const double *)part, nb, out);
    return hipGetLastError();
}

}  // namespace fmg
