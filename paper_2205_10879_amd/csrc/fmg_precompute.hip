// Coefficient precompute (Algorithm 2, training loop; Section 3, coefficient
// equation): for every training point i
//     K_ab = phi(||x_{N(i)_a} - x_{N(i)_b}||)  (a != b),   K_aa = amp + sigma^2,
//     C[i] = K^{-1} Y(X_{N(i)}).
// One wavefront per training point; lane a owns row a of K (k <= 64).
//   1. the k neighbour rows are staged in LDS (row stride d+1 against bank
//      conflicts); lane a forms its kernel row in registers;
//   2. right-looking Cholesky in registers: at step j the pivot comes from
//      lane j, column j of L is broadcast through LDS and every lane applies
//      its rank-1 update;
//   3. the factor is written to LDS and both triangular solves run column by
//      column, all ell right-hand sides at once;
//   4. MIXED precision only: one refinement step, r = Y_N - (K64 + sigma^2 I) C
//      with the kernel matrix re-evaluated in FP64 from the inputs, then
//      C += solve(L, r) with the FP32 factor.
// A non-positive or non-finite pivot marks the row as not positive definite:
// its C row is NaN and its status is 1.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int lane);
template <>
__device__ __forceinline__ float readlane_t<float>(float v, int lane) {
    return readlane_f32(v, lane);
}
template <>
__device__ __forceinline__ double readlane_t<double>(double v, int lane) {
    return readlane_f64(v, lane);
}

// Solve L L^T x = y in place for ELLMAX right-hand sides held one row per
// lane (y[c] of lane a is row a of column c).  L is in LDS, row stride ls.
template <typename T, int ELLMAX>
__device__ __forceinline__ void chol_solve(const T *__restrict__ Lm, int ls, int k, int ell, int a,
                                           T (&y)[ELLMAX]) {
    for (int j = 0; j < k; ++j) {
        const T ljj = Lm[j * ls + j];
        const T laj = (a > j && a < k) ? Lm[a * ls + j] : T(0);
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c < ell) {
                const T wj = readlane_t<T>(y[c], j) / ljj;
                if (a == j) y[c] = wj;
                else if (a > j) y[c] -= laj * wj;
            }
        }
    }
    for (int j = k - 1; j >= 0; --j) {
        const T ljj = Lm[j * ls + j];
        const T lja = (a < j) ? Lm[j * ls + a] : T(0);
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            if (c < ell) {
                const T cj = readlane_t<T>(y[c], j) / ljj;
                if (a == j) y[c] = cj;
                else if (a < j) y[c] -= lja * cj;
            }
        }
    }
}

template <typename T, int KMAX, int ELLMAX, bool REFINE>
__global__ __launch_bounds__(64) void precompute_kernel(PrecomputeArgs P) {
    extern __shared__ __align__(16) char smem[];
    const int64_t i = blockIdx.x;
    if (i >= P.n) return;
    const int a = threadIdx.x;
    const int k = P.k, d = P.d, ell = P.ell;
    const int xs_ld = d + 1, ls = k + 1;
    T *xs = (T *)smem;                 // [k, d+1]
    T *Lm = xs + k * xs_ld;            // [k, k+1]
    T *cb = Lm + k * ls;               // [64]
    float *cbuf = (float *)(cb + 64);  // [64, ELLMAX] (refinement)

    const T *__restrict__ X = (const T *)P.X;
    const T *__restrict__ Y = (const T *)P.Y;
    const int64_t p = (a < k) ? (int64_t)P.N[i * k + a] : 0;
    if (a < k)
        for (int c = 0; c < d; ++c) xs[a * xs_ld + c] = X[p * d + c];
    __syncthreads();

    const T inv_rho = (T)P.inv_rho, amp = (T)P.amp, diag = (T)(P.amp + P.noise);
    T K[KMAX];
#pragma unroll
    for (int b = 0; b < KMAX; ++b) {
        T v = T(0);
        if (b < k) {
            T D = T(0);
            if (a < k) {
                for (int c = 0; c < d; ++c) {
                    const T t = xs[a * xs_ld + c] - xs[b * xs_ld + c];
                    D += t * t;
                }
            }
            v = (a == b) ? diag : phi_t<T>(D, P.kc, inv_rho, amp);
        }
        K[b] = v;
    }

    // Cholesky, right-looking, column j broadcast through LDS.
    bool bad = false;
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
        if (j < k) {
            T piv = readlane_t<T>(K[j], j);
            if (!(piv > T(0)) || !isfinite((double)piv)) {
                bad = true;
                piv = T(1);
            }
            const T ljj = sqrt(piv);
            const T inv = T(1) / ljj;
            const T lj = (a == j) ? ljj : K[j] * inv;
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
#pragma unroll
        for (int b = 0; b < KMAX; ++b)
            if (b < k) Lm[a * ls + b] = K[b];
    }
    __syncthreads();

    T y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? Y[p * ell + c] : T(0);
    chol_solve<T, ELLMAX>(Lm, ls, k, ell, a, y);

    if constexpr (REFINE) {
        // r = Y_N - (K64 + sigma^2 I) C with K64 from the FP64 distances of the
        // inputs, then one correction solve with the FP32 factor.
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            if (c < ell) cbuf[a * ELLMAX + c] = (float)y[c];
        __syncthreads();
        double r[ELLMAX];
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            r[c] = (a < k && c < ell) ? (double)Y[p * ell + c] : 0.0;
        if (a < k) {
            for (int b = 0; b < k; ++b) {
                double kab;
                if (b == a) {
                    kab = P.amp + P.noise;
                } else {
                    double D = 0.0;
                    for (int c = 0; c < d; ++c) {
                        const double t = (double)xs[a * xs_ld + c] - (double)xs[b * xs_ld + c];
                        D = fma(t, t, D);
                    }
                    kab = phi64(D, P.kc, P.inv_rho, P.amp);
                }
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c)
                    if (c < ell) r[c] = fma(-kab, (double)cbuf[b * ELLMAX + c], r[c]);
            }
        }
        T dl[ELLMAX];
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) dl[c] = (T)r[c];
        chol_solve<T, ELLMAX>(Lm, ls, k, ell, a, dl);
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) y[c] += dl[c];
    }

    if (a < k) {
        T *__restrict__ C = (T *)P.C + (i * k + a) * ell;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            if (c < ell) C[c] = bad ? (T)NAN : y[c];
    }
    if (a == 0) P.status[i] = bad ? 1 : 0;
}

template <typename T, int KMAX, int ELLMAX, bool REFINE>
hipError_t launch_pc(const PrecomputeArgs &a, hipStream_t s) {
    size_t shm = sizeof(T) * ((size_t)a.k * (a.d + 1) + (size_t)a.k * (a.k + 1) + 64);
    if (REFINE) shm += sizeof(float) * 64 * ELLMAX;
    shm = (shm + 15) & ~(size_t)15;
    hipLaunchKernelGGL((precompute_kernel<T, KMAX, ELLMAX, REFINE>), dim3((unsigned)a.n),
                       dim3(64), shm, s, a);
    return hipGetLastError();
}

template <typename T, bool REFINE>
hipError_t launch_pc_k(const PrecomputeArgs &a, hipStream_t s) {
    if (a.ell > 16) return hipErrorInvalidValue;
    if (a.k <= 32) {
        if (a.ell <= 1) return launch_pc<T, 32, 1, REFINE>(a, s);
        return launch_pc<T, 32, 16, REFINE>(a, s);
    }
    if (a.ell <= 1) return launch_pc<T, 64, 1, REFINE>(a, s);
    return launch_pc<T, 64, 16, REFINE>(a, s);
}

}  // namespace

hipError_t launch_precompute(bool f64, bool refine, const PrecomputeArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (a.k > 64) return launch_precompute_wide(f64, a, s);
    if (f64) return launch_pc_k<double, false>(a, s);
    return launch_precompute32(refine, a, s);
}

}  // namespace fmg
