// Coefficient precompute for neighbourhoods wider than a wavefront
// (64 < k <= 256; Algorithm 2, training loop; Section 3, coefficient
// equation): for every training point i
//     K_ab = phi(||x_{N(i)_a} - x_{N(i)_b}||)  (a != b),   K_aa = amp + sigma^2,
//     C[i] = K^{-1} Y(X_{N(i)}),
// in the model's precision T (FP64 or FP32).  One workgroup of 1024 threads
// per training point (the packed factor leaves room for one or two
// workgroups per CU, so the workgroup itself supplies the waves that hide
// LDS latency); K lives in LDS as a packed lower triangle (row a at
// a (a + 1) / 2), so k = 150 in FP64 takes 90 KB:
//   1. the k neighbour rows are staged in LDS;
//   2. assembly over a 32 x 32 thread grid (thread (ty, tx) takes rows
//      ty + 32 r and columns tx + 32 s of the lower triangle);
//   3. right-looking Cholesky: at step j every thread reads the pivot,
//      thread a > j scales its entry of column j, and the trailing update
//      is spread over the same 32 x 32 grid (two barriers per step);
//   4. forward and back substitution, thread a owning row a of all ell
//      right-hand sides, the solved entry broadcast through LDS (double
//      buffered, one barrier per step).
// A non-positive or non-finite pivot marks the row as not positive definite:
// its C row is NaN and its status is 1.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

constexpr int WIDE_THREADS = 1024;
constexpr int WIDE_KMAX = 256;  // rows of the column and diagonal buffers
constexpr int GRID = 32;        // the thread grid is GRID x GRID

template <typename T>
__device__ __forceinline__ T sqdist_rows(const T *__restrict__ u, const T *__restrict__ v, int d) {
    T s = T(0);
    for (int c = 0; c < d; ++c) {
        const T t = u[c] - v[c];
        s += t * t;
    }
    return s;
}

__host__ __device__ __forceinline__ size_t wide_lds_elems(int k, int d, int ellmax) {
    return (size_t)k * (d + 1) + (size_t)k * (k + 1) / 2 + 2 * WIDE_KMAX + 2 * (size_t)ellmax;
}

template <typename T, int ELLMAX>
__global__ __launch_bounds__(WIDE_THREADS) void precompute_wide_kernel(PrecomputeArgs P) {
    extern __shared__ __align__(16) char smem[];
    const int64_t i = blockIdx.x;
    if (i >= P.n) return;
    const int a = threadIdx.x;  // row owned in the column steps and the solves
    const int ty = a / GRID, tx = a % GRID;
    const int k = P.k, d = P.d, ell = P.ell;
    const int xs_ld = d + 1;
    T *xs = (T *)smem;                          // [k, d + 1]
    T *A = xs + (size_t)k * xs_ld;              // packed lower triangle
    T *col = A + (size_t)k * (k + 1) / 2;       // [256] column j of L
    T *dg = col + WIDE_KMAX;                    // [256] L_jj
    T *bc = dg + WIDE_KMAX;                     // [2][ELLMAX] solve broadcast
    const T *__restrict__ X = (const T *)P.X;
    const T *__restrict__ Y = (const T *)P.Y;

    int64_t p = 0;
    if (a < k) {
        p = (int64_t)P.N[i * k + a];
        for (int c = 0; c < d; ++c) xs[a * xs_ld + c] = X[p * d + c];
    }
    __syncthreads();

    const T inv_rho = (T)P.inv_rho, amp = (T)P.amp, diag = (T)(P.amp + P.noise);
    for (int r = ty; r < k; r += GRID) {
        const size_t row = (size_t)r * (r + 1) / 2;
        for (int b = tx; b <= r; b += GRID)
            A[row + b] = (b == r) ? diag
                                  : phi_t<T>(sqdist_rows(xs + r * xs_ld, xs + b * xs_ld, d), P.kc,
                                             inv_rho, amp);
    }
    __syncthreads();

    bool bad = false;
    const size_t arow = (size_t)a * (a + 1) / 2;
    for (int j = 0; j < k; ++j) {
        const T piv = A[(size_t)j * (j + 1) / 2 + j];
        const bool ok = piv > T(0) && isfinite((double)piv);
        bad = bad || !ok;
        const T ljj = ok ? (T)sqrt(piv) : T(1);
        if (a == j) dg[j] = ljj;
        if (a > j && a < k) {
            const T l = A[arow + j] / ljj;
            A[arow + j] = l;
            col[a] = l;
        }
        __syncthreads();
        for (int r = j + 1 + ty; r < k; r += GRID) {
            const T lr = col[r];
            const size_t row = (size_t)r * (r + 1) / 2;
            for (int b = j + 1 + tx; b <= r; b += GRID) A[row + b] -= lr * col[b];
        }
        __syncthreads();
    }

    T y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? Y[p * ell + c] : T(0);
    for (int j = 0; j < k; ++j) {  // L w = y
        T *buf = bc + (j & 1) * ELLMAX;
        if (a == j) {
            const T ljj = dg[j];
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c) {
                y[c] = y[c] / ljj;
                buf[c] = y[c];
            }
        }
        __syncthreads();
        if (a > j && a < k) {
            const T l = A[arow + j];
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c) y[c] -= l * buf[c];
        }
    }
    __syncthreads();
    for (int j = k - 1; j >= 0; --j) {  // L^T x = w
        T *buf = bc + (j & 1) * ELLMAX;
        if (a == j) {
            const T ljj = dg[j];
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c) {
                y[c] = y[c] / ljj;
                buf[c] = y[c];
            }
        }
        __syncthreads();
        if (a < j) {
            const T l = A[(size_t)j * (j + 1) / 2 + a];
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c) y[c] -= l * buf[c];
        }
    }

    if (a < k) {
        T *__restrict__ C = (T *)P.C + (i * k + a) * ell;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c)
            if (c < ell) C[c] = bad ? (T)NAN : y[c];
    }
    if (a == 0) P.status[i] = bad ? 1 : 0;
}

template <typename T, int ELLMAX>
hipError_t launch_wide_t(const PrecomputeArgs &a, hipStream_t s) {
    const size_t shm = wide_lds_elems(a.k, a.d, ELLMAX) * sizeof(T);
    const hipError_t e = hipFuncSetAttribute((const void *)precompute_wide_kernel<T, ELLMAX>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((precompute_wide_kernel<T, ELLMAX>), dim3((unsigned)a.n),
                       dim3(WIDE_THREADS), shm, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_wide_e(const PrecomputeArgs &a, hipStream_t s) {
    if (a.ell <= 1) return launch_wide_t<T, 1>(a, s);
    if (a.ell <= 4) return launch_wide_t<T, 4>(a, s);
    return launch_wide_t<T, 16>(a, s);
}

}  // namespace

size_t precompute_wide_lds_bytes(bool f64, int k, int d) {
    return wide_lds_elems(k, d, 16) * (f64 ? 8 : 4);
}

hipError_t launch_precompute_wide(bool f64, const PrecomputeArgs &a, hipStream_t s) {
    if (a.n <= 0) return hipSuccess;
    if (a.k < 1 || a.k > WIDE_KMAX || a.ell < 1 || a.ell > 16 ||
        precompute_wide_lds_bytes(f64, a.k, a.d) > PRECOMPUTE_WIDE_LDS_MAX)
        return hipErrorInvalidValue;
    return f64 ? launch_wide_e<double>(a, s) : launch_wide_e<float>(a, s);
}

}  // namespace fmg
