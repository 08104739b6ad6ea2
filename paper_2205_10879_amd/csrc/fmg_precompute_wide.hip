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
//   3. right-looking Cholesky in blocks of NB columns: every wavefront that
//      holds rows at or below a block factors its NB x NB diagonal block in
//      registers (one entry per lane, cross-lane reads), and alongside it
//      each thread below the block derives its row's NB entries of L; the whole
//      workgroup applies the block's NB rank-one updates to the trailing
//      columns, two rows per thread (two barriers per block; every entry
//      sees the single-step updates in step order, so the factor equals the
//      column-at-a-time one bit for bit);
//   4. forward and back substitution, thread a owning row a of all ell
//      right-hand sides: a block's rows are solved in turn by one wavefront
//      (cross-lane reads) and published in LDS, and the rows still to solve
//      subtract the block's contributions in step order; the forward pass
//      rides along with the factorisation, the backward pass takes one
//      barrier per block.
// A non-positive or non-finite pivot marks the row as not positive definite:
// its C row is NaN and its status is 1.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

constexpr int WIDE_THREADS = 1024;
constexpr int WIDE_KMAX = 256;  // largest k; entries of the diagonal buffer
constexpr int GRID = 32;        // the thread grid is GRID x GRID
constexpr int NB = 8;           // columns per block (divides 64: a block's rows share a wavefront)

template <typename T>
__device__ __forceinline__ T lane_value(T v, int lane);
template <>
__device__ __forceinline__ double lane_value<double>(double v, int lane) {
    return readlane_f64(v, lane);
}
template <>
__device__ __forceinline__ float lane_value<float>(float v, int lane) {
    return readlane_f32(v, lane);
}
template <typename T>
__device__ __forceinline__ T lane_shfl(T v, int src);
template <>
__device__ __forceinline__ double lane_shfl<double>(double v, int src) {
    return __longlong_as_double((long long)shfl_u64((uint64_t)__double_as_longlong(v), src));
}
template <>
__device__ __forceinline__ float lane_shfl<float>(float v, int src) {
    return __int_as_float((int)shfl_u32((uint32_t)__float_as_int(v), src));
}

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
    // rows, packed factor, diagonal, solved blocks, flag
    return (size_t)k * (d + 1) + (size_t)k * (k + 1) / 2 + WIDE_KMAX + 2 * (size_t)NB * ellmax + 1;
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
    T *dg = A + (size_t)k * (k + 1) / 2;        // [256] L_jj
    T *wb = dg + WIDE_KMAX;                     // [2][NB][ELLMAX] block rows of the solves
    int *badf = (int *)(wb + 2 * NB * ELLMAX);  // a pivot was not positive
    T *wf = wb, *yb = wb + NB * ELLMAX;         // forward solve: solved rows, rows to solve
    const T *__restrict__ X = (const T *)P.X;
    const T *__restrict__ Y = (const T *)P.Y;
    const int wave = a >> 6, lane = a & 63;
    const size_t arow = (size_t)a * (a + 1) / 2;

    int64_t p = 0;
    if (a < k) {
        p = (int64_t)P.N[i * k + a];
        for (int c = 0; c < d; ++c) xs[a * xs_ld + c] = X[p * d + c];
    }
    if (a == 0) *badf = 0;
    T y[ELLMAX];
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) y[c] = (a < k && c < ell) ? Y[p * ell + c] : T(0);
    if (a < NB && a < k) {
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) yb[a * ELLMAX + c] = y[c];
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

    // The factorisation carries the forward substitution L w = y along: the
    // last wavefront (it holds no rows, k <= 256) solves each block's rows as
    // soon as the block's diagonal factor exists, and every row below takes
    // the block's contributions after the first barrier.
    const int dr = lane >> 3, dc = lane & 7;  // lane's entry of a diagonal block
    const bool solver = wave == WIDE_THREADS / 64 - 1;
    for (int jb = 0; jb < k; jb += NB) {
        const int je = jb + NB < k ? jb + NB : k, nb = je - jb;
        const bool owner = wave == (jb >> 6);  // holds the block's rows
        const bool rows = (wave + 1) * 64 > jb && wave * 64 < k;
        T v = T(0);
        T u[NB];  // row a's entries of L in the block's columns
#pragma unroll
        for (int t = 0; t < NB; ++t) u[t] = T(0);
        if (rows || solver) {
            // the diagonal block, factored in registers by every wavefront
            // that holds rows at or below it: entry (jb + dr, jb + dc); a
            // partial block is padded with the identity
            if (dc <= dr)
                v = dr < nb ? A[(size_t)(jb + dr) * (jb + dr + 1) / 2 + jb + dc]
                            : (dc == dr ? T(1) : T(0));
            T ljj[NB];
            bool wbad = false;
            // step t of the diagonal block (branch-free, so that the rows'
            // own chains interleave with it)
            auto diag_step = [&](int t) {
                const T piv = lane_value<T>(v, t * (NB + 1));
                const bool ok = piv > T(0) && isfinite((double)piv);
                wbad = wbad || (!ok && t < nb);
                ljj[t] = ok ? (T)sqrt(piv) : T(1);
                const T q = v / ljj[t];
                v = (dc == t && dr > t && dr < nb) ? q : v;
                const T lr = lane_shfl<T>(v, dr * NB + t);
                const T lb = lane_shfl<T>(v, dc * NB + t);
                const T nv = v - lr * lb;
                v = (dc > t && dc <= dr && dr < nb) ? nv : v;
            };
            if (solver) {
                // the block's rows of L w = y, lane t holding row jb + t (in
                // y: this wavefront holds no rows of its own)
                T *ys = y;
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) ys[c] = lane < nb ? yb[lane * ELLMAX + c] : T(0);
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    diag_step(t);
#pragma unroll
                    for (int c = 0; c < ELLMAX; ++c) {
                        const T q = ys[c] / ljj[t];
                        ys[c] = lane == t ? q : ys[c];
                    }
                    const T l = lane_shfl<T>(v, (lane & 7) * NB + t);
#pragma unroll
                    for (int c = 0; c < ELLMAX; ++c) {
                        const T wt = lane_value<T>(ys[c], t);
                        const T ny = ys[c] - l * wt;
                        ys[c] = (lane > t && lane < nb) ? ny : ys[c];
                    }
                }
                if (lane < nb) {
#pragma unroll
                    for (int c = 0; c < ELLMAX; ++c) wf[lane * ELLMAX + c] = ys[c];
                }
            } else {
                // the rows below the block take the block's steps in order
                // alongside it: a division by the pivot once the earlier
                // columns' updates are in, then this column's update of the
                // later ones (a block with rows below it is full)
                const bool mine = je < k && a >= je && a < k;
#pragma unroll
                for (int t = 0; t < NB; ++t) u[t] = mine ? A[arow + jb + t] : T(0);
#pragma unroll
                for (int t = 0; t < NB; ++t) {
                    diag_step(t);
                    u[t] = u[t] / ljj[t];
#pragma unroll
                    for (int j = t + 1; j < NB; ++j) u[j] -= u[t] * lane_value<T>(v, j * NB + t);
                }
                if (mine) {
#pragma unroll
                    for (int t = 0; t < NB; ++t) A[arow + jb + t] = u[t];
                }
            }
            if (owner && lane == 0) {
#pragma unroll
                for (int t = 0; t < NB; ++t)
                    if (t < nb) dg[jb + t] = ljj[t];
                if (wbad) *badf = 1;
            }
        }
        __syncthreads();
        if (owner && dc <= dr && dr < nb)
            A[(size_t)(jb + dr) * (jb + dr + 1) / 2 + jb + dc] = v;
        if (a >= jb && a < je) {  // the block's rows are solved
#pragma unroll
            for (int c = 0; c < ELLMAX; ++c) y[c] = wf[(a - jb) * ELLMAX + c];
        } else if (a >= je && a < k) {
#pragma unroll
            for (int t = 0; t < NB; ++t) {
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) y[c] -= u[t] * wf[t * ELLMAX + c];
            }
            if (a < je + NB) {  // the next block's rows
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) yb[(a - je) * ELLMAX + c] = y[c];
            }
        }
        // trailing columns, the block's steps in order; a thread takes two
        // rows at once, so each column's entries of L are read once for both
        // (one row in FP64 with more than four right-hand sides, which would
        // run out of registers)
        constexpr bool PAIR = !(sizeof(T) == 8 && ELLMAX > 4);
        for (int r1 = je + ty; r1 < k; r1 += (PAIR ? 2 : 1) * GRID) {
            const int r2 = r1 + GRID;
            const bool two = PAIR && r2 < k;
            const size_t rr1 = (size_t)r1 * (r1 + 1) / 2, rr2 = (size_t)r2 * (r2 + 1) / 2;
            T l1[NB], l2[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                l1[t] = A[rr1 + jb + t];
                l2[t] = two ? A[rr2 + jb + t] : T(0);
            }
            const int bmax = two ? r2 : r1;
            for (int b = je + tx; b <= bmax; b += GRID) {
                const T *lb = A + (size_t)b * (b + 1) / 2 + jb;
                T cb[NB];
#pragma unroll
                for (int t = 0; t < NB; ++t) cb[t] = lb[t];
                if (b <= r1) {
                    T x = A[rr1 + b];
#pragma unroll
                    for (int t = 0; t < NB; ++t) x -= l1[t] * cb[t];
                    A[rr1 + b] = x;
                }
                if (two) {
                    T x = A[rr2 + b];
#pragma unroll
                    for (int t = 0; t < NB; ++t) x -= l2[t] * cb[t];
                    A[rr2 + b] = x;
                }
            }
        }
        __syncthreads();
    }
    const bool bad = *badf != 0;

    for (int jb = ((k - 1) / NB) * NB, blk = 0; jb >= 0; jb -= NB, ++blk) {  // L^T x = w
        const int je = jb + NB < k ? jb + NB : k, nb = je - jb;
        T *w = wb + (blk & 1) * NB * ELLMAX;
        if (wave == (jb >> 6)) {
            T lc[NB], dj[NB];  // L_{j,a} and L_jj for the block's columns j
#pragma unroll
            for (int t = 0; t < NB; ++t) {
                const int j = jb + t;
                lc[t] = (t < nb && a >= jb && a < j) ? A[(size_t)j * (j + 1) / 2 + a] : T(0);
                dj[t] = t < nb ? dg[j] : T(1);
            }
#pragma unroll
            for (int t = NB - 1; t >= 0; --t) {
                const int j = jb + t;
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) {
                    const T q = y[c] / dj[t];
                    y[c] = a == j ? q : y[c];
                }
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) {
                    const T xj = lane_value<T>(y[c], j & 63);
                    const T ny = y[c] - lc[t] * xj;
                    y[c] = (t < nb && a >= jb && a < j) ? ny : y[c];
                }
            }
            if (a >= jb && a < je) {
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) w[(a - jb) * ELLMAX + c] = y[c];
            }
        }
        __syncthreads();
        if (a < jb) {
            T lc[NB];
#pragma unroll
            for (int t = 0; t < NB; ++t)
                lc[t] = t < nb ? A[(size_t)(jb + t) * (jb + t + 1) / 2 + a] : T(0);
#pragma unroll
            for (int t = NB - 1; t >= 0; --t) {
#pragma unroll
                for (int c = 0; c < ELLMAX; ++c) {
                    const T ny = y[c] - lc[t] * w[t * ELLMAX + c];
                    y[c] = t < nb ? ny : y[c];
                }
            }
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
