// Prediction gather-dot (Algorithm 2, prediction loop; Section 3, prediction
// equation): for query z with nearest training point j,
//     mu(z)[c] = sum_s phi(||z - x_{N(j)_s}||) * C[j][s][c].
// One wavefront per query; lane s gathers neighbour N(j)_s with 16-byte
// loads, forms its kernel value, multiplies it into row s of C[j] (ell
// contiguous values, so the wave reads C[j] as one contiguous k*ell block)
// and the ell sums are DPP wave reductions.  Neighbourhoods wider than the
// wave (k <= 256) give lane s the rows s + 64 r as well.  The
// cross-covariance carries no nugget.  Queries may be taken in a given order
// (nearby queries in consecutive waves share neighbour rows in the caches).
#include "fmg_device.h"
#include "fmg_kernels.h"

#include <type_traits>

namespace fmg {

namespace {

constexpr int G_WAVES = 4;

// Squared distance of one row pair, coordinates loaded 16 bytes at a time
// when rows are 16-byte aligned (VEC), with four independent partial sums so
// that all loads of the row are in flight together.
template <typename T, bool VEC>
__device__ __forceinline__ T row_sqdist(const T *__restrict__ z, const T *__restrict__ x, int d) {
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    if constexpr (VEC && sizeof(T) == 4) {
#pragma unroll 4
        for (int c = 0; c < d; c += 4) {
            const float4 u = *(const float4 *)(z + c);
            const float4 v = *(const float4 *)(x + c);
            const float t0 = u.x - v.x, t1 = u.y - v.y, t2 = u.z - v.z, t3 = u.w - v.w;
            s0 = fmaf(t0, t0, s0);
            s1 = fmaf(t1, t1, s1);
            s2 = fmaf(t2, t2, s2);
            s3 = fmaf(t3, t3, s3);
        }
    } else if constexpr (VEC) {
#pragma unroll 4
        for (int c = 0; c < d; c += 2) {
            const double2 u = *(const double2 *)(z + c);
            const double2 v = *(const double2 *)(x + c);
            const double t0 = u.x - v.x, t1 = u.y - v.y;
            s0 = fma(t0, t0, s0);
            s1 = fma(t1, t1, s1);
        }
    } else {
#pragma unroll 4
        for (int c = 0; c < d; ++c) {
            const T t = z[c] - x[c];
            s0 += t * t;
        }
    }
    return (s0 + s1) + (s2 + s3);
}

template <typename T, bool VEC, int ELLMAX, int KR>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
    const int lane = lane_id();
    const int64_t wq = (int64_t)blockIdx.x * G_WAVES + (threadIdx.x >> 6);
    if (wq >= a.m) return;
    const int64_t q = a.order ? (int64_t)a.order[wq] : wq;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Z = (const T *)a.Z;
    const T *__restrict__ C = (const T *)a.C;
    const int64_t zr = a.zrow ? (int64_t)a.zrow[q] : q;
    const int64_t j = a.nn ? (int64_t)a.nn[q] : q;
    const int ell = a.ell;
    T *__restrict__ out = (T *)a.out + q * ell;
    if (zr < 0 || zr >= a.zrows || j < 0 || j >= a.crows) {  // a caller's row list
        if (lane < ell) out[lane] = (T)NAN;
        return;
    }
    // Row s of C[j]: ell contiguous values; the wave's rows form one
    // contiguous block of k * ell values.  Its loads only need j, so they
    // are issued before the neighbour rows.
    T cv[KR][ELLMAX];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int s = lane + 64 * r;
        const T *__restrict__ Cj = C + (j * a.k + s) * ell;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) cv[r][c] = (s < a.k && c < ell) ? Cj[c] : T(0);
    }
    T w[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int s = lane + 64 * r;
        w[r] = T(0);
        if (s < a.k) {
            const int64_t p = a.N[j * a.k + s];
            const T D = row_sqdist<T, VEC>(Z + zr * a.d, X + p * a.d, a.d);
            w[r] = phi_t<T>(D, a.kc, (T)a.inv_rho, (T)a.amp);
        }
    }
    // Fixed trip count (columns past ell are zero and not stored), so the loop
    // unrolls and cv stays in registers.
#pragma unroll
    for (int c = 0; c < ELLMAX; ++c) {
        T v = w[0] * cv[0][c];
#pragma unroll
        for (int r = 1; r < KR; ++r) v += w[r] * cv[r][c];
        const T t = dpp_t_sum_last<T>(v, lane);
        if (lane == 63 && c < ell) out[c] = t;
    }
}

// Neighbourhoods of at most one row per lane, rows of 16-byte vectors, and
// no divergent branch before the reductions:
//   - what depends only on the query comes by scalar loads: its position in
//     the order, its coefficient row j, its coordinates (every lane needs
//     them);
//   - C[j] (k * ell contiguous values) is read by coalesced loads of the
//     whole block into the wave's LDS slice, from which lane s takes row s;
//   - every lane, live or not, loads a valid neighbour row (indices past k
//     repeat the last), all NV vectors issued before the first is used;
//     vectors past the row and lanes past k are masked out of the sums.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;

typedef float gv_f32x4 __attribute__((ext_vector_type(4)));
typedef double gv_f64x2 __attribute__((ext_vector_type(2)));

#ifndef FMG_GATHER_QPW
#define FMG_GATHER_QPW 2
#endif
constexpr int GQ = FMG_GATHER_QPW;  // consecutive queries (in the order) per wave
#ifndef FMG_GATHER_WAVES
#define FMG_GATHER_WAVES 4
#endif
constexpr int GV_WAVES = FMG_GATHER_WAVES;  // waves per workgroup

template <typename T, int NV, int ELLMAX>
__global__ __launch_bounds__(64 * GV_WAVES) void gather_vec_kernel(GatherArgs a) {
    typedef typename std::conditional<sizeof(T) == 4, gv_f32x4, gv_f64x2>::type V;
    constexpr int EPV = 16 / (int)sizeof(T);  // elements per vector
    constexpr int CB = 64 * ELLMAX + ELLMAX;  // one C[j] in LDS (row reads stay inside)
    __shared__ T cbuf[GV_WAVES * CB];
    const int lane = lane_id();
    const int wave = (int)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w0 = ((int64_t)blockIdx.x * GV_WAVES + wave) * GQ;
    if (w0 >= a.m) return;
    const int cnt = (int)(a.m - w0 < GQ ? a.m - w0 : GQ);
    const int ell = a.ell, k = a.k, d = a.d, nv = d / EPV, kl = k * ell;
    const int s = lane < k ? lane : k - 1;
    T *__restrict__ cb = cbuf + wave * CB;

    // Head of query w: its index, row of Z and coefficient row (scalar
    // loads), then its neighbour indices and C[j] block (vector loads).
    // A query whose rows fall outside the arrays reads row 0 and is written
    // as NaN.
    int64_t q = 0, zr = 0, j = 0, p = 0;
    bool ok = false;
    T cf[ELLMAX];
    auto head = [&](int64_t w) {
        q = a.order ? (int64_t)((const_ptr<uint32_t>)a.order)[w] : w;
        zr = a.zrow ? (int64_t)((const_ptr<int32_t>)a.zrow)[q] : q;
        j = a.nn ? (int64_t)((const_ptr<int32_t>)a.nn)[q] : q;
        ok = zr >= 0 && zr < a.zrows && j >= 0 && j < a.crows;
        if (!ok) zr = j = 0;
        p = a.N[j * k + s];
        const T *__restrict__ Cj = (const T *)a.C + j * kl;
#pragma unroll
        for (int t = 0; t < ELLMAX; ++t) {
            const int f = lane + 64 * t;
            cf[t] = Cj[f < kl ? f : kl - 1];
        }
    };
    head(w0);
    for (int i = 0; i < cnt; ++i) {
        const int64_t qi = q, zri = zr;
        const bool oki = ok;
        // this query's neighbour rows and coordinates
        const V *__restrict__ xr = (const V *)((const T *)a.X + p * d);
        V xv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) xv[v] = xr[v < nv ? v : nv - 1];
        const const_ptr<V> zc = (const_ptr<V>)((const T *)a.Z + zri * d);
        V zv[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) zv[v] = zc[v < nv ? v : nv - 1];
        // its C[j] into the wave's LDS slice (a wave's LDS accesses are
        // processed in order, so the previous query's reads are done), then
        // the next query's head
#pragma unroll
        for (int t = 0; t < ELLMAX; ++t) cb[lane + 64 * t] = cf[t];
        if (i + 1 < cnt) head(w0 + i + 1);
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const bool in = v < nv;
            if constexpr (sizeof(T) == 4) {
                const float t0 = in ? zv[v].x - xv[v].x : 0.0f;
                const float t1 = in ? zv[v].y - xv[v].y : 0.0f;
                const float t2 = in ? zv[v].z - xv[v].z : 0.0f;
                const float t3 = in ? zv[v].w - xv[v].w : 0.0f;
                s0 = fmaf(t0, t0, s0);
                s1 = fmaf(t1, t1, s1);
                s2 = fmaf(t2, t2, s2);
                s3 = fmaf(t3, t3, s3);
            } else {
                const double t0 = in ? zv[v].x - xv[v].x : 0.0, t1 = in ? zv[v].y - xv[v].y : 0.0;
                if (v & 1) {
                    s2 = fma(t0, t0, s2);
                    s3 = fma(t1, t1, s3);
                } else {
                    s0 = fma(t0, t0, s0);
                    s1 = fma(t1, t1, s1);
                }
            }
        }
        const T wk = phi_t<T>((s0 + s1) + (s2 + s3), a.kc, (T)a.inv_rho, (T)a.amp);
        const T wgt = lane < k ? wk : T(0);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const T *__restrict__ crow = cb + s * ell;
        T *__restrict__ out = (T *)a.out + qi * ell;
#pragma unroll
        for (int c = 0; c < ELLMAX; ++c) {
            const T t = dpp_t_sum_last<T>(wgt * crow[c], lane);
            if (lane == 63 && c < ell) out[c] = oki ? t : (T)NAN;
        }
    }
}

template <typename T, int NV>
void launch_gather_vec_nv(const GatherArgs &a, unsigned blocks, hipStream_t s) {
#define FMG_GV(E) hipLaunchKernelGGL((gather_vec_kernel<T, NV, E>), dim3(blocks), dim3(64 * GV_WAVES), 0, s, a)
    if (a.ell <= 1) FMG_GV(1);
    else if (a.ell <= 2) FMG_GV(2);
    else if (a.ell <= 4) FMG_GV(4);
    else if (a.ell <= 8) FMG_GV(8);
    else if (a.ell <= 10) FMG_GV(10);
    else if (a.ell <= 12) FMG_GV(12);
    else FMG_GV(16);
#undef FMG_GV
}

// Response columns are reduced up to ELLMAX (zeros past ell are not stored).
template <typename T, bool VEC, int KR>
void launch_gather_kr(const GatherArgs &a, unsigned blocks, hipStream_t s) {
    if (a.ell <= 1)
        hipLaunchKernelGGL((gather_kernel<T, VEC, 1, KR>), dim3(blocks), dim3(256), 0, s, a);
    else if (a.ell <= 4)
        hipLaunchKernelGGL((gather_kernel<T, VEC, 4, KR>), dim3(blocks), dim3(256), 0, s, a);
    else if (a.ell <= 8)
        hipLaunchKernelGGL((gather_kernel<T, VEC, 8, KR>), dim3(blocks), dim3(256), 0, s, a);
    else if (a.ell <= 12)
        hipLaunchKernelGGL((gather_kernel<T, VEC, 12, KR>), dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((gather_kernel<T, VEC, 16, KR>), dim3(blocks), dim3(256), 0, s, a);
}

template <typename T, bool VEC>
void launch_gather_t(const GatherArgs &a, unsigned blocks, hipStream_t s) {
    constexpr int EPV = 16 / (int)sizeof(T);
    const int nv = a.d / EPV;
    if (VEC && a.k <= 64 && nv <= 16) {
        blocks = (unsigned)((a.m + GV_WAVES * GQ - 1) / (GV_WAVES * GQ));
        if (nv <= 1) launch_gather_vec_nv<T, 1>(a, blocks, s);
        else if (nv <= 2) launch_gather_vec_nv<T, 2>(a, blocks, s);
        else if (nv <= 4) launch_gather_vec_nv<T, 4>(a, blocks, s);
        else if (nv <= 8) launch_gather_vec_nv<T, 8>(a, blocks, s);
        else if (nv <= 10) launch_gather_vec_nv<T, 10>(a, blocks, s);
        else if (nv <= 12) launch_gather_vec_nv<T, 12>(a, blocks, s);
        else launch_gather_vec_nv<T, 16>(a, blocks, s);
    } else if (a.k <= 64) launch_gather_kr<T, VEC, 1>(a, blocks, s);
    else launch_gather_kr<T, VEC, 4>(a, blocks, s);
}

}  // namespace

hipError_t launch_gather(bool f64, const GatherArgs &a, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.m + G_WAVES - 1) / G_WAVES);
    // Rows are 16-byte aligned when d is a multiple of 4 (float) or 2
    // (double) and both arrays start on a 16-byte boundary.
    if (a.ell > 16 || a.k > 256) return hipErrorInvalidValue;
    const bool base16 = (((uintptr_t)a.X | (uintptr_t)a.Z) & 15) == 0;
    const bool vec = f64 ? (a.d % 2 == 0 && base16) : (a.d % 4 == 0 && base16);
    if (f64) {
        if (vec) launch_gather_t<double, true>(a, blocks, s);
        else launch_gather_t<double, false>(a, blocks, s);
    } else {
        if (vec) launch_gather_t<float, true>(a, blocks, s);
        else launch_gather_t<float, false>(a, blocks, s);
    }
    return hipGetLastError();
}

}  // namespace fmg
