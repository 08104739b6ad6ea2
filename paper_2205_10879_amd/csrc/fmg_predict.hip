// Prediction gather-dot (Algorithm 2, prediction loop; Section 3, prediction
// equation): for query z with nearest training point j,
//     mu(z)[c] = sum_s phi(||z - x_{N(j)_s}||) * C[j][s][c].
// One wavefront per query; lane s gathers neighbour N(j)_s, forms its kernel
// value, multiplies it into row s of C[j] (ell contiguous values, so the
// wave reads C[j] as one contiguous k*ell block) and the ell sums are wave
// reductions.  The cross-covariance carries no nugget.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

constexpr int G_WAVES = 4;

template <typename T>
__device__ __forceinline__ T wave_sum_t(T v);
template <>
__device__ __forceinline__ float wave_sum_t<float>(float v) { return wave_sum_f32(v); }
template <>
__device__ __forceinline__ double wave_sum_t<double>(double v) { return wave_sum_f64(v); }

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
    const int lane = lane_id();
    const int64_t q = (int64_t)blockIdx.x * G_WAVES + (threadIdx.x >> 6);
    if (q >= a.m) return;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Z = (const T *)a.Z;
    const T *__restrict__ C = (const T *)a.C;
    const int64_t j = a.nn[q];
    T w = T(0);
    if (lane < a.k) {
        const int64_t p = a.N[j * a.k + lane];
        const T *__restrict__ xp = X + p * a.d;
        const T *__restrict__ zq = Z + q * a.d;
        T D = T(0);
        for (int c = 0; c < a.d; ++c) {
            const T t = zq[c] - xp[c];
            D += t * t;
        }
        w = phi_t<T>(D, a.kc, (T)a.inv_rho, (T)a.amp);
    }
    const T *__restrict__ Cj = C + (j * a.k + lane) * a.ell;
    T *__restrict__ out = (T *)a.out + q * a.ell;
    for (int c = 0; c < a.ell; ++c) {
        T v = (lane < a.k) ? w * Cj[c] : T(0);
        v = wave_sum_t<T>(v);
        if (lane == 0) out[c] = v;
    }
}

}  // namespace

hipError_t launch_gather(bool f64, const GatherArgs &a, hipStream_t s) {
    if (a.m <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((a.m + G_WAVES - 1) / G_WAVES);
    if (f64)
        hipLaunchKernelGGL(gather_kernel<double>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace fmg
