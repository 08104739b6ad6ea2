// Exact neighbour search in FP64 (Algorithm 2: the training-point and query
// neighbour lookups).  One wavefront per query row keeps the 64 smallest
// (distance, index) keys seen so far, one per lane in ascending order; each
// chunk of 64 training points is merged in only if one of its keys beats the
// current k-th.  Distances are computed exactly as the ranking defines them:
// coordinate differences, squares and sums in FP64, each rounded on its own,
// coordinates in increasing order.
//
// Used as the whole search in FP64 mode, and as the rescan of rows whose
// screened candidate list could not be certified exact.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

constexpr int EXACT_WAVES = 4;

template <typename T>
__global__ __launch_bounds__(256) void exact_topk_kernel(ExactArgs a) {
#pragma clang fp contract(off)
    extern __shared__ double zsh[];  // [EXACT_WAVES, d]
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    double *z = zsh + wave * a.d;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Qc = (const T *)a.Qc;
    const int64_t items = a.count ? (int64_t)(*a.count) : a.nq;
    for (int64_t w = (int64_t)blockIdx.x * EXACT_WAVES + wave; w < items;
         w += (int64_t)gridDim.x * EXACT_WAVES) {
        const int64_t q = a.list ? (int64_t)a.list[w] : w;
        for (int c = lane; c < a.d; c += 64) z[c] = (double)Qc[q * a.d + c];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int64_t self = a.loo ? q : -1;
        XKey list = xkey_empty();
        XKey kth = xkey_empty();
        for (int64_t base = 0; base < a.n; base += 64) {
            const int64_t p = base + lane;
            XKey key = xkey_empty();
            if (p < a.n && p != self) {
                const T *__restrict__ xp = X + p * a.d;
                double s = 0.0;
                for (int c = 0; c < a.d; ++c) {
                    const double t = z[c] - (double)xp[c];
                    const double t2 = t * t;
                    s = s + t2;
                }
                key = XKey{dkey(s), (uint32_t)p};
            }
            if (__ballot(xless(key, kth)) != 0) {
                list = wave_merge_x(list, key);
                kth = readlane_x(list, a.k - 1);
            }
        }
        int32_t *o = a.out + q * (int64_t)a.out_stride;
        if (a.self_first) {
            const uint32_t prev = shfl_u32(list.p, lane > 0 ? lane - 1 : 0);
            if (lane == 0) o[0] = (int32_t)q;
            else if (lane <= a.k) o[lane] = (int32_t)prev;
        } else if (lane < a.k) {
            o[lane] = (int32_t)list.p;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

}  // namespace

hipError_t launch_exact_topk(bool f64, const ExactArgs &a, int64_t max_items, hipStream_t s) {
    if (max_items <= 0) return hipSuccess;
    int64_t blocks = (max_items + EXACT_WAVES - 1) / EXACT_WAVES;
    if (blocks > 8192) blocks = 8192;
    const size_t shm = sizeof(double) * EXACT_WAVES * (size_t)a.d;
    if (f64)
        hipLaunchKernelGGL(exact_topk_kernel<double>, dim3((unsigned)blocks), dim3(256), shm, s,
                           a);
    else
        hipLaunchKernelGGL(exact_topk_kernel<float>, dim3((unsigned)blocks), dim3(256), shm, s,
                           a);
    return hipGetLastError();
}

}  // namespace fmg
