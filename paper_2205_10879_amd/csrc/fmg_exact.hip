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
//
// Neighbourhoods wider than a wavefront (64 < k <= 256) use a pool instead:
// each wave appends the keys that beat its current k-th to a 512-entry LDS
// pool; when the pool nears capacity it is sorted (wave bitonic sort, eight
// keys per lane) and cut back to its k smallest, whose largest becomes the
// new k-th.
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
            if (lane == 0) o[0] = (int32_t)q;
            if (lane < a.k) o[1 + lane] = (int32_t)list.p;  // a.k <= 64 others
        } else if (lane < a.k) {
            o[lane] = (int32_t)list.p;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

constexpr int WIDE_POOL = 512;
constexpr int WIDE_E = WIDE_POOL / 64;

__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Ascending wave bitonic sort of 64*E exact keys; element g = lane*E + e is
// register e of lane `lane`.
template <int E>
__device__ __forceinline__ void wave_sort_xkeys(XKey (&key)[E]) {
    const int lane = lane_id();
    constexpr int N = 64 * E;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride < E) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    if ((e & stride) == 0) {
                        const bool asc = ((lane * E + e) & size) == 0;
                        XKey &u = key[e];
                        XKey &v = key[e | stride];
                        const bool swap = asc ? xless(v, u) : xless(u, v);
                        if (swap) {
                            const XKey t = u;
                            u = v;
                            v = t;
                        }
                    }
                }
            } else {
                const int lstride = stride / E;
                const int partner = lane ^ lstride;
                const bool lower = (lane & lstride) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const bool asc = ((lane * E + e) & size) == 0;
                    const XKey o = shfl_x(key[e], partner);
                    const bool o_less = xless(o, key[e]);
                    const bool take = (lower == asc) ? o_less : xless(key[e], o);
                    if (take) key[e] = o;
                }
            }
        }
    }
}

// Sort the wave's pool of cnt keys and keep its min(cnt, k) smallest at the
// front, ascending; *kth becomes the k-th smallest once k keys are held.
__device__ __forceinline__ int wide_select(uint64_t *__restrict__ pd, uint32_t *__restrict__ pp,
                                           int cnt, int k, XKey *kth) {
    const int lane = lane_id();
    wave_lds_fence();
    XKey key[WIDE_E];
#pragma unroll
    for (int e = 0; e < WIDE_E; ++e) {
        const int slot = lane * WIDE_E + e;
        key[e] = slot < cnt ? XKey{pd[slot], pp[slot]} : xkey_empty();
    }
    wave_lds_fence();
    wave_sort_xkeys<WIDE_E>(key);
    const int keep = cnt < k ? cnt : k;
#pragma unroll
    for (int e = 0; e < WIDE_E; ++e) {
        const int slot = lane * WIDE_E + e;
        if (slot < keep) {
            pd[slot] = key[e].d;
            pp[slot] = key[e].p;
        }
    }
    wave_lds_fence();
    if (keep == k) *kth = XKey{pd[k - 1], pp[k - 1]};
    return keep;
}

template <typename T>
__global__ __launch_bounds__(256) void exact_wide_kernel(ExactArgs a) {
#pragma clang fp contract(off)
    extern __shared__ __align__(16) char wsm[];  // z [4][d], pool keys [4][512], indices [4][512]
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    double *z = (double *)wsm + wave * a.d;
    uint64_t *pd = (uint64_t *)(wsm + (size_t)EXACT_WAVES * a.d * 8) + wave * WIDE_POOL;
    uint32_t *pp = (uint32_t *)(wsm + (size_t)EXACT_WAVES * a.d * 8 +
                                (size_t)EXACT_WAVES * WIDE_POOL * 8) +
                   wave * WIDE_POOL;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Qc = (const T *)a.Qc;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t items = a.count ? (int64_t)(*a.count) : a.nq;
    for (int64_t w = (int64_t)blockIdx.x * EXACT_WAVES + wave; w < items;
         w += (int64_t)gridDim.x * EXACT_WAVES) {
        const int64_t q = a.list ? (int64_t)a.list[w] : w;
        for (int c = lane; c < a.d; c += 64) z[c] = (double)Qc[q * a.d + c];
        wave_lds_fence();
        const int64_t self = a.loo ? q : -1;
        int cnt = 0;
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
            const bool pass = xless(key, kth);
            const uint64_t m = __ballot(pass);
            if (m != 0) {
                if (pass) {
                    const int pos = cnt + __popcll(m & lt);
                    pd[pos] = key.d;
                    pp[pos] = key.p;
                }
                cnt += __popcll(m);
                if (cnt > WIDE_POOL - 64) cnt = wide_select(pd, pp, cnt, a.k, &kth);
            }
        }
        cnt = wide_select(pd, pp, cnt, a.k, &kth);
        int32_t *o = a.out + q * (int64_t)a.out_stride;
        const int off = a.self_first ? 1 : 0;
        for (int s = lane; s < cnt; s += 64) o[off + s] = (int32_t)pp[s];
        if (a.self_first && lane == 0) o[0] = (int32_t)q;
        wave_lds_fence();
    }
}

}  // namespace

hipError_t launch_exact_topk(bool f64, const ExactArgs &a, int64_t max_items, hipStream_t s) {
    if (max_items <= 0) return hipSuccess;
    if (a.k < 1 || a.k > 256) return hipErrorInvalidValue;
    int64_t blocks = (max_items + EXACT_WAVES - 1) / EXACT_WAVES;
    if (blocks > 8192) blocks = 8192;
    if (a.k > 64) {
        const size_t wshm = (size_t)EXACT_WAVES * (8 * (size_t)a.d + 12 * WIDE_POOL);
        if (f64)
            hipLaunchKernelGGL(exact_wide_kernel<double>, dim3((unsigned)blocks), dim3(256), wshm,
                               s, a);
        else
            hipLaunchKernelGGL(exact_wide_kernel<float>, dim3((unsigned)blocks), dim3(256), wshm,
                               s, a);
        return hipGetLastError();
    }
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
