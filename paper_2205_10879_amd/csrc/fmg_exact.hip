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
// The nearest point of a batch of queries (k = 1, the prediction's lookup)
// runs one query per lane instead: a wave takes 64 queries and one chunk of
// candidates, whose coordinates every lane reads at the same address; the
// chunks are sized so that about 8192 waves (NN_SPLIT_ENTRIES / 64) fill the
// device, and a merge
// takes the smallest (distance, index) over the chunks.
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

// Neighbourhoods wider than the wave (64 < k <= 256): each wave serves two
// queries, so every candidate row it loads is measured against both; each
// query keeps a pool of up to WIDE_POOL keys under its running k-th key.
constexpr int WIDE_Q = 2;  // queries per wave

template <typename T>
__global__ __launch_bounds__(256) void exact_wide_kernel(ExactArgs a) {
#pragma clang fp contract(off)
    // z [4][WIDE_Q][d], pool keys [4][WIDE_Q][512], indices [4][WIDE_Q][512]
    extern __shared__ __align__(16) char wsm[];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    double *zw = (double *)wsm + wave * WIDE_Q * a.d;
    uint64_t *pdw = (uint64_t *)(wsm + (size_t)EXACT_WAVES * WIDE_Q * a.d * 8) +
                    wave * WIDE_Q * WIDE_POOL;
    uint32_t *ppw = (uint32_t *)(wsm + (size_t)EXACT_WAVES * WIDE_Q * a.d * 8 +
                                 (size_t)EXACT_WAVES * WIDE_Q * WIDE_POOL * 8) +
                    wave * WIDE_Q * WIDE_POOL;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Qc = (const T *)a.Qc;
    const uint64_t lt = (1ull << lane) - 1ull;
    // FP64 rows of even length on a 16-byte aligned base load as double2
    const bool vec2 = sizeof(T) == 8 && (a.d % 2) == 0 && ((uintptr_t)a.X & 15) == 0;
    const int64_t items = a.count ? (int64_t)(*a.count) : a.nq;
    for (int64_t w = (int64_t)blockIdx.x * EXACT_WAVES + wave; w * WIDE_Q < items;
         w += (int64_t)gridDim.x * EXACT_WAVES) {
        int64_t q[WIDE_Q], self[WIDE_Q];
        bool act[WIDE_Q];
        int cnt[WIDE_Q];
        XKey kth[WIDE_Q];
#pragma unroll
        for (int h = 0; h < WIDE_Q; ++h) {
            const int64_t it = w * WIDE_Q + h;
            act[h] = it < items;
            q[h] = !act[h] ? 0 : a.list ? (int64_t)a.list[it] : it;
            self[h] = (a.loo && act[h]) ? q[h] : -1;
            cnt[h] = 0;
            kth[h] = xkey_empty();
            for (int c = lane; c < a.d; c += 64)
                zw[h * a.d + c] = act[h] ? (double)Qc[q[h] * a.d + c] : 0.0;
        }
        wave_lds_fence();
        // keys of candidate p (distances sd) offered to both rows' pools; the
        // pools keep every key below the running k-th, so the order in which
        // candidates are offered does not change the result
        auto offer = [&](int64_t p, const double (&sd)[WIDE_Q]) {
#pragma unroll
            for (int h = 0; h < WIDE_Q; ++h) {
                if (!act[h]) continue;  // uniform
                XKey key = xkey_empty();
                if (p < a.n && p != self[h]) key = XKey{dkey(sd[h]), (uint32_t)p};
                const bool pass = xless(key, kth[h]);
                const uint64_t m = __ballot(pass);
                if (m != 0) {
                    uint64_t *pd = pdw + h * WIDE_POOL;
                    uint32_t *pp = ppw + h * WIDE_POOL;
                    if (pass) {
                        const int pos = cnt[h] + __popcll(m & lt);
                        pd[pos] = key.d;
                        pp[pos] = key.p;
                    }
                    cnt[h] += __popcll(m);
                    if (cnt[h] > WIDE_POOL - 64) cnt[h] = wide_select(pd, pp, cnt[h], a.k, &kth[h]);
                }
            }
        };
        if (sizeof(T) == 8 && vec2 && a.d <= 8) {
            // short FP64 rows: two chunks of 64 candidates per step, both rows
            // loaded whole (16-byte loads) before any arithmetic, so the loads
            // of a step are in flight together; rows past n read row n - 1
            // and their keys are dropped
            const double *__restrict__ X8 = (const double *)a.X;
            for (int64_t base = 0; base < a.n; base += 128) {
                const int64_t p0 = base + lane, p1 = base + 64 + lane;
                const int64_t c0 = p0 < a.n ? p0 : a.n - 1, c1 = p1 < a.n ? p1 : a.n - 1;
                double2 r0[4], r1[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (2 * i < a.d) {
                        r0[i] = *(const double2 *)(X8 + c0 * a.d + 2 * i);
                        r1[i] = *(const double2 *)(X8 + c1 * a.d + 2 * i);
                    } else {
                        r0[i] = make_double2(0.0, 0.0);
                        r1[i] = make_double2(0.0, 0.0);
                    }
                }
                double s0[WIDE_Q], s1[WIDE_Q];
#pragma unroll
                for (int h = 0; h < WIDE_Q; ++h) s0[h] = s1[h] = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (2 * i < a.d) {
#pragma unroll
                        for (int h = 0; h < WIDE_Q; ++h) {
                            const double z0 = zw[h * a.d + 2 * i], z1 = zw[h * a.d + 2 * i + 1];
                            const double t0 = z0 - r0[i].x;
                            const double u0 = t0 * t0;
                            s0[h] = s0[h] + u0;
                            const double t1 = z1 - r0[i].y;
                            const double u1 = t1 * t1;
                            s0[h] = s0[h] + u1;
                            const double v0 = z0 - r1[i].x;
                            const double w0 = v0 * v0;
                            s1[h] = s1[h] + w0;
                            const double v1 = z1 - r1[i].y;
                            const double w1 = v1 * v1;
                            s1[h] = s1[h] + w1;
                        }
                    }
                }
                offer(p0, s0);
                offer(p1, s1);
            }
        } else {
            for (int64_t base = 0; base < a.n; base += 64) {
                const int64_t p = base + lane;
                double sd[WIDE_Q];
#pragma unroll
                for (int h = 0; h < WIDE_Q; ++h) sd[h] = 0.0;
                if (p < a.n) {
                    const T *__restrict__ xp = X + p * a.d;
                    if (vec2) {
                        // the row in 16-byte loads, coordinates still summed in order
                        for (int c = 0; c < a.d; c += 2) {
                            const double2 v = *(const double2 *)(xp + c);
#pragma unroll
                            for (int h = 0; h < WIDE_Q; ++h) {
                                const double t0 = zw[h * a.d + c] - v.x;
                                const double u0 = t0 * t0;
                                sd[h] = sd[h] + u0;
                                const double t1 = zw[h * a.d + c + 1] - v.y;
                                const double u1 = t1 * t1;
                                sd[h] = sd[h] + u1;
                            }
                        }
                    } else {
                        for (int c = 0; c < a.d; ++c) {
                            const double xv = (double)xp[c];
#pragma unroll
                            for (int h = 0; h < WIDE_Q; ++h) {
                                const double t = zw[h * a.d + c] - xv;
                                const double t2 = t * t;
                                sd[h] = sd[h] + t2;
                            }
                        }
                    }
                }
                offer(p, sd);
            }
        }
#pragma unroll
        for (int h = 0; h < WIDE_Q; ++h) {
            if (!act[h]) continue;
            uint64_t *pd = pdw + h * WIDE_POOL;
            uint32_t *pp = ppw + h * WIDE_POOL;
            const int kept = wide_select(pd, pp, cnt[h], a.k, &kth[h]);
            int32_t *o = a.out + q[h] * (int64_t)a.out_stride;
            const int off = a.self_first ? 1 : 0;
            for (int s2 = lane; s2 < kept; s2 += 64) o[off + s2] = (int32_t)pp[s2];
            if (a.self_first && lane == 0) o[0] = (int32_t)q[h];
        }
        wave_lds_fence();
    }
}

constexpr int64_t NN_WAVES = NN_SPLIT_ENTRIES / 64;

template <typename T, int DMAX>
__global__ __launch_bounds__(64) void nn_split_kernel(ExactArgs a, int64_t chunk, int splits) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * 64 + lane;
    const int y = blockIdx.y;
    const int64_t m = a.nq;
    const int d = a.d;
    const T *__restrict__ X = (const T *)a.X;
    const T *__restrict__ Qc = (const T *)a.Qc;
    double z[DMAX];
#pragma unroll
    for (int c = 0; c < DMAX; ++c) z[c] = (q < m && c < d) ? (double)Qc[q * d + c] : 0.0;
    const int64_t self = (a.loo && q < m) ? q : -1;
    const int64_t p0 = (int64_t)y * chunk;
    const int64_t p1 = (p0 + chunk < a.n) ? p0 + chunk : a.n;
    uint64_t bk = ~0ull;
    uint32_t bp = 0xffffffffu;
    // G candidates per iteration, their DMAX coordinates loaded unmasked (the
    // same rows for every lane, so scalar loads; X carries 64 elements of
    // padding past its last row) before any arithmetic; coordinates past d
    // contribute an exact +0 to the sum.
    constexpr int G = DMAX <= 4 ? 4 : (DMAX <= 8 ? 2 : 1);
    for (int64_t p = p0; p < p1; p += G) {
        double xv[G][DMAX];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t pr = (p + g < p1) ? p + g : p1 - 1;
            const T *__restrict__ xp = X + pr * d;
#pragma unroll
            for (int c = 0; c < DMAX; ++c) xv[g][c] = (double)xp[c];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < DMAX; ++c) {
                const double t = (c < d) ? z[c] - xv[g][c] : 0.0;
                const double t2 = t * t;
                s = s + t2;
            }
            const uint64_t key = dkey(s);
            const int64_t pg = p + g;
            if (pg < p1 && key < bk && pg != self) {  // ascending p: ties keep the smaller index
                bk = key;
                bp = (uint32_t)pg;
            }
        }
    }
    if (q < m) {
        if (splits == 1) {
            a.out[q * (int64_t)a.out_stride] = (int32_t)bp;
        } else {
            a.nn_key[(int64_t)y * m + q] = bk;
            a.nn_idx[(int64_t)y * m + q] = (int32_t)bp;
        }
    }
}

// Smallest (distance, index) over the chunks; one wave per query.
__global__ __launch_bounds__(256) void nn_merge_kernel(ExactArgs a, int splits) {
    const int lane = lane_id();
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (q >= a.nq) return;
    const int64_t m = a.nq;
    XKey key = xkey_empty();
    for (int y = lane; y < splits; y += 64) {
        const XKey o{a.nn_key[(int64_t)y * m + q], (uint32_t)a.nn_idx[(int64_t)y * m + q]};
        if (xless(o, key)) key = o;
    }
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const XKey o = shfl_x(key, lane ^ w);
        if (xless(o, key)) key = o;
    }
    if (lane == 0) a.out[q * (int64_t)a.out_stride] = (int32_t)key.p;
}

template <typename T, int DMAX>
hipError_t launch_nn_t(const ExactArgs &a, hipStream_t s) {
    const int64_t qb = (a.nq + 63) / 64;
    int64_t splits = a.nn_key && a.nn_idx ? NN_WAVES / qb : 1;
    const int64_t most = (a.n + 63) / 64;  // at least 64 candidates per chunk
    if (splits > most) splits = most;
    if (splits < 1) splits = 1;
    const int64_t chunk = (a.n + splits - 1) / splits;
    splits = (a.n + chunk - 1) / chunk;  // splits * nq <= NN_SPLIT_ENTRIES
    hipLaunchKernelGGL((nn_split_kernel<T, DMAX>), dim3((unsigned)qb, (unsigned)splits), dim3(64),
                       0, s, a, chunk, (int)splits);
    if (splits > 1)
        hipLaunchKernelGGL(nn_merge_kernel, dim3((unsigned)((a.nq + 3) / 4)), dim3(256), 0, s, a,
                           (int)splits);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_nn(const ExactArgs &a, hipStream_t s) {
    if (a.d <= 4) return launch_nn_t<T, 4>(a, s);
    if (a.d <= 8) return launch_nn_t<T, 8>(a, s);
    if (a.d <= 16) return launch_nn_t<T, 16>(a, s);
    if (a.d <= 32) return launch_nn_t<T, 32>(a, s);
    return launch_nn_t<T, 64>(a, s);
}

}  // namespace

hipError_t launch_exact_topk(bool f64, const ExactArgs &a, int64_t max_items, hipStream_t s) {
    if (max_items <= 0) return hipSuccess;
    if (a.k < 1 || a.k > 256) return hipErrorInvalidValue;
    if (a.k == 1 && !a.self_first && !a.list && !a.count && a.d <= 64)
        return f64 ? launch_nn<double>(a, s) : launch_nn<float>(a, s);
    int64_t blocks = (max_items + EXACT_WAVES - 1) / EXACT_WAVES;
    if (blocks > 8192) blocks = 8192;
    if (a.k > 64) {
        const size_t wshm = (size_t)EXACT_WAVES * WIDE_Q * (8 * (size_t)a.d + 12 * WIDE_POOL);
        blocks = (max_items + EXACT_WAVES * WIDE_Q - 1) / (EXACT_WAVES * WIDE_Q);
        if (blocks > 8192) blocks = 8192;
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
