// Device-side building blocks shared by the FastMuyGPs HIP kernels (gfx950,
// wave64): orderable keys, wave shuffles, wave-wide bitonic sorting and the
// Matern / RBF kernel functions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define FMG_WAVE 64

namespace fmg {

__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// ---------------------------------------------------------------------------
// Orderable keys.  A float / double maps to an unsigned integer whose
// unsigned order is the numeric order (NaN sorts after +inf).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fkey(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(uint32_t k) {
    uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t dkey(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(uint64_t k) {
    uint64_t u = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

// BF16 from FP32, round to nearest even (finite inputs), and back.
__device__ __forceinline__ uint16_t f32_to_bf16_rn(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float((uint32_t)h << 16);
}

// Screen key: (screened value, candidate index) packed in 64 bits so that one
// unsigned compare orders by value, then by index.
__device__ __forceinline__ uint64_t skey(float s, uint32_t p) {
    return ((uint64_t)fkey(s) << 32) | (uint64_t)p;
}
__device__ __forceinline__ float skey_val(uint64_t k) { return fkey_inv((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t skey_idx(uint64_t k) { return (uint32_t)k; }
constexpr uint64_t SKEY_EMPTY = ~0ull;

// Exact key: (FP64 distance, index).
struct XKey {
    uint64_t d;
    uint32_t p;
};
__device__ __forceinline__ bool xless(const XKey &a, const XKey &b) {
    return a.d < b.d || (a.d == b.d && a.p < b.p);
}
__device__ __forceinline__ XKey xkey_empty() { return XKey{~0ull, 0xffffffffu}; }

// ---------------------------------------------------------------------------
// Wave shuffles through ds_bpermute.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src_lane) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src_lane) {
    uint32_t lo = shfl_u32((uint32_t)v, src_lane);
    uint32_t hi = shfl_u32((uint32_t)(v >> 32), src_lane);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ XKey shfl_x(const XKey &k, int src_lane) {
    return XKey{shfl_u64(k.d, src_lane), shfl_u32(k.p, src_lane)};
}
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ float readlane_f32(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    return __longlong_as_double((long long)readlane_u64((uint64_t)__double_as_longlong(v), lane));
}
__device__ __forceinline__ XKey readlane_x(const XKey &k, int lane) {
    return XKey{readlane_u64(k.d, lane), (uint32_t)__builtin_amdgcn_readlane((int)k.p, lane)};
}

// Wave sums through DPP: quad permutes and row rotates give every lane its
// row-of-16 sum, then the row-15 and row-31 broadcasts carry row totals up;
// the full sum is valid in lane 63 only.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}
template <typename T>
__device__ __forceinline__ T dpp_t_sum_last(T v, int lane) {
    auto mv = [](auto x, auto ctrl_tag) {
        constexpr int C = decltype(ctrl_tag)::value;
        if constexpr (sizeof(T) == 4) return dpp_f32<C>(x);
        else return dpp_f64<C>(x);
    };
    v += mv(v, std::integral_constant<int, 0xb1>{});   // quad_perm [1,0,3,2]
    v += mv(v, std::integral_constant<int, 0x4e>{});   // quad_perm [2,3,0,1]
    v += mv(v, std::integral_constant<int, 0x124>{});  // row_ror:4
    v += mv(v, std::integral_constant<int, 0x128>{});  // row_ror:8
    T t = mv(v, std::integral_constant<int, 0x142>{}); // row_bcast:15
    if ((lane & 31) >= 16) v += t;
    t = mv(v, std::integral_constant<int, 0x143>{});   // row_bcast:31
    if (lane >= 32) v += t;
    return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}

// ---------------------------------------------------------------------------
// Wave-wide bitonic sort, ascending, of 64*E keys.  Element g = lane*E + e
// lives in register e of lane `lane`.  Partners closer than E are in the
// same lane; farther ones are exchanged across lanes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void cswap_u64(uint64_t &a, uint64_t &b, bool asc) {
    uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = asc ? lo : hi;
    b = asc ? hi : lo;
}

template <int E>
__device__ __forceinline__ void wave_sort_u64(uint64_t (&key)[E]) {
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
                        const int g = lane * E + e;
                        cswap_u64(key[e], key[e | stride], (g & size) == 0);
                    }
                }
            } else {
                const int lstride = stride / E;
                const int partner = lane ^ lstride;
                const bool lower = (lane & lstride) == 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int g = lane * E + e;
                    const bool asc = (g & size) == 0;
                    uint64_t other = shfl_u64(key[e], partner);
                    uint64_t mn = key[e] < other ? key[e] : other;
                    uint64_t mx = key[e] < other ? other : key[e];
                    key[e] = (lower == asc) ? mn : mx;
                }
            }
        }
    }
}

// One key per lane: full bitonic sort over the wave (ascending by lane).
__device__ __forceinline__ XKey wave_sort_x(XKey k) {
    const int lane = lane_id();
#pragma unroll
    for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int partner = lane ^ stride;
            const bool lower = (lane & stride) == 0;
            const bool asc = (lane & size) == 0;
            XKey o = shfl_x(k, partner);
            bool o_less = xless(o, k);
            // keep the smaller if (lower == asc), else the larger
            bool take = (lower == asc) ? o_less : xless(k, o);
            if (take) k = o;
        }
    }
    return k;
}

// `list` ascending by lane, `chunk` arbitrary: returns the 64 smallest of
// both, ascending by lane.
__device__ __forceinline__ XKey wave_merge_x(XKey list, XKey chunk) {
    const int lane = lane_id();
    XKey s = wave_sort_x(chunk);
    XKey rev = shfl_x(s, 63 - lane);
    XKey k = xless(rev, list) ? rev : list;  // bitonic sequence of the 64 smallest
#pragma unroll
    for (int stride = 32; stride > 0; stride >>= 1) {
        const int partner = lane ^ stride;
        const bool lower = (lane & stride) == 0;
        XKey o = shfl_x(k, partner);
        bool take = lower ? xless(o, k) : xless(k, o);
        if (take) k = o;
    }
    return k;
}

// ---------------------------------------------------------------------------
// Kernel functions phi (Section 2, Matern equation; the half-integer nu
// closed forms and the RBF limit), from the squared distance D.
// kcode: 0 = RBF, 1 = Matern 1/2, 2 = Matern 3/2, 3 = Matern 5/2.
// ---------------------------------------------------------------------------
enum { KC_RBF = 0, KC_M12 = 1, KC_M32 = 2, KC_M52 = 3 };

__device__ __forceinline__ double phi64(double D, int kc, double inv_rho, double amp) {
    if (kc == KC_RBF) return amp * exp(-0.5 * D * inv_rho * inv_rho);
    double r = sqrt(D);
    if (kc == KC_M12) return amp * exp(-r * inv_rho);
    if (kc == KC_M32) {
        double s = 1.7320508075688772 * r * inv_rho;
        return amp * (1.0 + s) * exp(-s);
    }
    double s = 2.2360679774997896 * r * inv_rho;
    return amp * (1.0 + s + s * s * (1.0 / 3.0)) * exp(-s);
}

__device__ __forceinline__ float phi32(float D, int kc, float inv_rho, float amp) {
    if (kc == KC_RBF) return amp * expf(-0.5f * D * inv_rho * inv_rho);
    float r = sqrtf(D);
    if (kc == KC_M12) return amp * expf(-r * inv_rho);
    if (kc == KC_M32) {
        float s = 1.7320508f * r * inv_rho;
        return amp * (1.0f + s) * expf(-s);
    }
    float s = 2.2360680f * r * inv_rho;
    return amp * (1.0f + s + s * s * (1.0f / 3.0f)) * expf(-s);
}

// The same four kernels in one branch-free form,
//     phi = amp (1 + c1 s + c2 s^2) exp(-s),  s = scale * (D or sqrt(D)),
// with the uniform parameters chosen once per launch; unrolled loops over
// many entries then inline one short sequence instead of four.
template <typename T>
struct PhiForm {
    bool root;  // s from sqrt(D) (Matern) or from D (RBF)
    T scale, c1, c2, amp;
};

template <typename T>
__device__ __forceinline__ PhiForm<T> phi_form(int kc, double inv_rho, double amp) {
    PhiForm<T> f;
    f.root = kc != KC_RBF;
    f.amp = (T)amp;
    f.c1 = (T)0;
    f.c2 = (T)0;
    if (kc == KC_RBF) {
        f.scale = (T)(0.5 * inv_rho * inv_rho);
    } else if (kc == KC_M12) {
        f.scale = (T)inv_rho;
    } else if (kc == KC_M32) {
        f.scale = (T)(1.7320508075688772 * inv_rho);
        f.c1 = (T)1;
    } else {
        f.scale = (T)(2.2360679774997896 * inv_rho);
        f.c1 = (T)1;
        f.c2 = (T)(1.0 / 3.0);
    }
    return f;
}

__device__ __forceinline__ float phi_eval(const PhiForm<float> &f, float D) {
    const float s = f.scale * (f.root ? sqrtf(D) : D);
    return f.amp * fmaf(fmaf(f.c2, s, f.c1), s, 1.0f) * expf(-s);
}

__device__ __forceinline__ double phi_eval(const PhiForm<double> &f, double D) {
    const double s = f.scale * (f.root ? sqrt(D) : D);
    return f.amp * fma(fma(f.c2, s, f.c1), s, 1.0) * exp(-s);
}

template <typename T>
__device__ __forceinline__ T phi_t(T D, int kc, T inv_rho, T amp);
template <>
__device__ __forceinline__ double phi_t<double>(double D, int kc, double inv_rho, double amp) {
    return phi64(D, kc, inv_rho, amp);
}
template <>
__device__ __forceinline__ float phi_t<float>(float D, int kc, float inv_rho, float amp) {
    return phi32(D, kc, inv_rho, amp);
}

// Squared distance with every operation rounded on its own, coordinates in
// increasing order: the definition the exact neighbour ranking uses.
template <typename T>
__device__ __forceinline__ double exact_sqdist(const T *__restrict__ a, const T *__restrict__ b,
                                               int d) {
#pragma clang fp contract(off)
    double s = 0.0;
    for (int c = 0; c < d; ++c) {
        double t = (double)a[c] - (double)b[c];
        double t2 = t * t;
        s = s + t2;
    }
    return s;
}

}  // namespace fmg
