// Distance screen with MFMA and per-query candidate selection (Algorithm 2:
// the neighbour lookups of training points and queries).
//
// For a block of queries q and all training points p of a column range, one
// MFMA product per 16x16 tile returns S'(p, q) = ||x~_p||^2 - 2 <x~_p, z~_q>,
// which orders candidates exactly as the screened squared distance
// ||x~_p - z~_q||^2 does (the query norm is a per-query constant).  Each
// query keeps a running threshold: values at or below it are appended to the
// query's pool; when a pool nears capacity the owning wave sorts it, keeps the
// best c and lowers the threshold to the c-th value.  At the end each pool is
// sorted and its best c keys, ordered by (S', index), are written out with the
// c-th value, from which the re-rank certifies exactness.
//
// Layout (wave64, 16x16 MFMA tiles; tile row = candidate, tile column =
// query):
//   workgroup = 4 waves x 64 queries; each wave holds its queries' operand
//   fragments in registers for the whole column range;
//   per iteration the workgroup stages 64 candidate rows in LDS (double
//   buffered, rows padded by 16 bytes against bank conflicts) and every wave
//   runs 4 (query tiles) x 4 (candidate tiles) x KSTEPS MFMAs;
//   lane l of a 16x16 result holds candidates 4*(l/16)+i (i < 4) of the tile
//   for query l%16 of the tile.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct OpBF16 {
    typedef bf16x8 frag_t;
    static constexpr int BPS = 16;  // bytes per lane per k-step
    static __device__ __forceinline__ frag_t load(const char *p) {
        uint4 v = *(const uint4 *)p;
        return __builtin_bit_cast(frag_t, v);
    }
    static __device__ __forceinline__ f32x4 mfma(frag_t a, frag_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

struct OpF32 {
    typedef float frag_t;
    static constexpr int BPS = 4;
    static __device__ __forceinline__ frag_t load(const char *p) { return *(const float *)p; }
    static __device__ __forceinline__ f32x4 mfma(frag_t a, frag_t b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

constexpr int TILE = SCREEN_TILE;
constexpr int CAP = SCREEN_CAP;
constexpr int PE = CAP / 64;  // pool entries per lane during a selection

// Sort the pool of one query (cnt entries), keep the best c in slots 0..c-1.
// Returns the c-th key (SKEY_EMPTY when fewer than c entries).
__device__ __forceinline__ uint64_t select_pool(uint64_t *__restrict__ pool, int cnt, int c,
                                                int lane) {
    uint64_t key[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) {
        const int slot = lane * PE + e;
        key[e] = slot < cnt ? pool[slot] : SKEY_EMPTY;
    }
    wave_sort_u64<PE>(key);
#pragma unroll
    for (int e = 0; e < PE; ++e) {
        const int slot = lane * PE + e;
        if (slot < c) pool[slot] = key[e];
    }
    const int cl = (c - 1) / PE, ce = (c - 1) % PE;
    uint64_t kc = SKEY_EMPTY;
#pragma unroll
    for (int e = 0; e < PE; ++e)
        if (e == ce) kc = readlane_u64(key[e], cl);
    return kc;
}

template <class Op, int KSTEPS>
__global__ __launch_bounds__(256, 2) void screen_kernel(ScreenArgs a) {
    constexpr int RB = 4 * KSTEPS * Op::BPS;  // row bytes
    constexpr int LR = RB + 16;               // LDS row stride
    constexpr int CPT = (TILE * RB / 16) / 256;  // 16-byte chunks per thread per tile
    static_assert(CPT >= 1 && (TILE * RB / 16) % 256 == 0, "tile load split");
    __shared__ __align__(16) char tile[2][TILE * LR];

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int64_t wq0 = (int64_t)blockIdx.x * SCREEN_QPB + wave * 64;
    const int split = blockIdx.y;
    const int64_t cb = (int64_t)split * a.col_chunk;
    const int64_t ce = (cb + a.col_chunk < a.n_pad) ? cb + a.col_chunk : a.n_pad;
    const char *__restrict__ Pb = (const char *)a.P;

    // Query fragments, held for the whole column range.
    typename Op::frag_t bq[4][KSTEPS];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const char *qrow = (const char *)a.Q + (wq0 + t * 16 + r16) * RB + g * KSTEPS * Op::BPS;
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) bq[t][s] = Op::load(qrow + s * Op::BPS);
    }
    float thr[4];
    int cnt[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t q = wq0 + t * 16 + r16;
        thr[t] = (q < a.m) ? INFINITY : -INFINITY;  // padding queries never append
        cnt[t] = 0;
    }
    const uint64_t sq = 0x0001000100010001ull << r16;          // lanes sharing my query
    const uint64_t lsq = sq & ((1ull << lane) - 1ull);          // ... below me
    uint64_t *__restrict__ pool = a.pool + ((int64_t)split * a.m_pad + wq0) * CAP;

    uint4 pre[CPT];
    auto gload = [&](int64_t col0) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int chunk = threadIdx.x + i * 256;
            const int row = chunk / (RB / 16), off = (chunk % (RB / 16)) * 16;
            pre[i] = *(const uint4 *)(Pb + (col0 + row) * RB + off);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int i = 0; i < CPT; ++i) {
            const int chunk = threadIdx.x + i * 256;
            const int row = chunk / (RB / 16), off = (chunk % (RB / 16)) * 16;
            *(uint4 *)(tile[buf] + row * LR + off) = pre[i];
        }
    };

    if (cb < ce) {
        gload(cb);
        lstore(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t col = cb; col < ce; col += TILE) {
        const bool has_next = col + TILE < ce;
        if (has_next) gload(col + TILE);

        f32x4 acc[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[t][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        const char *tb = tile[buf] + r16 * LR + g * KSTEPS * Op::BPS;
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            typename Op::frag_t af[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) af[mt] = Op::load(tb + mt * 16 * LR + s * Op::BPS);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) acc[t][mt] = Op::mfma(af[mt], bq[t][s], acc[t][mt]);
        }

        // Candidate selection.
        bool appended = false;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            float mn = acc[t][0][0];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) mn = fminf(mn, acc[t][mt][i]);
            if (__ballot(mn <= thr[t]) != 0) {
                appended = true;
                const int64_t self = a.loo ? wq0 + t * 16 + r16 : -1;
                uint64_t *__restrict__ qp = pool + (t * 16 + r16) * CAP;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int64_t p = col + mt * 16 + g * 4 + i;
                        const float v = acc[t][mt][i];
                        const bool pass = (v <= thr[t]) && (p != self) && (p < a.n);
                        const uint64_t mask = __ballot(pass);
                        if (mask != 0) {
                            const int below = __popcll(mask & lsq);
                            const int tot = __popcll(mask & sq);
                            if (pass) qp[cnt[t] + below] = skey(v, (uint32_t)p);
                            cnt[t] += tot;
                        }
                    }
                }
            }
        }
        if (appended) {
            // Select in every pool that could overflow during the next tile.
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                uint64_t need = __ballot(cnt[t] > CAP - TILE) & 0xffffull;
                while (need != 0) {
                    const int rl = __ffsll((long long)need) - 1;
                    need &= need - 1;
                    const int c_now = __builtin_amdgcn_readlane(cnt[t], rl);
                    const uint64_t kc = select_pool(pool + (t * 16 + rl) * CAP, c_now, a.c, lane);
                    if (r16 == rl) {
                        cnt[t] = a.c < c_now ? a.c : c_now;
                        if (kc != SKEY_EMPTY) thr[t] = skey_val(kc);
                    }
                }
            }
        }
        if (has_next) lstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }

    // Final selection and output of every real query of this wave.
    for (int ql = 0; ql < 64; ++ql) {
        const int64_t q = wq0 + ql;
        if (q >= a.m) break;
        const int t = ql >> 4, rl = ql & 15;
        int c_now = 0;
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
            if (tt == t) c_now = __builtin_amdgcn_readlane(cnt[tt], rl);
        uint64_t *qp = pool + ql * CAP;
        const uint64_t kc = select_pool(qp, c_now, a.c, lane);
        uint64_t *__restrict__ out = a.cand + ((int64_t)split * a.m + q) * a.c;
        for (int r = lane; r < a.c; r += 64) out[r] = r < c_now ? qp[r] : SKEY_EMPTY;
        if (lane == 0) a.tq[(int64_t)split * a.m + q] = (kc != SKEY_EMPTY) ? skey_val(kc) : INFINITY;
    }
}

}  // namespace

hipError_t launch_screen(const ScreenGeom &g, const ScreenArgs &a, hipStream_t s) {
    dim3 grid((unsigned)(a.m_pad / SCREEN_QPB), (unsigned)a.splits);
    if (g.mode == SCREEN_BF16) {
        if (g.ksteps == 2)
            hipLaunchKernelGGL((screen_kernel<OpBF16, 2>), grid, dim3(256), 0, s, a);
        else
            return hipErrorInvalidValue;
    } else {
        switch (g.ksteps) {
        case 4: hipLaunchKernelGGL((screen_kernel<OpF32, 4>), grid, dim3(256), 0, s, a); break;
        case 8: hipLaunchKernelGGL((screen_kernel<OpF32, 8>), grid, dim3(256), 0, s, a); break;
        case 12: hipLaunchKernelGGL((screen_kernel<OpF32, 12>), grid, dim3(256), 0, s, a); break;
        case 16: hipLaunchKernelGGL((screen_kernel<OpF32, 16>), grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

}  // namespace fmg
