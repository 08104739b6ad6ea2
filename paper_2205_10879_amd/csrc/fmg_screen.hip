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
//   buffered, loaded by LDS-DMA one tile ahead, 16-byte chunks XOR-swizzled
//   against bank conflicts) and every wave runs 4 (query tiles) x
//   4 (candidate tiles) x KSTEPS MFMAs;
//   lane l of a 16x16 result holds candidates 4*(l/16)+i (i < 4) of the tile
//   for query l%16 of the tile.
#include "fmg_device.h"
#include "fmg_kernels.h"

#include <type_traits>

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

// Pool entries hold the raw pair (index << 32 | float bits of S'); selection
// works on keys (orderable value << 32 | index), which order by (S', index).
__device__ __forceinline__ uint64_t raw_entry(float v, uint32_t p) {
    return ((uint64_t)p << 32) | (uint64_t)__float_as_uint(v);
}
__device__ __forceinline__ uint64_t raw_to_key(uint64_t r) {
    return ((uint64_t)fkey(__uint_as_float((uint32_t)r)) << 32) | (r >> 32);
}
__device__ __forceinline__ uint64_t key_to_raw(uint64_t k) {
    return ((uint64_t)(uint32_t)k << 32) | (uint64_t)__float_as_uint(skey_val(k));
}

__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = shfl_u64(v, lane_id() ^ m);
        v = o > v ? o : v;
    }
    return v;
}
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Inclusive prefix sum over the wave with DPP: row shifts by 1, 2, 4 and 8
// within each row of 16 lanes, then the row-15 and row-31 broadcasts carry
// the row totals across rows (no LDS round trip).
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
    const int rl = lane & 15;
    int t = __builtin_amdgcn_mov_dpp(v, 0x111, 0xf, 0xf, false);  // row_shr:1
    if (rl >= 1) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x112, 0xf, 0xf, false);  // row_shr:2
    if (rl >= 2) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x114, 0xf, 0xf, false);  // row_shr:4
    if (rl >= 4) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x118, 0xf, 0xf, false);  // row_shr:8
    if (rl >= 8) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x142, 0xf, 0xf, false);  // row_bcast:15
    if ((lane & 31) >= 16) v += t;
    t = __builtin_amdgcn_mov_dpp(v, 0x143, 0xf, 0xf, false);  // row_bcast:31
    if (lane >= 32) v += t;
    return v;
}

// The bin of a 256-bin LDS histogram that holds the need-th smallest item
// (1 <= need <= total): *before = items in lower bins, *inbin = items in it.
__device__ __forceinline__ int hist_find(const uint32_t *__restrict__ hist, int need, int lane,
                                         int *before_out, int *inbin_out) {
    const uint4 h = ((const uint4 *)hist)[lane];
    const int own = (int)(h.x + h.y + h.z + h.w);
    const int incl = wave_incl_scan(own, lane);
    const int excl = incl - own;
    const bool mine = excl < need && need <= incl;
    int bin = 3, before = excl + (int)(h.x + h.y + h.z), inbin = (int)h.w;
    if (excl + (int)(h.x + h.y + h.z) >= need) { bin = 2; before = excl + (int)(h.x + h.y); inbin = (int)h.z; }
    if (excl + (int)(h.x + h.y) >= need) { bin = 1; before = excl + (int)h.x; inbin = (int)h.y; }
    if (excl + (int)h.x >= need) { bin = 0; before = excl; inbin = (int)h.x; }
    const int L = __ffsll((long long)__ballot(mine)) - 1;
    *before_out = __builtin_amdgcn_readlane(before, L);
    *inbin_out = __builtin_amdgcn_readlane(inbin, L);
    return L * 4 + __builtin_amdgcn_readlane(bin, L);
}

// Radix selection (8-bit digits, most significant first) of the c-th
// smallest of the wave's 64*PE keys (~0 marks an empty slot).  Returns a bound
// B such that exactly the c smallest keys satisfy key <= B, or ~0 when fewer
// than c keys are present (keep them all).  hist: 256 words of LDS.
template <int PE>
__device__ __forceinline__ uint64_t radix_kth(const uint64_t (&key)[PE], int c,
                                              uint32_t *__restrict__ hist, int lane) {
    int valid = 0;
#pragma unroll
    for (int e = 0; e < PE; ++e) valid += __popcll(__ballot(key[e] != ~0ull));
    if (valid <= c) return ~0ull;
    uint64_t prefix = 0;
    int need = c;
    for (int r = 0; r < 8; ++r) {
        const int shift = 56 - 8 * r;
        ((uint4 *)hist)[lane] = uint4{0u, 0u, 0u, 0u};
        wave_lds_sync();
#pragma unroll
        for (int e = 0; e < PE; ++e) {
            const bool in = key[e] != ~0ull && (r == 0 || (key[e] >> (shift + 8)) == (prefix >> (shift + 8)));
            if (in) atomicAdd(&hist[(uint32_t)(key[e] >> shift) & 255u], 1u);
        }
        wave_lds_sync();
        int cb, cin;
        const int digit = hist_find(hist, need, lane, &cb, &cin);
        prefix |= (uint64_t)digit << shift;
        need -= cb;
        wave_lds_sync();
        if (cin == need) return prefix | ((shift > 0) ? ((1ull << shift) - 1ull) : 0ull);
    }
    return prefix;
}

// A bound for the selections during the scan, in one histogram pass: the
// keys' value parts (key >> 32) are binned in 256 bins of 2^sh values from
// the smallest one (sh the least shift that puts the largest one in bin 255),
// and the bound takes every key up to the end of the bin that holds the c-th
// smallest.  At least c keys (and so the c smallest) satisfy key <= bound; a
// few more may, which only keeps the threshold a little higher until the next
// selection (the final selection is exact).  Should more than c + 32 keys
// fall at or below it (values crowded into one bin), the exact radix
// selection decides instead.  ~0 when at most c keys are present.
template <int PE>
__device__ __forceinline__ uint64_t bin_bound(const uint64_t (&key)[PE], int c,
                                              uint32_t *__restrict__ hist, int lane) {
    int valid = 0;
    uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
    for (int e = 0; e < PE; ++e) {
        const bool v = key[e] != ~0ull;
        valid += __popcll(__ballot(v));
        const uint32_t u = (uint32_t)(key[e] >> 32);
        if (v) {
            lo = u < lo ? u : lo;
            hi = u > hi ? u : hi;
        }
    }
    if (valid <= c) return ~0ull;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const uint32_t ol = (uint32_t)__shfl_xor((int)lo, m), oh = (uint32_t)__shfl_xor((int)hi, m);
        lo = ol < lo ? ol : lo;
        hi = oh > hi ? oh : hi;
    }
    const uint32_t span = hi - lo;
    const int bits = span == 0u ? 0 : 32 - __clz((int)span);
    const int sh = bits > 8 ? bits - 8 : 0;
    ((uint4 *)hist)[lane] = uint4{0u, 0u, 0u, 0u};
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < PE; ++e)
        if (key[e] != ~0ull) atomicAdd(&hist[((uint32_t)(key[e] >> 32) - lo) >> sh], 1u);
    wave_lds_sync();
    int before, inbin;
    const int b = hist_find(hist, c, lane, &before, &inbin);
    wave_lds_sync();
    if (before + inbin > c + 32) return radix_kth<PE>(key, c, hist, lane);
    const uint64_t top = (uint64_t)lo + ((uint64_t)(b + 1) << sh) - 1ull;
    return ((top < 0xffffffffull ? top : 0xffffffffull) << 32) | 0xffffffffull;
}

// Keep the c smallest entries (final == true; during the scan at least the c
// smallest, see bin_bound) of one query's pool (four sub-pools of SUB
// entries, counts cg[0..3]).  Entries of the query's own index (leave-one-out)
// and of padding candidates (index >= n) are dropped here: the screen appends
// without checking them.  The kept entries go back to the sub-pools round
// robin (final == false) or to the LDS staging array in any order
// (final == true).  Returns the kept count; *kmax = largest kept key, or ~0
// if fewer than c were present (then every candidate seen so far is kept and
// no threshold exists yet).  With exactly c present the largest of them is
// the threshold: every entry dropped earlier, and every value never appended,
// lies at or above it.
template <int PE, int SUB>
__device__ __forceinline__ int select_pool(uint64_t *__restrict__ qpool, const int (&cg)[4], int c,
                                           uint32_t self, uint32_t n,
                                           uint32_t *__restrict__ hist,
                                           uint64_t *__restrict__ stage, bool final,
                                           uint64_t *kmax) {
    const int lane = lane_id();
    uint64_t key[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) {
        const int slot = lane * PE + e;
        const int g = slot / SUB, idx = slot % SUB;
        const int cnt = g == 0 ? cg[0] : g == 1 ? cg[1] : g == 2 ? cg[2] : cg[3];
        key[e] = ~0ull;
        if (idx < cnt) {
            const uint64_t r = qpool[g * SUB + idx];
            const uint32_t p = (uint32_t)(r >> 32);
            if (p != self && p < n) key[e] = raw_to_key(r);
        }
    }
    const uint64_t bound = final ? radix_kth<PE>(key, c, hist, lane) : bin_bound<PE>(key, c, hist, lane);
    const uint64_t lt = (1ull << lane) - 1ull;
    int base = 0;
    uint64_t mx = 0;
#pragma unroll
    for (int e = 0; e < PE; ++e) {
        const bool keep = key[e] != ~0ull && key[e] <= bound;
        const uint64_t m = __ballot(keep);
        if (keep) {
            const int pos = base + __popcll(m & lt);
            if (final)
                stage[pos] = key[e];
            else
                qpool[(pos & 3) * SUB + (pos >> 2)] = key_to_raw(key[e]);
            mx = key[e] > mx ? key[e] : mx;
        }
        base += __popcll(m);
    }
    const uint64_t mxall = wave_max_u64(mx);
    *kmax = (base < c) ? ~0ull : mxall;
    return base;
}

#ifndef FMG_SCREEN_TPB
#define FMG_SCREEN_TPB 4
#endif
#ifndef FMG_SCREEN_WGS
#define FMG_SCREEN_WGS 2
#endif

template <class Op, int KSTEPS, int CAP, bool PRUNE>
__global__ __launch_bounds__(256, FMG_SCREEN_WGS) void screen_kernel(ScreenArgs a) {
    constexpr int RB = 4 * KSTEPS * Op::BPS;  // row bytes
    constexpr int CH = RB / 16;               // 16-byte chunks per row
    constexpr int SWZ = (CH % 8 == 0) ? 7 : 3;  // chunk XOR swizzle (bank spread)
    constexpr int LDI = CH / 4;               // LDS-DMA loads per wave per tile
    constexpr int TPB = FMG_SCREEN_TPB;       // tiles per barrier period
    constexpr int SUB = CAP / 4;              // sub-pool per lane group
    constexpr int TRIG = SUB - 16;            // select when a sub-pool exceeds this (after a tile)
    constexpr int PE = CAP / 64;
    static_assert(CH % 4 == 0, "tile load split");
    // Candidate tiles: 64 rows x RB bytes, unpadded; 16-byte chunk c of row r
    // is stored at chunk position c ^ (r & SWZ).  Two rings of TPB tiles: one
    // is screened while LDS-DMA fills the other.
    __shared__ __align__(16) char ringA[TPB][TILE * RB];
    __shared__ __align__(16) char ringB[TPB][TILE * RB];
    __shared__ __align__(16) uint32_t hist_all[4][256];
    __shared__ __align__(16) uint64_t stage_all[4][SCREEN_CMAX];
    // Pruned scans: super-tiles some wave of the workgroup cannot skip (one
    // bit each), and their list in scan order.
    __shared__ uint32_t sup_keep[PRUNE ? SCREEN_SUPER_MAX / 32 : 1];
    __shared__ uint16_t sup_list[PRUNE ? SCREEN_SUPER_MAX : 1];
    // Pruned scans: per group of a quad (four groups of 16 tiles) the tiles
    // some wave needs (one bit each, OR over the waves; three buffers used in
    // turn), and each wave's own skip bits.
    __shared__ uint32_t need_q[PRUNE ? 3 : 1][4];
    __shared__ uint32_t my_skip[PRUNE ? 4 : 1][4];

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wq0 = (int)blockIdx.x * SCREEN_QPB + wave * 64;
    const int split = blockIdx.y;
    const int cb = split * (int)a.col_chunk;
    const int ce = (cb + a.col_chunk < a.n_pad) ? cb + (int)a.col_chunk : (int)a.n_pad;
    // Columns are visited at virtual positions v = 0, TILE, ... < len.
    // Without pruning: in order.  With pruning (one split, n_pad a multiple
    // of SCREEN_SUPER_ROWS) in two phases: first this workgroup's own
    // super-tile, starting at its own rows (the self-join's rows and columns
    // share one order; a prediction's start column comes from rot_tab) and
    // wrapping within the super-tile; then, in order after it, the other
    // super-tiles that some wave cannot skip with its thresholds at the end
    // of the first phase (sup_list).
    int len = ce - cb;
    int own_sup = 0, rot_t = 0;
    if constexpr (PRUNE) {
        const int start = a.rot_tab ? (int)(a.rot_tab[blockIdx.x] % (ce - cb))
                                    : (int)(((int64_t)blockIdx.x * SCREEN_QPB) % (ce - cb));
        own_sup = start / SCREEN_SUPER_ROWS;
        rot_t = ((start % SCREEN_SUPER_ROWS) / TILE) & ~(SCREEN_GROUP - 1);  // whole groups
        len = SCREEN_SUPER_ROWS;  // the first phase
        if (threadIdx.x < SCREEN_SUPER_MAX / 32) sup_keep[threadIdx.x] = 0u;
        if (threadIdx.x < 12) need_q[threadIdx.x / 4][threadIdx.x % 4] = 0u;
    }
    auto phys = [&](int v) -> int {
        if constexpr (!PRUNE) {
            return cb + v;
        } else {
            const int t = v / TILE;
            if (t < SCREEN_SUPER) return (own_sup * SCREEN_SUPER + ((rot_t + t) & (SCREEN_SUPER - 1))) * TILE;
            return ((int)sup_list[(t - SCREEN_SUPER) / SCREEN_SUPER] * SCREEN_SUPER +
                    (t & (SCREEN_SUPER - 1))) * TILE;
        }
    };
    const int n_real = (int)a.n, m_real = (int)a.m;
    const char *__restrict__ Pb = (const char *)a.P;
    uint32_t *hist = hist_all[wave];
    uint64_t *stage = stage_all[wave];

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
    // pool of query (wave query ql), sub-pool gg: pool + ((ql * 4) + gg) * SUB
    uint64_t *__restrict__ pool = a.pool + ((int64_t)split * a.m_pad + wq0) * CAP;
    // this lane's sub-pool of query tile t starts at mysub + t * 64 * SUB
    uint64_t *const mysub = pool + (r16 * 4 + g) * SUB;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int q = wq0 + t * 16 + r16;
        thr[t] = (q < m_real) ? INFINITY : -INFINITY;  // padding queries never append
        cnt[t] = 0;
    }

    // Tile loads go straight from global memory to LDS (global_load_lds):
    // wave w fills slots [w*LDI*64, (w+1)*LDI*64), lane l of load j writes slot
    // (w*LDI + j)*64 + l, i.e. row slot/CH, chunk position slot%CH.
    auto load_tile = [&](int col0, char *dst) {
#pragma unroll
        for (int j = 0; j < LDI; ++j) {
            const int slot = (wave * LDI + j) * 64 + lane;
            const int r = slot / CH, pc = slot % CH;
            const int c = pc ^ (r & SWZ);
            const char *src = Pb + (size_t)(col0 + r) * RB + c * 16;
            __builtin_amdgcn_global_load_lds(
                (const void *)src,
                (__attribute__((address_space(3))) void *)(dst + (wave * LDI + j) * 1024), 16, 0, 0);
        }
    };
    // This lane's fragment offsets inside a tile (row r16 of each 16-row block).
    int frag_off[KSTEPS];
#pragma unroll
    for (int s = 0; s < KSTEPS; ++s) {
        const int byte = g * KSTEPS * Op::BPS + s * Op::BPS;
        frag_off[s] = r16 * RB + (((byte >> 4) ^ (r16 & SWZ)) << 4) + (byte & 15);
    }

    // Tile pruning.  Every 16 tiles the wave screens their centroid rows
    // (8 MFMAs) and marks a tile skipped when for all of its 64 queries
    //   (||z~ - c~|| - r)^2 - ||z~||^2 - A > threshold   (with a margin),
    // where ||z~ - c~||^2 >= S'(c, z) + ||z~||^2 - A bounds the centroid
    // distance from below, r bounds every row of the tile around c~ (triangle
    // inequality), and A bounds the MFMA error of a screened value (centroid
    // norms are within 1.02 of the largest row norm).  Every row of a skipped
    // tile would therefore have screened above the threshold, which only
    // decreases: the kept keys, and the certificate's premise that every
    // non-candidate screened at or above T', are unchanged.
    float nzq[4], aq[4];
    const float margin_nx = (float)(1.0e-6 * a.nx_max);
    uint32_t skip16 = 0;
    if constexpr (PRUNE) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int q = wq0 + t * 16 + r16;
            nzq[t] = (q < m_real) ? a.nzq[q] : 0.0f;
            aq[t] = (float)(a.acc_coef * (2.01 * 1.02 * a.nx_max + (double)nzq[t]) +
                            1.0e-6 * 1.02 * a.nx_max);
        }
    }
    // Skip bits of 16 balls: ball_row(j) and ball_rad(j) give the centre row
    // and radius of ball j < 16 (a radius of +inf for a ball past the range:
    // never skipped).  The test is branch free (bitwise logic on the
    // comparisons, the hardware square root), which made it several times
    // cheaper than with short-circuit conditions.
    struct Balls {
        typename Op::frag_t af[KSTEPS];
        float rad[4];  // this lane's balls 4g + i
    };
    auto ball_load = [&](auto ball_row, auto ball_rad, Balls &b) {
        const char *crow = ball_row(r16);
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s)
            b.af[s] = Op::load(crow + g * KSTEPS * Op::BPS + s * Op::BPS);
#pragma unroll
        for (int i = 0; i < 4; ++i) b.rad[i] = ball_rad(4 * g + i);
    };
    auto ball_test = [&](const Balls &b) -> uint32_t {
        f32x4 ac[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            ac[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s) ac[t] = Op::mfma(b.af[s], bq[t][s], ac[t]);
        }
        uint32_t skip = 0xffffu;
        bool pad[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) pad[t] = thr[t] == -INFINITY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint64_t all = ~0ull;  // lanes whose query (of any query tile) can skip ball 4g + i
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // branch free; the square root is the hardware one (within
                // 1 ulp), whose error the margins cover many times over.  A
                // non-positive L gives dl <= 0: never skipped.
                const float L = ac[t][i] + nzq[t] - aq[t];
                const float dl = __builtin_amdgcn_sqrtf(fmaxf(L, 0.0f)) - b.rad[i];
                const float d2 = dl * dl;
                const bool pr = pad[t] |  // padding query
                                ((dl > 0.0f) &
                                 (d2 - nzq[t] - aq[t] - 1.0e-5f * (d2 + nzq[t]) - margin_nx > thr[t]));
                all &= __ballot(pr);
            }
#pragma unroll
            for (int gg = 0; gg < 4; ++gg)
                if (((all >> (16 * gg)) & 0xffffull) != 0xffffull) skip &= ~(1u << (4 * gg + i));
        }
        return skip;
    };
    auto ball_mask = [&](auto ball_row, auto ball_rad) -> uint32_t {
        Balls b;
        ball_load(ball_row, ball_rad, b);
        return ball_test(b);
    };
    // The 16 tiles at virtual positions v0 + j * TILE.
    auto prune_load = [&](int v0, Balls &b) {
        ball_load(
            [&](int j) {
                const int vr = v0 + j * TILE;
                return (const char *)a.tile_c + (int64_t)(phys(vr < len ? vr : 0) / TILE) * RB;
            },
            [&](int j) {
                const int vj = v0 + j * TILE;
                return vj < len ? a.tile_r[phys(vj) / TILE] : INFINITY;
            },
            b);
    };
    auto prune_mask = [&](int v0) -> uint32_t {
        Balls b;
        prune_load(v0, b);
        return ball_test(b);
    };

    // Counts of the four sub-pools of wave query (t, rl).
    auto counts = [&](int t, int rl, int (&cg)[4]) {
        const int ct = t == 0 ? cnt[0] : t == 1 ? cnt[1] : t == 2 ? cnt[2] : cnt[3];
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) cg[gg] = __builtin_amdgcn_readlane(ct, rl + 16 * gg);
    };

    // Select in every query of the wave with a sub-pool above the trigger.
    auto flush_full = [&]() {
        for (int t = 0; t < 4; ++t) {
            const int ct = t == 0 ? cnt[0] : t == 1 ? cnt[1] : t == 2 ? cnt[2] : cnt[3];
            const uint64_t m = __ballot(ct > TRIG);
            uint64_t need = (m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xffffull;
            while (need != 0) {
                const int rl = __ffsll((long long)need) - 1;
                need &= need - 1;
                int cg[4];
                counts(t, rl, cg);
                uint64_t kmax;
                const uint32_t self = a.loo ? (uint32_t)(wq0 + t * 16 + rl) : 0xffffffffu;
                const int kept = select_pool<PE, SUB>(pool + (t * 16 + rl) * 4 * SUB, cg, a.c, self,
                                                      (uint32_t)n_real, hist, stage, false, &kmax);
                if (r16 == rl) {
                    const int nc = (kept + 3 - g) >> 2;
                    const float nt = skey_val(kmax);
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt) {
                        if (tt == t) {
                            cnt[tt] = nc;
                            if (kmax != ~0ull) thr[tt] = nt;
                        }
                    }
                }
            }
        }
    };

    // MFMA screen of one tile and candidate selection.
    auto screen_tile = [&](int col, const char *cur, int j16) {
        if constexpr (PRUNE) {
            if ((skip16 >> j16) & 1u) return;
        }
        f32x4 acc[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[t][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (std::is_same<Op, OpBF16>::value && KSTEPS == 2 && RB == 128) {
            // The eight 16-byte fragments of the tile in one asm block that
            // also waits for them.  Read through the compiler, every tile
            // read would first wait for all vector memory operations in
            // flight (the next period's LDS-DMA loads and this wave's pool
            // appends), since the compiler cannot tell the DMA's LDS target
            // from the ring being read.  The ring read here was filled before
            // the last period's barrier, which waited for its loads.
            const uint32_t base =
                (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)cur;
            uint4 f0, f1, f2, f3, f4, f5, f6, f7;
            asm volatile(
                "ds_read_b128 %0, %8\n\t"
                "ds_read_b128 %1, %8 offset:2048\n\t"
                "ds_read_b128 %2, %8 offset:4096\n\t"
                "ds_read_b128 %3, %8 offset:6144\n\t"
                "ds_read_b128 %4, %9\n\t"
                "ds_read_b128 %5, %9 offset:2048\n\t"
                "ds_read_b128 %6, %9 offset:4096\n\t"
                "ds_read_b128 %7, %9 offset:6144\n\t"
                "s_waitcnt lgkmcnt(0)"
                : "=&v"(f0), "=&v"(f1), "=&v"(f2), "=&v"(f3), "=&v"(f4), "=&v"(f5), "=&v"(f6),
                  "=&v"(f7)
                : "v"(base + (uint32_t)frag_off[0]), "v"(base + (uint32_t)frag_off[1])
                : "memory");
            static_assert(16 * RB == 2048, "fragment offsets of the asm block");
            const bf16x8 a0[4] = {__builtin_bit_cast(bf16x8, f0), __builtin_bit_cast(bf16x8, f1),
                                  __builtin_bit_cast(bf16x8, f2), __builtin_bit_cast(bf16x8, f3)};
            const bf16x8 a1[4] = {__builtin_bit_cast(bf16x8, f4), __builtin_bit_cast(bf16x8, f5),
                                  __builtin_bit_cast(bf16x8, f6), __builtin_bit_cast(bf16x8, f7)};
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) acc[t][mt] = Op::mfma(a0[mt], bq[t][0], acc[t][mt]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) acc[t][mt] = Op::mfma(a1[mt], bq[t][1], acc[t][mt]);
        } else {
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s) {
                typename Op::frag_t af[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) af[mt] = Op::load(cur + mt * 16 * RB + frag_off[s]);
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[t][mt] = Op::mfma(af[mt], bq[t][s], acc[t][mt]);
            }
        }

        // Candidate selection.  For each query tile t a lane holds 16 values
        // of its query (4 candidate tiles x 4 rows); their minimum (a chain of
        // v_min3, no canonicalisation: the file is built without IEEE mode,
        // every screened value being finite) is tested against the query's
        // threshold, so a query tile whose candidates all fail costs one
        // wave-wide branch.  Otherwise all 16 comparisons are made at once,
        // each into a wave mask of its own, and each mask that has a lane set
        // becomes the execution mask of one append (a lane appends to its own
        // sub-pool): the comparisons do not wait on one another, and the
        // appends cost scalar branches only.  The query's own index and
        // padding candidates may be appended here; the selection drops them.
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float th = thr[t];
            float m16 = acc[t][0][0];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = (mt == 0 ? 1 : 0); i < 4; ++i) m16 = fminf(m16, acc[t][mt][i]);
            if (__ballot(m16 <= th) == 0) continue;
            uint64_t B[16];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) B[mt * 4 + i] = __ballot(acc[t][mt][i] <= th);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (__builtin_amdgcn_inverse_ballot_w64(B[mt * 4 + i])) {
                        const uint32_t p = (uint32_t)(col + mt * 16 + g * 4 + i);
                        mysub[(uint32_t)(t * 64 * SUB) + (uint32_t)cnt[t]] =
                            raw_entry(acc[t][mt][i], p);
                        cnt[t] += 1;
                    }
                }
        }
    };

    // One barrier period: LDS-DMA of the next period's TPB tiles into `nxt`
    // while this period's tiles in `cur` are screened (a period of compute
    // covers the load latency); then pool maintenance and one workgroup
    // barrier.
    auto period = [&](int v, char (*cur)[TILE * RB], char (*nxt)[TILE * RB]) {
#pragma unroll
        for (int j = 0; j < TPB; ++j)
            if (v + (TPB + j) * TILE < len) load_tile(phys(v + (TPB + j) * TILE), nxt[j]);
        if constexpr (PRUNE) {
            if ((v & (16 * TILE - 1)) == 0) skip16 = prune_mask(v);
        }
#pragma unroll 1
        for (int j = 0; j < TPB; ++j)
            if (v + j * TILE < len) {
                screen_tile(phys(v + j * TILE), cur[j], ((v >> 6) + j) & 15);
                if (__ballot(cnt[0] > TRIG || cnt[1] > TRIG || cnt[2] > TRIG || cnt[3] > TRIG) != 0)
                    flush_full();
            }
        // the next period's tiles must have landed in LDS before any wave reads them
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    };

    // Pruned scans go a super-tile, then a quad of four groups, then a group
    // of 16 tiles at a time.  Super-tiles start at multiples of
    // SCREEN_SUPER_ROWS and groups at multiples of SCREEN_GROUP_ROWS (virtual
    // and physical positions alike), so the group balls line up with the
    // scan.  At a super-tile's start every wave tests its 16 group balls.  At
    // a quad's start every wave computes the skip bits of its needed groups'
    // tiles and the workgroup ORs the tiles some wave needs per group (one
    // barrier per quad); only those are loaded, and a group no wave needs
    // costs nothing.  (Loading the four groups' centre rows and radii
    // together, ahead of their tests, spilled registers and was slower.)
    // Within a group the periods run as in the full scan, the next period's
    // needed tiles loading while the current one is screened.
    int qc = 0;  // quads entered, for the need_q buffers
    auto run_groups = [&](int v_begin) {
        uint32_t gmine = 0u;
        int qb = 0;
        for (int v0 = v_begin; v0 < len; v0 += SCREEN_GROUP_ROWS) {
            const int jg = (v0 / SCREEN_GROUP_ROWS) & (SCREEN_GROUP - 1);
            if (jg == 0) {
                gmine = ~ball_mask(
                            [&](int j) {
                                return (const char *)a.grp_c +
                                       (int64_t)(phys(v0 + j * SCREEN_GROUP_ROWS) /
                                                 SCREEN_GROUP_ROWS) * RB;
                            },
                            [&](int j) {
                                return a.grp_r[phys(v0 + j * SCREEN_GROUP_ROWS) /
                                               SCREEN_GROUP_ROWS];
                            }) &
                        0xffffu;
            }
            if ((jg & 3) == 0) {
                qb = qc % 3;
#pragma unroll 1
                for (int u = 0; u < 4; ++u) {
                    const uint32_t sk =
                        ((gmine >> (jg + u)) & 1u) ? prune_mask(v0 + u * SCREEN_GROUP_ROWS) : 0xffffu;
                    if (lane == 0) {
                        my_skip[wave][u] = sk;
                        if (sk != 0xffffu) atomicOr(&need_q[qb][u], ~sk & 0xffffu);
                    }
                }
                __syncthreads();
                // the buffer of two quads ago: read before this barrier, next
                // written after the next quad's barrier
                if (threadIdx.x < 4) need_q[(qc + 2) % 3][threadIdx.x] = 0u;
                ++qc;
            }
            const uint32_t need = need_q[qb][jg & 3];
            if (need == 0u) continue;
            skip16 = my_skip[wave][jg & 3];
            auto load_period = [&](int vp, char (*dst)[TILE * RB]) {
#pragma unroll
                for (int j = 0; j < TPB; ++j) {
                    const int t = ((vp - v0) >> 6) + j;
                    if (vp + j * TILE < len && ((need >> t) & 1u)) load_tile(phys(vp + j * TILE), dst[j]);
                }
            };
            load_period(v0, ringA);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
#pragma unroll 1
            for (int p = 0; p < 16 / TPB; ++p) {
                const int vp = v0 + p * TPB * TILE;
                char(*cur)[TILE * RB] = (p & 1) ? ringB : ringA;
                char(*nxt)[TILE * RB] = (p & 1) ? ringA : ringB;
                if (p + 1 < 16 / TPB) load_period(vp + TPB * TILE, nxt);
#pragma unroll 1
                for (int j = 0; j < TPB; ++j)
                    if (vp + j * TILE < len) {
                        screen_tile(phys(vp + j * TILE), cur[j], ((vp >> 6) + j) & 15);
                        if (__ballot(cnt[0] > TRIG || cnt[1] > TRIG || cnt[2] > TRIG || cnt[3] > TRIG) != 0)
                            flush_full();
                    }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
            }
        }
    };
    if constexpr (!PRUNE) {
#pragma unroll
        for (int j = 0; j < TPB; ++j)
            if (j * TILE < len) load_tile(phys(j * TILE), ringA[j]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        for (int v = 0; v < len; v += 2 * TPB * TILE) {
            period(v, ringA, ringB);
            if (v + TPB * TILE < len) period(v + TPB * TILE, ringB, ringA);
        }
    } else {
        __syncthreads();  // the LDS words above are cleared
        run_groups(0);
        // Second phase: every wave marks the super-tiles it cannot skip with
        // its current thresholds (which only fall, so a super-tile skipped
        // now holds no candidate for any later threshold either); the kept
        // ones after the own super-tile, in order and wrapping, are scanned.
        const int nsup = (int)((ce - cb) / SCREEN_SUPER_ROWS);
        for (int s0 = 0; s0 < nsup; s0 += 16) {
            const uint32_t skip = ball_mask(
                [&](int j) {
                    const int sj = s0 + j < nsup ? s0 + j : s0;
                    return (const char *)a.sup_c + (int64_t)sj * RB;
                },
                [&](int j) { return s0 + j < nsup ? a.sup_r[s0 + j] : INFINITY; });
            const uint32_t keep = ~skip & 0xffffu;
            if (lane == 0 && keep) atomicOr(&sup_keep[s0 / 32], keep << (s0 & 31));
        }
        __syncthreads();
        if (wave == 0) {
            // list: own + 1, ..., nsup - 1, then 0, ..., own - 1 (lane w
            // counts word w; two exclusive scans place the indices)
            int total = 0;
            for (int part = 0; part < 2; ++part) {
                for (int w0 = 0; w0 < SCREEN_SUPER_MAX / 32; w0 += 64) {
                    const int w = w0 + lane;
                    uint32_t bits = 0u;
                    if (w * 32 < nsup) {
                        bits = sup_keep[w];
                        for (int b = 0; b < 32; ++b) {
                            const int sidx = w * 32 + b;
                            const bool in = sidx < nsup && sidx != own_sup &&
                                            (part == 0 ? sidx > own_sup : sidx < own_sup);
                            if (!in) bits &= ~(1u << b);
                        }
                    }
                    const int cnt = __popc(bits);
                    const int incl = wave_incl_scan(cnt, lane);
                    int pos = total + incl - cnt;
                    while (bits) {
                        const int b = __ffs(bits) - 1;
                        bits &= bits - 1;
                        sup_list[pos++] = (uint16_t)(w * 32 + b);
                    }
                    total += __builtin_amdgcn_readlane(incl, 63);
                }
            }
            if (lane == 0) sup_keep[0] = (uint32_t)total;  // the count, for every wave
        }
        __syncthreads();
        const int kept = (int)sup_keep[0];
        len = SCREEN_SUPER_ROWS * (1 + kept);
        run_groups(SCREEN_SUPER_ROWS);
    }

    // Final selection, sort and output of every real query of this wave.
    for (int ql = 0; ql < 64; ++ql) {
        const int q = wq0 + ql;
        if (q >= m_real) break;
        int cg[4];
        counts(ql >> 4, ql & 15, cg);
        uint64_t kmax;
        const uint32_t self = a.loo ? (uint32_t)q : 0xffffffffu;
        const int kept = select_pool<PE, SUB>(pool + ql * 4 * SUB, cg, a.c, self, (uint32_t)n_real,
                                              hist, stage, true, &kmax);
        wave_lds_sync();
        constexpr int E2 = SCREEN_CMAX / 64;
        uint64_t key[E2];
#pragma unroll
        for (int e = 0; e < E2; ++e) {
            const int slot = lane * E2 + e;
            key[e] = slot < kept ? stage[slot] : ~0ull;
        }
        wave_sort_u64<E2>(key);
        uint64_t *__restrict__ out = a.cand + ((int64_t)split * a.m + q) * a.c;
#pragma unroll
        for (int e = 0; e < E2; ++e) {
            const int slot = lane * E2 + e;
            if (slot < a.c) out[slot] = key[e];
        }
        if (lane == 0)
            a.tq[(int64_t)split * a.m + q] = (kmax != ~0ull) ? skey_val(kmax) : INFINITY;
        wave_lds_sync();
    }
}

}  // namespace

// A pruned screen: one split over whole super-tiles, with every bound array.
bool pruned_args_ok(const ScreenArgs &a) {
    return a.splits == 1 && a.col_chunk >= a.n_pad && a.tile_c && a.tile_r && a.sup_c &&
           a.sup_r && a.grp_c && a.grp_r && a.nzq && a.n_pad % SCREEN_SUPER_ROWS == 0 &&
           a.n_pad / SCREEN_SUPER_ROWS <= SCREEN_SUPER_MAX;
}

template <int CAP>
hipError_t launch_screen_cap(const ScreenGeom &g, const ScreenArgs &a, hipStream_t s) {
    dim3 grid((unsigned)(a.m_pad / SCREEN_QPB), (unsigned)a.splits);
#define FMG_SCREEN_LAUNCH(OP, KS) \
    hipLaunchKernelGGL((screen_kernel<OP, KS, CAP, false>), grid, dim3(256), 0, s, a)
#define FMG_SCREEN_LAUNCH_PRUNED(OP, KS) \
    hipLaunchKernelGGL((screen_kernel<OP, KS, CAP, true>), grid, dim3(256), 0, s, a)
    if (g.mode == SCREEN_BF16) {
        if (g.ksteps != 2) return hipErrorInvalidValue;
        if (a.prune) {
            if (!pruned_args_ok(a)) return hipErrorInvalidValue;
            FMG_SCREEN_LAUNCH_PRUNED(OpBF16, 2);
        } else {
            FMG_SCREEN_LAUNCH(OpBF16, 2);
        }
    } else if (a.prune) {
        if (!pruned_args_ok(a)) return hipErrorInvalidValue;
        switch (g.ksteps) {
        case 4: FMG_SCREEN_LAUNCH_PRUNED(OpF32, 4); break;
        case 8: FMG_SCREEN_LAUNCH_PRUNED(OpF32, 8); break;
        case 12: FMG_SCREEN_LAUNCH_PRUNED(OpF32, 12); break;
        case 16: FMG_SCREEN_LAUNCH_PRUNED(OpF32, 16); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (g.ksteps) {
        case 4: FMG_SCREEN_LAUNCH(OpF32, 4); break;
        case 8: FMG_SCREEN_LAUNCH(OpF32, 8); break;
        case 12: FMG_SCREEN_LAUNCH(OpF32, 12); break;
        case 16: FMG_SCREEN_LAUNCH(OpF32, 16); break;
        default: return hipErrorInvalidValue;
        }
    }
#undef FMG_SCREEN_LAUNCH
#undef FMG_SCREEN_LAUNCH_PRUNED
    return hipGetLastError();
}

hipError_t launch_screen(const ScreenGeom &g, const ScreenArgs &a, hipStream_t s) {
    if (a.c < 1 || a.c > SCREEN_CMAX) return hipErrorInvalidValue;
    return a.c <= SCREEN_CAP_SMALL_C ? launch_screen_cap<SCREEN_CAP_SMALL>(g, a, s)
                                     : launch_screen_cap<SCREEN_CAP>(g, a, s);
}

}  // namespace fmg
