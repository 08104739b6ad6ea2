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

// Four 16-byte LDS reads at addr, addr + OFF, addr + 2 OFF, addr + 3 OFF,
// waited for inside the asm block (so no result is used, and no register is
// reused, before its read has landed).
template <int OFF>
__device__ __forceinline__ void lds_read4(uint32_t addr, uint4 &r0, uint4 &r1, uint4 &r2,
                                          uint4 &r3) {
    asm volatile(
        "ds_read_b128 %0, %4\n\t"
        "ds_read_b128 %1, %4 offset:%5\n\t"
        "ds_read_b128 %2, %4 offset:%6\n\t"
        "ds_read_b128 %3, %4 offset:%7\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
        : "v"(addr), "i"(OFF), "i"(2 * OFF), "i"(3 * OFF)
        : "memory");
}

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

    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4, r16 = lane & 15;
    const int wq0 = (int)blockIdx.x * SCREEN_QPB + wave * 64;
    const int split = blockIdx.y;
    const int cb = split * (int)a.col_chunk;
    const int ce = (cb + a.col_chunk < a.n_pad) ? cb + (int)a.col_chunk : (int)a.n_pad;
    // Without pruning the workgroup visits the columns of its range in order,
    // every wave screening every tile.  With pruning (one split, n_pad a
    // multiple of SCREEN_SUPER_ROWS) every wave scans on its own, in two
    // phases: first the workgroup's own super-tile, starting at its own group
    // (the self-join's rows and columns share one order; a prediction's start
    // column comes from rot_tab) and wrapping within the super-tile; then the
    // other super-tiles in order after it, wrapping.
    const int len = ce - cb;
    int own_sup = 0, rot_g = 0;
    if constexpr (PRUNE) {
        const int start = a.rot_tab ? (int)(a.rot_tab[blockIdx.x] % (ce - cb))
                                    : (int)(((int64_t)blockIdx.x * SCREEN_QPB) % (ce - cb));
        own_sup = start / SCREEN_SUPER_ROWS;
        rot_g = (start % SCREEN_SUPER_ROWS) / SCREEN_GROUP_ROWS;
    }
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

    // Tile loads go straight from global memory to LDS (global_load_lds).
    // Loads j0 .. j0 + nj - 1 of a tile's CH (lane l of load j writes slot
    // j*64 + l, i.e. row slot/CH, chunk position slot%CH): a full scan's waves
    // share each tile (wave w issues loads w*LDI ..), a pruned scan's wave
    // loads its own tiles whole.
    auto load_tile_part = [&](int col0, char *dst, int j0, int nj) __attribute__((always_inline)) {
#pragma unroll
        for (int j = j0; j < j0 + nj; ++j) {
            const int slot = j * 64 + lane;
            const int r = slot / CH, pc = slot % CH;
            const int c = pc ^ (r & SWZ);
            const char *src = Pb + (size_t)(col0 + r) * RB + c * 16;
            __builtin_amdgcn_global_load_lds(
                (const void *)src, (__attribute__((address_space(3))) void *)(dst + j * 1024), 16, 0,
                0);
        }
    };
    auto load_tile = [&](int col0, char *dst) { load_tile_part(col0, dst, wave * LDI, LDI); };
    // A lane's fragment offsets inside a tile (row l % 16 of each 16-row
    // block).  The tile reads form them afresh from a lane index that the
    // compiler cannot see through: kept live across the scan they were
    // spilled, and their reload from scratch, coming after the next tile's
    // LDS-DMA load was issued, made every tile wait for that load.
    auto frag_offsets = [&](int (&off)[KSTEPS]) __attribute__((always_inline)) {
        int ln = lane_id();
        asm volatile("" : "+v"(ln));
        const int r = ln & 15, gg = ln >> 4;
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s) {
            const int byte = gg * KSTEPS * Op::BPS + s * Op::BPS;
            off[s] = r * RB + (((byte >> 4) ^ (r & SWZ)) << 4) + (byte & 15);
        }
    };

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
    auto ball_load = [&](auto ball_row, auto ball_rad, Balls &b) __attribute__((always_inline)) {
        const char *crow = ball_row(r16);
#pragma unroll
        for (int s = 0; s < KSTEPS; ++s)
            b.af[s] = Op::load(crow + g * KSTEPS * Op::BPS + s * Op::BPS);
#pragma unroll
        for (int i = 0; i < 4; ++i) b.rad[i] = ball_rad(4 * g + i);
    };
    auto ball_test = [&](const Balls &b) __attribute__((always_inline)) -> uint32_t {
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
    auto ball_mask = [&](auto ball_row, auto ball_rad) __attribute__((always_inline)) -> uint32_t {
        Balls b;
        ball_load(ball_row, ball_rad, b);
        return ball_test(b);
    };
    // Skip bits of the 16 tiles t0 .. t0 + 15, of the 16 groups g0 .. g0 + 15
    // (a super-tile's), and of the 16 super-tiles s(0) .. s(15).
    auto tile_mask = [&](int t0) __attribute__((always_inline)) -> uint32_t {
        return ball_mask([&](int j) { return (const char *)a.tile_c + (int64_t)(t0 + j) * RB; },
                         [&](int j) { return a.tile_r[t0 + j]; });
    };
    auto group_mask = [&](int g0) __attribute__((always_inline)) -> uint32_t {
        return ball_mask([&](int j) { return (const char *)a.grp_c + (int64_t)(g0 + j) * RB; },
                         [&](int j) { return a.grp_r[g0 + j]; });
    };

    // Counts of the four sub-pools of wave query (t, rl).
    auto counts = [&](int t, int rl, int (&cg)[4]) {
        const int ct = t == 0 ? cnt[0] : t == 1 ? cnt[1] : t == 2 ? cnt[2] : cnt[3];
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) cg[gg] = __builtin_amdgcn_readlane(ct, rl + 16 * gg);
    };

    // Select in every query of the wave with a sub-pool above the trigger.
    auto flush_full = [&]() __attribute__((always_inline)) {
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
    auto screen_tile = [&](int col, const char *cur) __attribute__((always_inline)) {
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
            int frag_off[KSTEPS];
            frag_offsets(frag_off);
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
            // FP32 rows: k-steps 4q .. 4q + 3 of candidate block mt are one
            // 16-byte chunk (frag_off[4q]); the four blocks' chunks of each q
            // are read in one asm block, for the same reason as above.
            static_assert(KSTEPS % 4 == 0, "whole 16-byte chunks per lane");
            const uint32_t base =
                (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)cur;
            int frag_off[KSTEPS];
            frag_offsets(frag_off);
            float af[4][KSTEPS];
#pragma unroll
            for (int q = 0; q < KSTEPS / 4; ++q) {
                uint4 f[4];
                lds_read4<16 * RB>(base + (uint32_t)frag_off[4 * q], f[0], f[1], f[2], f[3]);
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    af[mt][4 * q] = __uint_as_float(f[mt].x);
                    af[mt][4 * q + 1] = __uint_as_float(f[mt].y);
                    af[mt][4 * q + 2] = __uint_as_float(f[mt].z);
                    af[mt][4 * q + 3] = __uint_as_float(f[mt].w);
                }
            }
#pragma unroll
            for (int s = 0; s < KSTEPS; ++s)
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
                        acc[t][mt] = Op::mfma(af[mt][s], bq[t][s], acc[t][mt]);
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
            if (v + (TPB + j) * TILE < len) load_tile(cb + v + (TPB + j) * TILE, nxt[j]);
#pragma unroll 1
        for (int j = 0; j < TPB; ++j)
            if (v + j * TILE < len) {
                screen_tile(cb + v + j * TILE, cur[j]);
                if (__ballot(cnt[0] > TRIG || cnt[1] > TRIG || cnt[2] > TRIG || cnt[3] > TRIG) != 0)
                    flush_full();
            }
        // the next period's tiles must have landed in LDS before any wave reads them
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    };

    if constexpr (!PRUNE) {
#pragma unroll
        for (int j = 0; j < TPB; ++j)
            if (j * TILE < len) load_tile(cb + j * TILE, ringA[j]);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        for (int v = 0; v < len; v += 2 * TPB * TILE) {
            period(v, ringA, ringB);
            if (v + TPB * TILE < len) period(v + TPB * TILE, ringB, ringA);
        }
    } else {
        // Pruned scan, every wave on its own: no workgroup barrier, so a wave
        // busy with a selection holds up no other.  The wave goes a super-tile,
        // then a group of 16 tiles, at a time: at a super-tile it tests the 16
        // group balls, at a needed group the 16 tile balls (thresholds as they
        // stand then), and it loads and screens only the tiles it needs,
        // through two LDS slots of its own: a tile's load is issued before
        // the previous tile is screened.  In the second phase the super-tile
        // balls are tested 16 at a time ahead of the scan; thresholds only
        // fall, so a ball skipped with a threshold holds no candidate for any
        // later one either.
        static_assert(TPB == 4, "a wave's two slots are ringA[wave] and ringB[wave]");
        int pend = -1, ps = 0;  // the tile in flight (not yet screened) and its slot
        auto screen_pending = [&]() __attribute__((always_inline)) {
            screen_tile(pend * TILE, ps ? ringB[wave] : ringA[wave]);
            if (__ballot(cnt[0] > TRIG || cnt[1] > TRIG || cnt[2] > TRIG || cnt[3] > TRIG) != 0)
                flush_full();
        };
        auto visit = [&](int tile) __attribute__((always_inline)) {
            if (pend >= 0) {
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the pending tile has landed
                load_tile_part(tile * TILE, ps ? ringA[wave] : ringB[wave], 0, CH);
                screen_pending();
                ps ^= 1;
            } else {
                load_tile_part(tile * TILE, ps ? ringB[wave] : ringA[wave], 0, CH);
            }
            pend = tile;
        };
        auto scan_group = [&](int gidx) __attribute__((always_inline)) {
            uint32_t need = ~tile_mask(gidx * SCREEN_GROUP) & 0xffffu;
            while (need != 0u) {
                const int j = __ffs(need) - 1;
                need &= need - 1u;
                visit(gidx * SCREEN_GROUP + j);
            }
        };
        // first phase: the own super-tile from the own group, wrapping
#pragma unroll 1
        for (int jj = 0; jj < SCREEN_GROUP; ++jj)
            scan_group(own_sup * SCREEN_GROUP + ((rot_g + jj) & (SCREEN_GROUP - 1)));
        // second phase: the other super-tiles, in order after the own one
        const int nsup = (int)((ce - cb) / SCREEN_SUPER_ROWS);
#pragma unroll 1
        for (int q0 = 1; q0 < nsup; q0 += 16) {
            auto sidx = [&](int j) {
                const int sj = own_sup + q0 + j;
                return sj < nsup ? sj : sj - nsup;
            };
            uint32_t sneed =
                ~ball_mask([&](int j) {
                    return (const char *)a.sup_c + (int64_t)(q0 + j < nsup ? sidx(j) : own_sup) * RB;
                },
                           [&](int j) { return q0 + j < nsup ? a.sup_r[sidx(j)] : -1.0e18f; }) &
                0xffffu;
            while (sneed != 0u) {
                const int j = __ffs(sneed) - 1;
                sneed &= sneed - 1u;
                const int sup = sidx(j);
                uint32_t gneed = ~group_mask(sup * SCREEN_GROUP) & 0xffffu;
                while (gneed != 0u) {
                    const int jg = __ffs(gneed) - 1;
                    gneed &= gneed - 1u;
                    scan_group(sup * SCREEN_GROUP + jg);
                }
            }
        }
        if (pend >= 0) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            screen_pending();
        }
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
