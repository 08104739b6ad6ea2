// Tile pruning for the build's neighbour screen (Algorithm 2, the
// training-point neighbour lookups): an order of the training points in which
// 64-row candidate tiles are compact, and per tile a ball that bounds its
// rows, so that the screen can skip tiles no query of a wave can take.
//
//   1. P pivots (evenly spaced training points), labelled along a greedy
//      nearest-neighbour chain so that consecutive labels are close, and the
//      nearest pivot of every point (FP32 distances of the centred
//      coordinates; any assignment is correct, a good one makes tiles
//      compact);
//   2. a stable sort by pivot label (a one-pass counting sort: per-tile label
//      counts, their exclusive scan in (label, tile) order, and an in-order
//      scatter), giving the permutation perm: position i of the screen holds
//      point perm[i]; the cells of one cluster form a run;
//   3. the screening rows gathered into that order, with the query norms;
//   4. per tile of 64 rows: the centroid of its screening rows (BF16 or
//      FP32), itself rounded to the row's format (so it is an exact point of
//      the screened space) and written as a candidate row, and the FP64
//      radius max ||x~ - c~|| over the tile's real rows, rounded up;
//   5. the re-rank takes the rows in the same order and maps each
//      candidate's index back to its training index, so that the certificate
//      runs unchanged.
#include "fmg_device.h"
#include "fmg_kernels.h"

namespace fmg {

namespace {

// Sort key of points Pts [n, d]: the label of the nearest pivot in the top
// 8 bits and, for low-dimensional data, a Morton code of the centred
// coordinates in the low 24 bits, so that the points of one cell are ordered
// along a space-filling curve and 64 consecutive points form a compact tile.
// Pivot j is training row j * stride of X.  Coordinates are zero padded to
// DP (a multiple of 16 covering d), so the loop has no guards and reads each
// pivot row as 16-byte vectors.  The nearest pivot minimises
// ||p_j||^2 - 2 x.p_j (||x||^2 is common to all j): one FMA per coordinate.
// Any assignment and any order serve the pruning (the tile radii are
// measured on the tiles' actual rows), so the rounding of this form is
// harmless.  box (nullable): per coordinate the low end and 2^bits / width
// of the training points' centred bounding box; bits = Morton bits per
// coordinate (bits * d <= 24).
template <int DP>
__global__ __launch_bounds__(256) void pivot_assign_kernel(const float *__restrict__ X,
                                                           const float *__restrict__ Pts,
                                                           int64_t n, int d,
                                                           const float *__restrict__ mu, int P,
                                                           int64_t stride,
                                                           const int32_t *__restrict__ label,
                                                           const float *__restrict__ box,
                                                           int bits,
                                                           uint32_t *__restrict__ key) {
    extern __shared__ __align__(16) float piv[];  // [P, DP] centred pivots, zero past d; [P] norms
    float *pn = piv + P * DP;
    for (int e = threadIdx.x; e < P * DP; e += blockDim.x) {
        const int j = e / DP, c = e % DP;
        piv[e] = c < d ? X[(int64_t)j * stride * d + c] - mu[c] : 0.0f;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < P; j += blockDim.x) {
        float s = 0.0f;
        for (int c = 0; c < DP; ++c) s = fmaf(piv[j * DP + c], piv[j * DP + c], s);
        pn[j] = s;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[DP];
#pragma unroll
    for (int c = 0; c < DP; ++c) x[c] = c < d ? Pts[i * d + c] - mu[c] : 0.0f;
    float best = INFINITY;
    uint32_t bj = 0;
    for (int j = 0; j < P; ++j) {
        const float4 *pj = (const float4 *)(piv + j * DP);
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
#pragma unroll
        for (int c4 = 0; c4 < DP / 4; ++c4) {
            const float4 v = pj[c4];
            s0 = fmaf(x[4 * c4], v.x, s0);
            s1 = fmaf(x[4 * c4 + 1], v.y, s1);
            s2 = fmaf(x[4 * c4 + 2], v.z, s2);
            s3 = fmaf(x[4 * c4 + 3], v.w, s3);
        }
        const float sj = fmaf(-2.0f, (s0 + s1) + (s2 + s3), pn[j]);
        if (sj < best) {
            best = sj;
            bj = (uint32_t)j;
        }
    }
    uint32_t code = 0;
    if (box && bits > 0) {
        const uint32_t top = (1u << bits) - 1u;
        uint32_t q[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            q[c] = 0u;
            if (c < d) {
                const float t = (x[c < DP ? c : 0] - box[c]) * box[64 + c];
                q[c] = t <= 0.0f ? 0u : (t >= (float)top ? top : (uint32_t)t);
            }
        }
        for (int b = bits - 1; b >= 0; --b)
            for (int c = 0; c < d; ++c) code = (code << 1) | ((q[c] >> b) & 1u);
    }
    key[i] = ((uint32_t)label[bj] << 24) | code;
}

// Pivot labels along a greedy nearest-neighbour chain (pivot 0 first, then
// repeatedly the nearest unlabelled pivot, ties to the smaller pivot), so
// that pivots with consecutive labels are close and the cells of one cluster
// form a run of the order.  One workgroup of 256 threads, thread j holding
// pivot j (P <= 256).
__global__ __launch_bounds__(256) void pivot_chain_kernel(const float *__restrict__ X, int d,
                                                          const float *__restrict__ mu, int P,
                                                          int64_t stride,
                                                          int32_t *__restrict__ label) {
    __shared__ float piv[256 * 64];
    __shared__ uint64_t best[4];
    __shared__ int cur_sh;
    const int j = threadIdx.x;
    for (int e = j; e < P * 64; e += 256) {
        const int q = e / 64, c = e % 64;
        piv[e] = c < d ? X[(int64_t)q * stride * d + c] - mu[c] : 0.0f;
    }
    bool used = j >= P;
    if (j == 0) {
        label[0] = 0;
        cur_sh = 0;
    }
    if (j == 0) used = true;
    __syncthreads();
    for (int step = 1; step < P; ++step) {
        const int cur = cur_sh;
        float s = 0.0f;
        for (int c = 0; c < d; ++c) {
            const float t = piv[j * 64 + c] - piv[cur * 64 + c];
            s = fmaf(t, t, s);
        }
        // key: distance bits, then pivot index (non-negative floats order as integers)
        uint64_t key = used ? ~0ull : (((uint64_t)__float_as_uint(s)) << 32) | (uint32_t)j;
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) {
            const uint64_t o = ((uint64_t)(uint32_t)__shfl_xor((int)(key >> 32), w) << 32) |
                               (uint32_t)__shfl_xor((int)(uint32_t)key, w);
            key = o < key ? o : key;
        }
        if ((j & 63) == 0) best[j >> 6] = key;
        __syncthreads();
        if (j == 0) {
            uint64_t b = best[0];
            for (int w = 1; w < 4; ++w) b = best[w] < b ? best[w] : b;
            const int nxt = (int)(uint32_t)b;
            label[nxt] = step;
            cur_sh = nxt;
        }
        __syncthreads();
        if (j == cur_sh) used = true;
    }
}

template <int DP>
void launch_assign_t(const float *X, const float *Pts, int64_t n, int d, const float *mu, int P,
                     int64_t stride, const int32_t *label, const float *box, int bits,
                     uint32_t *key, hipStream_t s) {
    const size_t shm = (size_t)P * (DP + 1) * sizeof(float);
    (void)hipFuncSetAttribute((const void *)pivot_assign_kernel<DP>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL((pivot_assign_kernel<DP>), dim3((unsigned)((n + 255) / 256)), dim3(256), shm,
                       s, X, Pts, n, d, mu, P, stride, label, box, bits, key);
}

void launch_assign(const float *X, const float *Pts, int64_t n, int d, const float *mu, int P,
                   int64_t stride, const int32_t *label, const float *box, int bits,
                   uint32_t *key, hipStream_t s) {
    if (d <= 16) launch_assign_t<16>(X, Pts, n, d, mu, P, stride, label, box, bits, key, s);
    else if (d <= 32) launch_assign_t<32>(X, Pts, n, d, mu, P, stride, label, box, bits, key, s);
    else if (d <= 48) launch_assign_t<48>(X, Pts, n, d, mu, P, stride, label, box, bits, key, s);
    else launch_assign_t<64>(X, Pts, n, d, mu, P, stride, label, box, bits, key, s);
}

// Centred bounding box of the training points: per coordinate the minimum
// and maximum of x - mu, kept as order-preserving unsigned bits (atomics).
__device__ __forceinline__ uint32_t ord_bits(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord_float(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

__global__ __launch_bounds__(256) void box_init_kernel(uint32_t *__restrict__ ob, int d) {
    const int c = threadIdx.x;
    if (c < d) {
        ob[c] = 0xffffffffu;  // min
        ob[64 + c] = 0u;      // max
    }
}

__global__ __launch_bounds__(256) void box_kernel(const float *__restrict__ X, int64_t n, int d,
                                                  const float *__restrict__ mu,
                                                  uint32_t *__restrict__ ob) {
    const int lane = lane_id();
    for (int c = 0; c < d; ++c) {
        uint32_t lo = 0xffffffffu, hi = 0u;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            const uint32_t o = ord_bits(X[i * d + c] - mu[c]);
            lo = o < lo ? o : lo;
            hi = o > hi ? o : hi;
        }
#pragma unroll
        for (int w = 32; w >= 1; w >>= 1) {
            const uint32_t a = (uint32_t)__shfl_xor((int)lo, w), b = (uint32_t)__shfl_xor((int)hi, w);
            lo = a < lo ? a : lo;
            hi = b > hi ? b : hi;
        }
        if (lane == 0) {
            atomicMin(&ob[c], lo);
            atomicMax(&ob[64 + c], hi);
        }
    }
}

// box[c] = low end, box[64 + c] = 2^bits / width (0 for a constant coordinate).
__global__ __launch_bounds__(64) void box_final_kernel(const uint32_t *__restrict__ ob, int d,
                                                       int bits, float *__restrict__ box) {
    const int c = threadIdx.x;
    if (c < 64) {
        float lo = 0.0f, sc = 0.0f;
        if (c < d) {
            lo = ord_float(ob[c]);
            const float w = ord_float(ob[64 + c]) - lo;
            sc = w > 0.0f ? (float)(1u << bits) / w : 0.0f;
        }
        box[c] = lo;
        box[64 + c] = sc;
    }
}

// Rows i < n come from point perm[i]; padding rows stay in place.
__global__ __launch_bounds__(256) void gather_rows_kernel(const uint4 *__restrict__ Qrows,
                                                          const uint4 *__restrict__ Prows,
                                                          const double *__restrict__ nz,
                                                          const uint32_t *__restrict__ perm,
                                                          int64_t n, int64_t n_pad, int chunks,
                                                          uint4 *__restrict__ Qout,
                                                          uint4 *__restrict__ Pout,
                                                          float *__restrict__ nzq) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_pad * chunks) return;
    const int64_t i = e / chunks;
    const int ch = (int)(e % chunks);
    const int64_t src = i < n ? (int64_t)perm[i] : i;
    Qout[i * chunks + ch] = Qrows[src * chunks + ch];
    if (Pout) Pout[i * chunks + ch] = Prows[src * chunks + ch];
    if (ch == 0) nzq[i] = i < n ? (float)nz[src] : 0.0f;
}

// One wave per tile of 64 BF16 candidate rows [-2 x~, norm parts, 0 ...]
// (kp = 64).  The rows go through LDS so that lane c sums column c; then
// every lane measures its own row against the centroid.
__global__ __launch_bounds__(64) void tile_bounds_kernel(const uint16_t *__restrict__ Prows,
                                                         int64_t n, int d,
                                                         uint16_t *__restrict__ cen,
                                                         float *__restrict__ rad) {
    constexpr int KP = 64;
    __shared__ __align__(16) uint16_t rows[SCREEN_TILE * KP];
    __shared__ float ctr[KP];
    const int64_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t row = tile * SCREEN_TILE + lane;
    const bool real = row < n;
    const int cnt = (int)__popcll(__ballot(real));
    uint16_t *crow = cen + tile * KP;
    if (cnt == 0) {  // padding only: no candidate, always skipped
        crow[lane] = lane == d ? f32_to_bf16_rn(1.0e30f) : (uint16_t)0;
        if (lane == 0) rad[tile] = -1.0e18f;
        return;
    }
    {
        const uint4 *src = (const uint4 *)(Prows + row * KP);
        uint4 *dst = (uint4 *)(rows + lane * KP);
#pragma unroll
        for (int w = 0; w < KP / 8; ++w) dst[w] = real ? src[w] : make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    // centroid of the rows' x~ = -(row) / 2 (exact), rounded to BF16
    double ct = 0.0;
    if (lane < d) {
        double sum = 0.0;
        for (int r = 0; r < SCREEN_TILE; ++r) sum += -0.5 * (double)bf16_to_f32(rows[r * KP + lane]);
        const uint16_t h = f32_to_bf16_rn((float)(sum / cnt));
        ct = (double)bf16_to_f32(h);
        crow[lane] = f32_to_bf16_rn(-2.0f * bf16_to_f32(h));  // exact scale
    }
    ctr[lane] = (float)ct;  // exact: a BF16 value
    const double nc = wave_sum_f64(ct * ct);
    __syncthreads();
    double r2 = 0.0;
    if (real) {
        for (int c = 0; c < d; ++c) {
            const double t = -0.5 * (double)bf16_to_f32(rows[lane * KP + c]) - (double)ctr[c];
            r2 += t * t;
        }
    }
    double mx = r2;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const double o = __shfl_xor(mx, w);
        mx = o > mx ? o : mx;
    }
    // norm parts of the centroid row
    const uint16_t hi = f32_to_bf16_rn((float)nc);
    const double q1 = nc - (double)bf16_to_f32(hi);
    const uint16_t mid = f32_to_bf16_rn((float)q1);
    const double q2 = q1 - (double)bf16_to_f32(mid);
    const uint16_t lo = f32_to_bf16_rn((float)q2);
    if (lane >= d)
        crow[lane] = (lane == d) ? hi : (lane == d + 1) ? mid : (lane == d + 2) ? lo : (uint16_t)0;
    if (lane == 0) rad[tile] = (float)(sqrt(mx) * (1.0 + 1.0e-6)) * (1.0f + 1.0e-6f);
}

// One wave per tile of 64 FP32 candidate rows [-2 x~, ||x~||^2, 0 ...] (kp
// floats, a multiple of 16): the centroid of the rows' x~, rounded to FP32,
// written as a candidate row (its norm rounded to FP32, within the 1e-6
// relative slack of the screen's error bound), and the FP64 radius.
__global__ __launch_bounds__(64) void tile_bounds_f32_kernel(const float *__restrict__ Prows,
                                                             int64_t n, int d, int kp,
                                                             float *__restrict__ cen,
                                                             float *__restrict__ rad) {
    __shared__ __align__(16) float rows[SCREEN_TILE * 64];
    __shared__ float ctr[64];
    const int64_t tile = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t row = tile * SCREEN_TILE + lane;
    const bool real = row < n;
    const int cnt = (int)__popcll(__ballot(real));
    float *crow = cen + tile * kp;
    if (cnt == 0) {  // padding only: no candidate, always skipped
        if (lane < kp) crow[lane] = lane == d ? 1.0e30f : 0.0f;
        if (lane == 0) rad[tile] = -1.0e18f;
        return;
    }
    for (int c = 0; c < kp; c += 4) {
        const float4 v = real ? *(const float4 *)(Prows + row * kp + c) : float4{0.f, 0.f, 0.f, 0.f};
        *(float4 *)(rows + lane * 64 + c) = v;
    }
    __syncthreads();
    // centroid of the rows' x~ = -(row) / 2 (exact), rounded to FP32
    double ct = 0.0;
    if (lane < d) {
        double sum = 0.0;
        for (int r = 0; r < SCREEN_TILE; ++r) sum += -0.5 * (double)rows[r * 64 + lane];
        const float h = (float)(sum / cnt);
        ct = (double)h;
        crow[lane] = -2.0f * h;  // exact scale
    }
    ctr[lane] = (float)ct;
    const double nc = wave_sum_f64(ct * ct);
    __syncthreads();
    double r2 = 0.0;
    if (real) {
        for (int c = 0; c < d; ++c) {
            const double t = -0.5 * (double)rows[lane * 64 + c] - (double)ctr[c];
            r2 += t * t;
        }
    }
    double mx = r2;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const double o = __shfl_xor(mx, w);
        mx = o > mx ? o : mx;
    }
    if (lane >= d && lane < kp) crow[lane] = (lane == d) ? (float)nc : 0.0f;
    if (lane == 0) rad[tile] = (float)(sqrt(mx) * (1.0 + 1.0e-6)) * (1.0f + 1.0e-6f);
}

// One wave per ball of `fan` consecutive tiles (a group or a super-tile): the
// centroid row of the ball (the mean of its real tiles' centroids, rounded to
// the row format: BF16 rows hold -2 c then three BF16 parts of ||c||^2, FP32
// rows -2 c then ||c||^2) and the radius max_t (||c_t - c|| + r_t) over its
// real tiles (FP64, rounded up): by the triangle inequality every row of the
// ball's tiles lies within it.  Coordinates are recovered exactly from the
// rows' -2 x entries.
template <bool BF16>
__global__ __launch_bounds__(64) void super_bounds_kernel(const void *__restrict__ tile_c,
                                                          const float *__restrict__ tile_r,
                                                          int d, int kp, int fan,
                                                          void *__restrict__ sup_c,
                                                          float *__restrict__ sup_r) {
    __shared__ double ctr[64];
    const int lane = threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.x * fan;
    auto coord = [&](int64_t t, int c) -> double {
        if (BF16) return -0.5 * (double)bf16_to_f32(((const uint16_t *)tile_c)[t * kp + c]);
        return -0.5 * (double)((const float *)tile_c)[t * kp + c];
    };
    // real tiles: radius not negative
    int cnt = 0;
    double sum = 0.0;
    for (int t = 0; t < fan; ++t) {
        if (!(tile_r[s0 + t] >= 0.0f)) continue;
        ++cnt;
        if (lane < d) sum += coord(s0 + t, lane);
    }
    double ct = 0.0;
    if (cnt > 0 && lane < d) {
        if (BF16) {
            const uint16_t h = f32_to_bf16_rn((float)(sum / cnt));
            ct = (double)bf16_to_f32(h);
        } else {
            ct = (double)(float)(sum / cnt);
        }
    }
    ctr[lane] = ct;
    __syncthreads();
    const double nc = wave_sum_f64(ct * ct);
    // radius: lane handles tiles lane, lane + 64, ...
    double mx = cnt > 0 ? 0.0 : -1.0e18;
    for (int t = lane; t < fan; t += 64) {
        const float r = tile_r[s0 + t];
        if (!(r >= 0.0f)) continue;
        double e2 = 0.0;
        for (int c = 0; c < d; ++c) {
            const double u = coord(s0 + t, c) - ctr[c];
            e2 += u * u;
        }
        const double b = sqrt(e2) * (1.0 + 1.0e-12) + (double)r;
        mx = b > mx ? b : mx;
    }
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const double o = __shfl_xor(mx, w);
        mx = o > mx ? o : mx;
    }
    if (lane == 0)
        sup_r[blockIdx.x] = cnt > 0 ? (float)(mx * (1.0 + 1.0e-6)) * (1.0f + 1.0e-6f) : -1.0e18f;
    if (BF16) {
        uint16_t *row = (uint16_t *)sup_c + (int64_t)blockIdx.x * kp;
        if (cnt == 0) {
            row[lane] = lane == d ? f32_to_bf16_rn(1.0e30f) : (uint16_t)0;
            return;
        }
        const uint16_t hi = f32_to_bf16_rn((float)nc);
        const double q1 = nc - (double)bf16_to_f32(hi);
        const uint16_t mid = f32_to_bf16_rn((float)q1);
        const double q2 = q1 - (double)bf16_to_f32(mid);
        const uint16_t lo = f32_to_bf16_rn((float)q2);
        if (lane < d)
            row[lane] = f32_to_bf16_rn(-2.0f * (float)ct);  // exact scale of a BF16 value
        else
            row[lane] = (lane == d) ? hi : (lane == d + 1) ? mid : (lane == d + 2) ? lo : (uint16_t)0;
    } else {
        float *row = (float *)sup_c + (int64_t)blockIdx.x * kp;
        if (lane >= kp) return;
        if (cnt == 0) {
            row[lane] = lane == d ? 1.0e30f : 0.0f;
            return;
        }
        row[lane] = lane < d ? -2.0f * (float)ct : (lane == d ? (float)nc : 0.0f);
    }
}

// Stable LSD radix sort of 32-bit keys by 8-bit digits, one pass per
// digit: tile t of SORT_TILE consecutive items counts its digits into
// cnt[digit * tiles + t]; the exclusive scan of cnt in that (digit, tile)
// order gives every (digit, tile) its first output position; each tile then
// scatters its items in index order.  vals_out[pos] = the item's value
// (vals_in[item], or the item's index when vals_in is null).
constexpr int SORT_TILE = 4096;

int sort_tiles(int64_t n) { return (int)((n + SORT_TILE - 1) / SORT_TILE); }

__global__ __launch_bounds__(64) void digit_count_kernel(const uint32_t *__restrict__ key,
                                                         int64_t n, int shift, int tiles,
                                                         uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[256];
    const int lane = threadIdx.x;
    for (int l = lane; l < 256; l += 64) h[l] = 0u;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int i = lane; i < SORT_TILE; i += 64) {
        const int64_t g = base + i;
        if (g < n) atomicAdd(&h[(key[g] >> shift) & 255u], 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int l = lane; l < 256; l += 64) cnt[(int64_t)l * tiles + blockIdx.x] = h[l];
}

// Exclusive scan of cnt[len] in place, one workgroup of 1024 threads (each
// sums a contiguous chunk, the chunk totals are scanned in LDS, then each
// chunk is rewritten).
__global__ __launch_bounds__(1024) void digit_scan_kernel(uint32_t *__restrict__ cnt,
                                                          int64_t len) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (len + 1023) / 1024;
    const int64_t b = t * per, e = b + per < len ? b + per : len;
    uint32_t sum = 0;
    for (int64_t i = b; i < e; ++i) sum += cnt[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int64_t i = b; i < e; ++i) {
        const uint32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
}

// One wave per tile: 64 items at a time in index order; lanes with equal
// digits are found by ballots over the digit's bits, ranked by lane, and
// placed after the digit's running position (kept in LDS).
__global__ __launch_bounds__(64) void digit_scatter_kernel(const uint32_t *__restrict__ key_in,
                                                           const uint32_t *__restrict__ val_in,
                                                           int64_t n, int shift, int tiles,
                                                           const uint32_t *__restrict__ start,
                                                           uint32_t *__restrict__ key_out,
                                                           uint32_t *__restrict__ val_out) {
    __shared__ uint32_t off[256];
    const int lane = threadIdx.x;
    for (int l = lane; l < 256; l += 64) off[l] = start[(int64_t)l * tiles + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_TILE; r += 64) {
        if (base + r >= n) break;
        const int64_t g = base + r + lane;
        const bool valid = g < n;
        const uint32_t k = valid ? key_in[g] : 0u;
        const uint32_t l = valid ? ((k >> shift) & 255u) : 256u;  // 256: no item (9 bits)
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 9; ++b) {
            const uint64_t m = __ballot((l >> b) & 1u);
            peers &= ((l >> b) & 1u) ? m : ~m;
        }
        const int leader = __ffsll((long long)peers) - 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        uint32_t first = 0u;
        if (valid && lane == leader) {
            first = off[l];
            off[l] = first + (uint32_t)__popcll(peers);
        }
        first = (uint32_t)__shfl((int)first, leader);
        if (valid) {
            const uint32_t pos = first + (uint32_t)__popcll(peers & lt);
            key_out[pos] = k;
            val_out[pos] = val_in ? val_in[g] : (uint32_t)g;
        }
    }
}

// Morton bits per coordinate for d-dimensional points (0: no Morton order;
// high-dimensional cells have no finer structure worth ordering).
int morton_bits(int d) { return d <= 8 ? 24 / d : 0; }

// Radix passes over the key digits in use: the Morton bits (low 24), then
// the pivot label (top 8).  The keys start in buffer `(npass + 1) % 2` of
// {ka, kb} and end in kb, the values in perm.
int sort_passes(int d) { return (morton_bits(d) * d + 7) / 8 + 1; }

hipError_t launch_key_sort(int d, int64_t n, uint32_t *ka, uint32_t *kb, uint32_t *va,
                           uint32_t *perm, void *tmp, size_t tmp_bytes, hipStream_t s) {
    const int tiles = sort_tiles(n);
    if (tmp_bytes < (size_t)256 * tiles * 4) return hipErrorInvalidValue;
    uint32_t *cnt = (uint32_t *)tmp;
    const int np = sort_passes(d);
    const int low = np - 1;  // Morton digit passes (bits 0-7, 8-15, 16-23 as needed)
    uint32_t *K[2] = {ka, kb}, *V[2] = {va, perm};
    int cur = (np + 1) % 2;
    for (int p = 0; p < np; ++p) {
        const int shift = p < low ? 8 * p : 24;
        hipLaunchKernelGGL(digit_count_kernel, dim3(tiles), dim3(64), 0, s, K[cur], n, shift, tiles,
                           cnt);
        hipLaunchKernelGGL(digit_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, (int64_t)256 * tiles);
        hipLaunchKernelGGL(digit_scatter_kernel, dim3(tiles), dim3(64), 0, s, K[cur],
                           p == 0 ? (const uint32_t *)nullptr : V[cur], n, shift, tiles, cnt,
                           K[cur ^ 1], V[cur ^ 1]);
        cur ^= 1;
    }
    return hipGetLastError();
}

// cell[j] = first position of pivot j in the sorted keys (j <= P).
__global__ __launch_bounds__(256) void cell_start_kernel(const uint32_t *__restrict__ keys,
                                                         int64_t n, int P,
                                                         int32_t *__restrict__ cell) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > P) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((keys[mid] >> 24) < (uint32_t)j) lo = mid + 1;
        else hi = mid;
    }
    cell[j] = (int32_t)lo;
}

// Start column of query block b: where the key of the block's first query
// falls among the training points' sorted keys (its pivot cell and, in low
// dimensions, its place on the cell's space-filling curve), rounded down to
// a tile.
__global__ __launch_bounds__(256) void block_start_kernel(const uint32_t *__restrict__ qkeys,
                                                          int64_t m, int64_t blocks,
                                                          const uint32_t *__restrict__ keys,
                                                          int64_t n, int32_t *__restrict__ rot) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= blocks) return;
    const int64_t q = b * SCREEN_QPB < m ? b * SCREEN_QPB : m - 1;
    const uint32_t key = qkeys[q];
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    if (lo >= n) lo = n - 1;
    rot[b] = (int32_t)(lo & ~(int64_t)(SCREEN_TILE - 1));
}

}  // namespace

int prune_pivots(int64_t n) {
    const int64_t p = n / 2048;
    return (int)(p < 1 ? 1 : (p > 256 ? 256 : p));
}

hipError_t prune_sort_bytes(int64_t n, size_t *bytes) {
    *bytes = (size_t)256 * sort_tiles(n) * 4 + 1024;
    return hipSuccess;
}

hipError_t launch_prune_order(const float *X, int64_t n, int d, const float *mu, void *sort_tmp,
                              size_t sort_bytes, int32_t *label, float *box, uint32_t *ka,
                              uint32_t *keys, uint32_t *va, uint32_t *perm, hipStream_t s) {
    const int P = prune_pivots(n);
    const int64_t stride = n / P;
    if (d > 64 || P > 256 || sort_bytes < (size_t)256 * sort_tiles(n) * 4 + 1024)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(pivot_chain_kernel, dim3(1), dim3(256), 0, s, X, d, mu, P, stride, label);
    const int bits = morton_bits(d);
    if (bits > 0) {
        // the bounding box's order bits sit past the sort counters
        uint32_t *ob = (uint32_t *)((char *)sort_tmp + (size_t)256 * sort_tiles(n) * 4);
        const int64_t nb = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
        hipLaunchKernelGGL(box_init_kernel, dim3(1), dim3(256), 0, s, ob, d);
        hipLaunchKernelGGL(box_kernel, dim3((unsigned)nb), dim3(256), 0, s, X, n, d, mu, ob);
        hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(64), 0, s, ob, d, bits, box);
    } else {
        hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(64), 0, s, (const uint32_t *)nullptr, 0,
                           0, box);
    }
    uint32_t *first = (sort_passes(d) + 1) % 2 == 0 ? ka : keys;
    launch_assign(X, X, n, d, mu, P, stride, label, bits > 0 ? box : nullptr, bits, first, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_key_sort(d, n, ka, keys, va, perm, sort_tmp, sort_bytes, s);
}

hipError_t launch_prune_rows(const ScreenGeom &g, const void *Qrows, const void *Prows,
                             const double *nz, const uint32_t *perm, int64_t n, int64_t n_pad,
                             int d, void *Qout, void *Pout, float *nzq, void *tile_c,
                             float *tile_r, void *grp_c, float *grp_r, void *sup_c, float *sup_r,
                             hipStream_t s) {
    if (g.row_bytes % 16 != 0 || n_pad % SCREEN_SUPER_ROWS != 0) return hipErrorInvalidValue;
    const int chunks = g.row_bytes / 16;
    const int64_t items = n_pad * chunks;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s,
                       (const uint4 *)Qrows, (const uint4 *)Prows, nz, perm, n, n_pad, chunks,
                       (uint4 *)Qout, (uint4 *)Pout, nzq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (g.mode == SCREEN_BF16) {
        if (g.kp != 64) return hipErrorInvalidValue;
        hipLaunchKernelGGL(tile_bounds_kernel, dim3((unsigned)(n_pad / SCREEN_TILE)), dim3(64), 0,
                           s, (const uint16_t *)Pout, n, d, (uint16_t *)tile_c, tile_r);
    } else {
        if (g.kp > 64 || g.kp % 16 != 0 || d >= g.kp) return hipErrorInvalidValue;
        hipLaunchKernelGGL(tile_bounds_f32_kernel, dim3((unsigned)(n_pad / SCREEN_TILE)), dim3(64),
                           0, s, (const float *)Pout, n, d, g.kp, (float *)tile_c, tile_r);
    }
    for (int level = 0; level < 2; ++level) {
        const int fan = level == 0 ? SCREEN_GROUP : SCREEN_SUPER;
        const unsigned balls = (unsigned)(n_pad / SCREEN_TILE / fan);
        void *bc = level == 0 ? grp_c : sup_c;
        float *br = level == 0 ? grp_r : sup_r;
        if (g.mode == SCREEN_BF16)
            hipLaunchKernelGGL(super_bounds_kernel<true>, dim3(balls), dim3(64), 0, s,
                               (const void *)tile_c, (const float *)tile_r, d, g.kp, fan, bc, br);
        else
            hipLaunchKernelGGL(super_bounds_kernel<false>, dim3(balls), dim3(64), 0, s,
                               (const void *)tile_c, (const float *)tile_r, d, g.kp, fan, bc, br);
    }
    return hipGetLastError();
}

hipError_t launch_cell_starts(const uint32_t *keys, int64_t n, int P, int32_t *cell,
                              hipStream_t s) {
    hipLaunchKernelGGL(cell_start_kernel, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, s,
                       keys, n, P, cell);
    return hipGetLastError();
}

hipError_t launch_prune_queries(const float *X, int64_t n, const float *Z, int64_t m, int d,
                                const float *mu, void *sort_tmp, size_t sort_bytes,
                                const int32_t *label, const float *box, uint32_t *ka,
                                uint32_t *kb, uint32_t *va, uint32_t *qperm, const ScreenGeom &g,
                                const void *Zq, const double *nzz, int64_t m_pad, void *Zq_out,
                                float *nzq, const uint32_t *keys, int32_t *rot, hipStream_t s) {
    if (d > 64 || g.row_bytes % 16 != 0) return hipErrorInvalidValue;
    const int P = prune_pivots(n);
    const int64_t stride = n / P;
    const int bits = morton_bits(d);
    uint32_t *first = (sort_passes(d) + 1) % 2 == 0 ? ka : kb;
    launch_assign(X, Z, m, d, mu, P, stride, label, bits > 0 ? box : nullptr, bits, first, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_key_sort(d, m, ka, kb, va, qperm, sort_tmp, sort_bytes, s);
    if (e != hipSuccess) return e;
    const int chunks = g.row_bytes / 16;
    const int64_t items = m_pad * chunks;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s,
                       (const uint4 *)Zq, (const uint4 *)nullptr, nzz, qperm, m, m_pad, chunks,
                       (uint4 *)Zq_out, (uint4 *)nullptr, nzq);
    const int64_t blocks = m_pad / SCREEN_QPB;
    hipLaunchKernelGGL(block_start_kernel, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s,
                       kb, m, blocks, keys, n, rot);
    return hipGetLastError();
}

hipError_t prune_query_sort_bytes(int64_t n, int64_t m, size_t *bytes) {
    (void)n;
    *bytes = (size_t)256 * sort_tiles(m) * 4;
    return hipSuccess;
}

}  // namespace fmg
