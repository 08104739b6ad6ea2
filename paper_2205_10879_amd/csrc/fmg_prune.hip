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

// Nearest pivot of points Pts [n, d]; pivot j is training row j * stride of X.
// Coordinates are zero padded to DP (a multiple of 16 covering d), so the
// loop has no guards and reads each pivot row as 16-byte vectors.  The
// nearest pivot minimises ||p_j||^2 - 2 x.p_j (||x||^2 is common to all j):
// one FMA per coordinate.  Any assignment serves the pruning (the tile radii
// are measured on the tiles' actual rows), so the rounding of this form is
// harmless.
template <int DP>
__global__ __launch_bounds__(256) void pivot_assign_kernel(const float *__restrict__ X,
                                                           const float *__restrict__ Pts,
                                                           int64_t n, int d,
                                                           const float *__restrict__ mu, int P,
                                                           int64_t stride,
                                                           const int32_t *__restrict__ label,
                                                           uint32_t *__restrict__ asg,
                                                           uint32_t *__restrict__ idx) {
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
    asg[i] = (uint32_t)label[bj];
    idx[i] = (uint32_t)i;
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
                     int64_t stride, const int32_t *label, uint32_t *asg, uint32_t *idx,
                     hipStream_t s) {
    const size_t shm = (size_t)P * (DP + 1) * sizeof(float);
    (void)hipFuncSetAttribute((const void *)pivot_assign_kernel<DP>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    hipLaunchKernelGGL((pivot_assign_kernel<DP>), dim3((unsigned)((n + 255) / 256)), dim3(256), shm,
                       s, X, Pts, n, d, mu, P, stride, label, asg, idx);
}

void launch_assign(const float *X, const float *Pts, int64_t n, int d, const float *mu, int P,
                   int64_t stride, const int32_t *label, uint32_t *asg, uint32_t *idx,
                   hipStream_t s) {
    if (d <= 16) launch_assign_t<16>(X, Pts, n, d, mu, P, stride, label, asg, idx, s);
    else if (d <= 32) launch_assign_t<32>(X, Pts, n, d, mu, P, stride, label, asg, idx, s);
    else if (d <= 48) launch_assign_t<48>(X, Pts, n, d, mu, P, stride, label, asg, idx, s);
    else launch_assign_t<64>(X, Pts, n, d, mu, P, stride, label, asg, idx, s);
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
    if (cnt == 0) {  // padding only: never skipped
        crow[lane] = lane == d ? f32_to_bf16_rn(1.0e30f) : (uint16_t)0;
        if (lane == 0) rad[tile] = INFINITY;
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
    if (cnt == 0) {  // padding only: never skipped
        if (lane < kp) crow[lane] = lane == d ? 1.0e30f : 0.0f;
        if (lane == 0) rad[tile] = INFINITY;
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

// Stable sort of labels < P <= 256 (a counting sort in one pass): tile t of
// SORT_TILE consecutive items counts its labels into cnt[label * tiles + t];
// the exclusive scan of cnt in that (label, tile) order gives every
// (label, tile) its first output position; each tile then scatters its items
// in index order.  perm[pos] = the item's index, sorted[pos] = its label.
constexpr int SORT_TILE = 4096;

int sort_tiles(int64_t n) { return (int)((n + SORT_TILE - 1) / SORT_TILE); }

__global__ __launch_bounds__(64) void label_count_kernel(const uint32_t *__restrict__ lab,
                                                         int64_t n, int P, int tiles,
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
        if (g < n) atomicAdd(&h[lab[g]], 1u);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int l = lane; l < P; l += 64) cnt[(int64_t)l * tiles + blockIdx.x] = h[l];
}

// Exclusive scan of cnt[len] in place, one workgroup of 1024 threads (each
// sums a contiguous chunk, the chunk totals are scanned in LDS, then each
// chunk is rewritten).
__global__ __launch_bounds__(1024) void label_scan_kernel(uint32_t *__restrict__ cnt,
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
// labels are found by ballots over the label's bits, ranked by lane, and
// placed after the label's running position (kept in LDS).
__global__ __launch_bounds__(64) void label_scatter_kernel(const uint32_t *__restrict__ lab,
                                                           int64_t n, int P, int tiles,
                                                           const uint32_t *__restrict__ start,
                                                           uint32_t *__restrict__ sorted,
                                                           uint32_t *__restrict__ perm) {
    __shared__ uint32_t off[256];
    const int lane = threadIdx.x;
    for (int l = lane; l < P; l += 64) off[l] = start[(int64_t)l * tiles + blockIdx.x];
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_TILE; r += 64) {
        if (base + r >= n) break;
        const int64_t g = base + r + lane;
        const bool valid = g < n;
        const uint32_t l = valid ? lab[g] : 256u;  // 256: no item (9 label bits)
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
            sorted[pos] = l;
            perm[pos] = (uint32_t)g;
        }
    }
}

hipError_t launch_label_sort(const uint32_t *lab, int64_t n, int P, void *tmp, size_t tmp_bytes,
                             uint32_t *sorted, uint32_t *perm, hipStream_t s) {
    const int tiles = sort_tiles(n);
    if (P < 1 || P > 256 || tmp_bytes < (size_t)P * tiles * 4) return hipErrorInvalidValue;
    uint32_t *cnt = (uint32_t *)tmp;
    hipLaunchKernelGGL(label_count_kernel, dim3(tiles), dim3(64), 0, s, lab, n, P, tiles, cnt);
    hipLaunchKernelGGL(label_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, (int64_t)P * tiles);
    hipLaunchKernelGGL(label_scatter_kernel, dim3(tiles), dim3(64), 0, s, lab, n, P, tiles, cnt,
                       sorted, perm);
    return hipGetLastError();
}

// cell[j] = first position of pivot j in the sorted assignment (j <= P).
__global__ __launch_bounds__(256) void cell_start_kernel(const uint32_t *__restrict__ asg_sorted,
                                                         int64_t n, int P,
                                                         int32_t *__restrict__ cell) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > P) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (asg_sorted[mid] < (uint32_t)j) lo = mid + 1;
        else hi = mid;
    }
    cell[j] = (int32_t)lo;
}

// Start column of query block b: the cell of the block's first query's pivot,
// rounded down to a tile.
__global__ __launch_bounds__(256) void block_start_kernel(const uint32_t *__restrict__ qasg_sorted,
                                                          int64_t m, int64_t blocks,
                                                          const int32_t *__restrict__ cell,
                                                          int32_t *__restrict__ rot) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= blocks) return;
    const int64_t q = b * SCREEN_QPB < m ? b * SCREEN_QPB : m - 1;
    rot[b] = cell[qasg_sorted[q]] & ~(SCREEN_TILE - 1);
}

}  // namespace

int prune_pivots(int64_t n) {
    const int64_t p = n / 2048;
    return (int)(p < 1 ? 1 : (p > 256 ? 256 : p));
}

hipError_t prune_sort_bytes(int64_t n, size_t *bytes) {
    *bytes = (size_t)prune_pivots(n) * sort_tiles(n) * 4;
    return hipSuccess;
}

hipError_t launch_prune_order(const float *X, int64_t n, int d, const float *mu, void *sort_tmp,
                              size_t sort_bytes, int32_t *label, uint32_t *asg,
                              uint32_t *asg_sorted, uint32_t *idx, uint32_t *perm,
                              hipStream_t s) {
    const int P = prune_pivots(n);
    const int64_t stride = n / P;
    if (d > 64 || P > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pivot_chain_kernel, dim3(1), dim3(256), 0, s, X, d, mu, P, stride, label);
    launch_assign(X, X, n, d, mu, P, stride, label, asg, idx, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    (void)idx;
    return launch_label_sort(asg, n, P, sort_tmp, sort_bytes, asg_sorted, perm, s);
}

hipError_t launch_prune_rows(const ScreenGeom &g, const void *Qrows, const void *Prows,
                             const double *nz, const uint32_t *perm, int64_t n, int64_t n_pad,
                             int d, void *Qout, void *Pout, float *nzq, void *tile_c,
                             float *tile_r, hipStream_t s) {
    if (g.row_bytes % 16 != 0) return hipErrorInvalidValue;
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
    return hipGetLastError();
}

hipError_t launch_cell_starts(const uint32_t *asg_sorted, int64_t n, int P, int32_t *cell,
                              hipStream_t s) {
    hipLaunchKernelGGL(cell_start_kernel, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, s,
                       asg_sorted, n, P, cell);
    return hipGetLastError();
}

hipError_t launch_prune_queries(const float *X, int64_t n, const float *Z, int64_t m, int d,
                                const float *mu, void *sort_tmp, size_t sort_bytes,
                                const int32_t *label, uint32_t *asg, uint32_t *asg_sorted,
                                uint32_t *idx,
                                uint32_t *qperm, const ScreenGeom &g, const void *Zq,
                                const double *nzz, int64_t m_pad, void *Zq_out, float *nzq,
                                const int32_t *cell, int32_t *rot, hipStream_t s) {
    if (d > 64 || g.row_bytes % 16 != 0) return hipErrorInvalidValue;
    const int P = prune_pivots(n);
    const int64_t stride = n / P;
    launch_assign(X, Z, m, d, mu, P, stride, label, asg, idx, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    (void)idx;
    e = launch_label_sort(asg, m, P, sort_tmp, sort_bytes, asg_sorted, qperm, s);
    if (e != hipSuccess) return e;
    const int chunks = g.row_bytes / 16;
    const int64_t items = m_pad * chunks;
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s,
                       (const uint4 *)Zq, (const uint4 *)nullptr, nzz, qperm, m, m_pad, chunks,
                       (uint4 *)Zq_out, (uint4 *)nullptr, nzq);
    const int64_t blocks = m_pad / SCREEN_QPB;
    hipLaunchKernelGGL(block_start_kernel, dim3((unsigned)((blocks + 255) / 256)), dim3(256), 0, s,
                       asg_sorted, m, blocks, cell, rot);
    return hipGetLastError();
}

hipError_t prune_query_sort_bytes(int64_t n, int64_t m, size_t *bytes) {
    *bytes = (size_t)prune_pivots(n) * sort_tiles(m) * 4;
    return hipSuccess;
}

}  // namespace fmg
