// Internal launch interface between the host runtime (fmg_api.cpp) and the
// HIP kernels.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmg {

// Screening arithmetic.
enum ScreenMode { SCREEN_BF16 = 0, SCREEN_F32 = 1 };

// Candidates per iteration of the screen (one 64-row tile of training points).
constexpr int SCREEN_TILE = 64;
// Queries per screen workgroup (4 waves x 64 queries).
constexpr int SCREEN_QPB = 256;
// Pool entries per query in the screen (candidate keys awaiting selection),
// and the largest number of candidates kept per query and split.  Screens
// keeping at most SCREEN_CAP_SMALL_C candidates use pools of SCREEN_CAP_SMALL
// entries (selections come more often, each over fewer entries); pool
// buffers are sized for SCREEN_CAP.
constexpr int SCREEN_CAP = 512;
constexpr int SCREEN_CAP_SMALL = 256;
constexpr int SCREEN_CAP_SMALL_C = 112;
constexpr int SCREEN_CMAX = 128;
// Pruned screens group tiles into super-tiles of SCREEN_SUPER tiles (a
// pruned model pads its candidate rows to whole super-tiles) and keep at
// most SCREEN_SUPER_MAX of them (n <= 33.5M).
constexpr int SCREEN_SUPER = 256;
constexpr int SCREEN_SUPER_ROWS = SCREEN_SUPER * SCREEN_TILE;
constexpr int SCREEN_SUPER_MAX = 2048;
// Between the two, groups of SCREEN_GROUP tiles (16 per super-tile), the
// unit in which a pruned scan loads tiles.
constexpr int SCREEN_GROUP = 16;
constexpr int SCREEN_GROUP_ROWS = SCREEN_GROUP * SCREEN_TILE;

// Row layout of the screening arrays: `kp` elements per row (bf16 or f32),
// row bytes = kp * elem.  bf16: kp = 64 (2 MFMA k-steps of 32); f32: kp a
// multiple of 16.
struct ScreenGeom {
    int mode;    // ScreenMode
    int kp;      // elements per row
    int ksteps;  // MFMA k-steps per tile
    int row_bytes;
};

struct ScreenArgs {
    const void *Q;      // [m_pad, kp] query-side rows
    const void *P;      // [n_pad, kp] candidate-side rows
    int64_t m, m_pad;   // queries (real, padded to SCREEN_QPB)
    int64_t n, n_pad;   // candidates (real, padded to SCREEN_TILE)
    int64_t col_chunk;  // candidate columns per split (multiple of SCREEN_TILE)
    int splits;
    int loo;            // 1: query q never takes candidate q
    int c;              // candidates kept per (query, split), 1..SCREEN_CMAX
    uint64_t *pool;     // [splits, m_pad, SCREEN_CAP] scratch
    uint64_t *cand;     // [splits, m, c] sorted screen keys (value, index)
    float *tq;          // [splits, m] c-th kept value, +inf when fewer than c
    // Tile pruning (BF16 screen of a self-join whose rows are ordered so that
    // 64-row tiles are compact; prune != 0): per candidate tile a centroid row
    // in the candidate-row format and a radius bounding its rows, the query
    // rows' squared norms, and the accumulation-error coefficients of the
    // certificate.  Each workgroup then starts its scan at its own rows.
    int prune;
    const void *tile_c;  // [n_pad / SCREEN_TILE, kp]
    const float *tile_r; // [n_pad / SCREEN_TILE]
    const void *sup_c;   // [n_pad / SCREEN_SUPER_ROWS, kp] super-tile centroid rows
    const float *sup_r;  // [n_pad / SCREEN_SUPER_ROWS] super-tile radii
    const void *grp_c;   // [n_pad / SCREEN_GROUP_ROWS, kp] group centroid rows
    const float *grp_r;  // [n_pad / SCREEN_GROUP_ROWS] group radii
    const float *nzq;    // [m_pad] ||z~||^2 of the query rows
    double acc_coef, nx_max;
    // Optional start column of each workgroup (a multiple of SCREEN_TILE);
    // without it a pruned self-join starts at the workgroup's own rows.
    const int32_t *rot_tab;
};

struct RerankArgs {
    const uint64_t *cand;
    const float *tq;
    int splits, c;
    int64_t m;
    const void *X;       // [n, d] training coordinates (float)
    const void *Zc;      // [m, d] query coordinates (float)
    int d;
    const double *nzq;   // [m] exact ||z~||^2 of the screened query rows
    const double *eq;    // [m] rounding radius of the screened query rows
    double e_max;        // max rounding radius over training rows
    double acc_coef;     // A_q = acc_coef * (2.01 nx_max + nz_q) + 1e-6 nx_max
    double nx_max;
    int k;               // neighbours to keep
    int self_first;      // write q first, then k results (SELF mode)
    int32_t *out;
    int out_stride;
    int32_t *fb_list;    // rows that failed the certificate
    int32_t *fb_count;
    // Optional (screens run in a pivot order): wave w handles query order[w],
    // whose candidates are cand / tq row w (nearby queries in consecutive
    // waves share candidate rows in the caches), and a screened index below
    // n_idx maps to training index cand_idx[index].
    const uint32_t *order;
    const uint32_t *cand_idx;
    int64_t n_idx;
};

struct ExactArgs {
    const void *X;        // [n, d] training coordinates (float or double), followed by
                          // 64 readable elements (the model's padded copy)
    int64_t n;
    int d;
    const void *Qc;       // [*, d] query coordinates
    const int32_t *list;  // optional list of query rows
    const int32_t *count; // optional device count of `list`
    int64_t nq;           // number of query rows when count == nullptr
    int loo;              // exclude candidate == query row index
    int k;                // 1..256 (k > 64: the pooled search)
    int self_first;
    int32_t *out;
    int out_stride;
    // Optional scratch for the nearest-point search (k = 1, query batches):
    // partial minima of a scan split over candidate chunks, NN_SPLIT_ENTRIES
    // each.  Without it every query is scanned by one lane over all points.
    uint64_t *nn_key;
    int32_t *nn_idx;
};

// Split nearest-point search: chunks x queries stays within this many
// partial minima (8192 waves of 64 queries).
constexpr int64_t NN_SPLIT_ENTRIES = 8192 * 64;

struct PrecomputeArgs {
    const void *X;   // [n, d]
    const void *Y;   // [n, ell]
    int64_t n;
    int d, ell, k;
    const int32_t *N;  // [n, k]
    void *C;           // [n, k, ell]
    int32_t *status;   // [n] 0 ok, 1 not positive definite
    const void *Ctr;   // [n, d] centre of row i's neighbourhood (nullptr: X row i);
                       // any point works: kernel values depend on differences only
    int kc;            // kernel code (fmg_device.h)
    double inv_rho, amp, noise;
    // optional: workgroup b factors point order[b] (a permutation of [0, n);
    // FP32 / mixed kernel), so that nearby points run together and share
    // neighbour rows in the caches
    const uint32_t *order;
};

struct GatherArgs {
    const void *X;
    const void *Z;         // query coordinates
    const uint32_t *order; // optional: wave w handles query order[w] (a permutation of [0, m))
    const int32_t *zrow;   // optional: query q is row zrow[q] of Z (else row q)
    const int32_t *nn;     // optional: coefficient row of query q (else q)
    const int32_t *N;      // neighbourhood rows [*, k]
    const void *C;         // coefficient rows [*, k, ell]
    int64_t m;
    int64_t zrows;         // rows of Z (bound of zrow entries)
    int64_t crows;         // rows of N and C (bound of nn entries)
    int d, ell, k;
    int kc;
    double inv_rho, amp;
    void *out;
};

struct GradArgs {
    const void *X;        // [n, d] training coordinates (float or double)
    const void *Y;        // [n, ell] responses
    const int32_t *N;     // [n, k] leave-one-out neighbour lists
    const int32_t *rows;  // [b] batch training points
    int64_t b, n;
    int d, ell, k;
    int kc;               // kernel code (fmg_device.h)
    double inv_rho, amp, noise;
    double *terms;        // [b, 3] per-point (sum_c e_c^2, d/drho, d/dsigma^2)
    int *bad;             // set when a row index is outside [0, n)
};

// Column mean of X [n, d] into mu [d] (deterministic); part is scratch of
// col_mean_blocks(n) * d doubles.
int col_mean_blocks(int64_t n);
hipError_t launch_col_mean(const void *X, bool f64, int64_t n, int d, float *mu, double *part,
                           hipStream_t s);
hipError_t launch_finite_check(const void *A, bool f64, int64_t count, int *flag, hipStream_t s);
hipError_t launch_prep_rows(const ScreenGeom &g, const float *X, int64_t n, int64_t n_pad, int d,
                            const float *mu, void *Qrows, void *Prows, double *e_out,
                            double *nz_out, unsigned long long *emax_bits,
                            unsigned long long *nxmax_bits, hipStream_t s);
hipError_t launch_screen(const ScreenGeom &g, const ScreenArgs &a, hipStream_t s);
hipError_t launch_rerank(const RerankArgs &a, hipStream_t s);
hipError_t launch_exact_topk(bool f64, const ExactArgs &a, int64_t max_items, hipStream_t s);
// k <= 64: one wavefront per point (fmg_precompute*.hip); 64 < k <= 256: one
// workgroup per point with the factor in LDS (fmg_precompute_wide.hip, no
// refinement step), needing precompute_wide_lds_bytes(f64, k, d) <=
// PRECOMPUTE_WIDE_LDS_MAX.
hipError_t launch_precompute(bool f64, bool refine, const PrecomputeArgs &a, hipStream_t s);
constexpr size_t PRECOMPUTE_WIDE_LDS_MAX = 160 * 1024;
size_t precompute_wide_lds_bytes(bool f64, int k, int d);
hipError_t launch_precompute_wide(bool f64, const PrecomputeArgs &a, hipStream_t s);
// FP32 precompute (FP32 and MIXED precision), refinement optional.
hipError_t launch_precompute32(bool refine, const PrecomputeArgs &a, hipStream_t s);
hipError_t launch_gather(bool f64, const GatherArgs &a, hipStream_t s);
hipError_t launch_count_nonzero(const int32_t *a, int64_t n, unsigned long long *out,
                                hipStream_t s);
// N[i] = i for every row (self-inclusive neighbourhoods of size 1).
hipError_t launch_self_rows(int32_t *N, int64_t n, hipStream_t s);
// Zero `count` 32-bit words with a kernel (safe inside captured graphs).
hipError_t launch_zero_u32(void *ptr, int64_t count, hipStream_t s);
// Leave-one-out loss helpers (fmg_loss.hip): gather X, N and Y rows of a
// batch of training points (*bad set for an index outside [0, n)), and the
// deterministic sum of squared differences of `count` values (part holds
// sq_err_blocks(count) doubles).
hipError_t launch_batch_rows(bool f64, const void *X, const int32_t *N, const void *Y,
                             const int32_t *rows, int64_t b, int64_t n, int d, int k, int ell,
                             void *Xb, int32_t *Nb, void *Yb, int *bad, hipStream_t s);
int sq_err_blocks(int64_t count);
hipError_t launch_sq_err(bool f64, const void *Y, const void *mu, int64_t count, double *part,
                         double *out, hipStream_t s);

// Leave-one-out loss and its gradient in (rho, sigma^2), FP64 (fmg_grad.hip):
// per-point terms, then their column sums into out[3]; part holds
// loo_grad_blocks(b) * 3 doubles.  hipErrorInvalidValue when k > 64,
// ell > 16 or the staged rows exceed 64 KB of LDS (loo_grad_lds_bytes).
size_t loo_grad_lds_bytes(int k, int d);
int loo_grad_blocks(int64_t b);
hipError_t launch_loo_grad(bool f64, const GradArgs &a, double *part, double *out,
                           hipStream_t s);

// Tile pruning of the build screen (fmg_prune.hip): the order of the training
// points by (nearest pivot, Morton code in low dimensions) (perm), the
// screening rows and query norms gathered into it with the per-tile centroid
// rows and radii (the re-rank then takes the rows in the same order).
int prune_pivots(int64_t n);
hipError_t prune_sort_bytes(int64_t n, size_t *bytes);
// label [P]: pivot labels along a nearest-neighbour chain; box [128]: the
// centred bounding box of the Morton code; keys [n]: the sorted keys (all
// three written here and kept by the model for predictions); ka, va [n]:
// scratch; perm [n]: position -> training point.
hipError_t launch_prune_order(const float *X, int64_t n, int d, const float *mu, void *sort_tmp,
                              size_t sort_bytes, int32_t *label, float *box, uint32_t *ka,
                              uint32_t *keys, uint32_t *va, uint32_t *perm, hipStream_t s);
// Also the group and super-tile balls: per SCREEN_GROUP (SCREEN_SUPER) tiles a
// centroid row (the mean of the tiles' real centroids, in the row format) and
// a radius max_t (||c_t - c|| + r_t) (FP64, rounded up); n_pad must be a
// multiple of SCREEN_SUPER_ROWS.  Balls with no real row get a negative radius
// of -1e18, so every screen skips them.
hipError_t launch_prune_rows(const ScreenGeom &g, const void *Qrows, const void *Prows,
                             const double *nz, const uint32_t *perm, int64_t n, int64_t n_pad,
                             int d, void *Qout, void *Pout, float *nzq, void *tile_c,
                             float *tile_r, void *grp_c, float *grp_r, void *sup_c, float *sup_r,
                             hipStream_t s);
// cell[j], j <= P: first position of pivot j in the sorted keys.
hipError_t launch_cell_starts(const uint32_t *keys, int64_t n, int P, int32_t *cell,
                              hipStream_t s);
// Queries of a prediction in the same key order: their keys (the model's
// pivots and box), the stable sort (qperm: position -> query; ka, kb, va:
// scratch [m]), the query rows and norms gathered into that order, and each
// workgroup's start column (where its first query's key falls among the
// model's sorted training keys).
hipError_t prune_query_sort_bytes(int64_t n, int64_t m, size_t *bytes);
hipError_t launch_prune_queries(const float *X, int64_t n, const float *Z, int64_t m, int d,
                                const float *mu, void *sort_tmp, size_t sort_bytes,
                                const int32_t *label, const float *box, uint32_t *ka,
                                uint32_t *kb, uint32_t *va, uint32_t *qperm, const ScreenGeom &g,
                                const void *Zq, const double *nzz, int64_t m_pad, void *Zq_out,
                                float *nzq, const uint32_t *keys, int32_t *rot, hipStream_t s);

// y[i] = the FP64 exponential of x[i] <= 0 that the refinement's residual
// evaluates kernel values with (fmg_precompute32.hip).
hipError_t launch_exp_nonpos64(const double *x, double *y, int64_t n, hipStream_t s);
hipError_t launch_exp_nonpos32(const float *x, float *y, int64_t n, hipStream_t s);

// *dst += *src
hipError_t launch_accum(const int32_t *src, unsigned long long *dst, hipStream_t s);

}  // namespace fmg
