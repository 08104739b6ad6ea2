// Host-side internals shared by the library's C ABI (fmg_api.hip) and its
// request server (fmg_server.hip): the model object, the prediction
// workspace and the residency helpers.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "fastmuygps.h"
#include "fmg_kernels.h"

namespace fmg {

enum { EV_START = 0, EV_PREP, EV_SCREEN, EV_RERANK, EV_FALLBACK, EV_LAST, EV_COUNT };

// Device arrays of a model, in the order they are moved between device and
// host memory by model_offload / model_restore.
enum { MA_X = 0, MA_N, MA_C, MA_XP, MA_MU, MA_Y, MA_PERM, MA_XPP, MA_TC, MA_TR, MA_CELL, MA_KEYS,
       MA_BOX, MA_SC, MA_SR, MA_GC, MA_GR, MA_COUNT };

}  // namespace fmg

struct fmg_model {
    int64_t n = 0;
    int d = 0, ell = 0, k = 0;
    fmg_hyper hyper{};
    int prec = 0;
    uint32_t flags = 0;
    int kc = 0;
    double inv_rho = 1.0, amp = 1.0;
    bool self_inc = false;
    int device = 0;

    void *X = nullptr;     // [n, d] (+ 64 zero elements)
    int32_t *N = nullptr;  // [n, k]
    void *C = nullptr;     // [n, k, ell]
    void *Y = nullptr;     // [n, ell] responses (MuyGPs and leave-one-out predictions)

    fmg::ScreenGeom geom{};
    int64_t n_pad = 0;
    void *Xp = nullptr;   // [n_pad, kp] candidate-side screening rows
    float *mu = nullptr;  // [d]
    // Tile pruning (MIXED): the pivot order of the training points
    // (perm[position] = point), the candidate rows in that order, per-tile
    // centroid rows and radii, and the first position of each pivot's cell.
    uint32_t *perm = nullptr;  // [n]
    void *Xpp = nullptr;       // [n_pad, kp]
    void *tile_c = nullptr;    // [n_pad / 64, kp]
    float *tile_r = nullptr;   // [n_pad / 64]
    int32_t *cell = nullptr;   // [pivots + 1] cell starts, then [pivots] pivot labels
    uint32_t *keys = nullptr;  // [n] sort keys in the pivot order (pivot label, Morton code)
    float *box = nullptr;      // [128] the Morton code's box: low ends, then scales
    void *sup_c = nullptr;     // [n_pad / SCREEN_SUPER_ROWS, kp] super-tile centroid rows
    float *sup_r = nullptr;    // [n_pad / SCREEN_SUPER_ROWS] super-tile radii
    void *grp_c = nullptr;     // [n_pad / SCREEN_GROUP_ROWS, kp] group centroid rows
    float *grp_r = nullptr;    // [n_pad / SCREEN_GROUP_ROWS] group radii
    double e_max = 0.0, nx_max = 0.0, acc_coef = 0.0;
    int c_build = 0, c_query = 0;
    int64_t nonpd = 0, build_fb = 0;
    unsigned long long *pred_fb = nullptr;
    uint64_t bytes = 0;  // device bytes of the arrays below while resident

    // Residency: sizes of the movable arrays, and their host copies while the
    // model is offloaded (resident == false).
    size_t arr_bytes[fmg::MA_COUNT]{};
    size_t fb_bytes = 0;  // the prediction fallback counter
    void *host[fmg::MA_COUNT]{};
    bool resident = true;

    bool timing = false;
    hipEvent_t evb[fmg::EV_COUNT]{};
    hipEvent_t evp[fmg::EV_COUNT]{};
    bool pred_recorded = false;
    double build_ms[fmg::EV_COUNT]{};
};

namespace fmg {

// Preallocated device buffers for predictions of up to max_m queries, so
// that a prediction allocates nothing.  Sized for any model the library can
// build (screen rows of at most 256 bytes, c' <= SCREEN_CMAX).
struct PredictWs {
    void *base = nullptr;   // the one block the buffers below are carved from
    int64_t max_m = 0;
    int64_t pool_rows = 0;  // capacity of the screen pool in (split, query) rows
    void *Zq = nullptr;
    double *ez = nullptr, *nzz = nullptr;
    uint64_t *pool = nullptr, *cand = nullptr;
    float *tq = nullptr;
    int32_t *fbl = nullptr, *fbc = nullptr, *nn = nullptr;
    uint64_t *nn_key = nullptr;  // split nearest-point search (FP64 models)
    int32_t *nn_idx = nullptr;
    uint64_t bytes = 0;
};

constexpr int PREDICT_MAX_SPLITS = 32;
constexpr int64_t WS_ROW_BYTES = 256;  // largest screening row (FP32, kp = 64)

constexpr uint64_t ws_align(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

// Bytes of a workspace for up to max_m queries whose screen pool holds
// pool_rows (split, query) rows, in the layout of predict_ws_carve: each
// buffer starts on a 256-byte boundary.
constexpr uint64_t predict_ws_span(int64_t max_m, int64_t pool_rows) {
    const uint64_t m_pad = (uint64_t)((max_m + SCREEN_QPB - 1) / SCREEN_QPB * SCREEN_QPB);
    return ws_align(m_pad * WS_ROW_BYTES)                      // Zq
           + 2 * ws_align((uint64_t)max_m * 8)                 // ez, nzz
           + ws_align((uint64_t)pool_rows * SCREEN_CAP * 8)    // pool
           + ws_align((uint64_t)pool_rows * SCREEN_CMAX * 8)   // cand (c' <= SCREEN_CMAX)
           + ws_align((uint64_t)pool_rows * 4)                 // tq
           + 2 * ws_align((uint64_t)max_m * 4)                 // fbl, nn
           + ws_align(16)                                      // fbc
           + ws_align((uint64_t)NN_SPLIT_ENTRIES * 8)          // nn_key
           + ws_align((uint64_t)NN_SPLIT_ENTRIES * 4);         // nn_idx
}

// Point the buffers of ws into [base, base + predict_ws_span(max_m,
// pool_rows)).  Nothing is allocated or written.
void predict_ws_carve(PredictWs *ws, void *base, int64_t max_m, int64_t pool_rows);
// Direct predictions of at least this many queries on a model with a pivot
// order use the pruned screen (enough workgroups to fill the device from one
// column range).
#ifndef FMG_PREDICT_PRUNE_MIN
#define FMG_PREDICT_PRUNE_MIN 65536
#endif
constexpr int64_t PREDICT_PRUNE_MIN = FMG_PREDICT_PRUNE_MIN;

fmg_status set_error(fmg_status st, const char *fmt, ...);
// Clear the calling thread's last error message.
void clear_error();
// Bytes of a workspace for max_m queries.
uint64_t predict_ws_bytes(int64_t max_m);
fmg_status predict_ws_alloc(PredictWs *ws, int64_t max_m);
void predict_ws_free(PredictWs *ws);
// Prediction for m queries on stream s; ws == nullptr allocates scratch
// stream-ordered, otherwise every buffer comes from ws (m <= ws->max_m).
fmg_status predict_run(fmg_model *M, const void *Z, int64_t m, void *out, int32_t *nn_out,
                       hipStream_t s, const PredictWs *ws);
// Move the model's arrays to pinned host memory and free their device memory
// (synchronous), or bring them back.  The arrays never change after the
// build, so host copies kept from an earlier offload are reused without a
// copy.  idle: no work on the device still reads the model, so neither a
// device-wide synchronisation nor a synchronising free is needed (its device
// arrays go to the library's array cache).  keep_host: keep the host copies
// for later offloads.
fmg_status model_offload(fmg_model *M, bool idle = false);
fmg_status model_restore(fmg_model *M, bool keep_host = false);

}  // namespace fmg
