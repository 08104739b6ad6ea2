// Host runtime behind the C ABI (include/fastmuygps.h): argument checks, the
// model object and its device memory, and the order of kernel launches for
// offline training and online prediction (Algorithm 2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fastmuygps.h"
#include "fmg_device.h"
#include "fmg_internal.h"
#include "fmg_kernels.h"

using namespace fmg;

namespace {

thread_local std::string g_err;

fmg_status fail(fmg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

fmg_status hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(FMG_E_OOM, "%s: out of device memory (%s)", what, hipGetErrorString(e));
    return fail(FMG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                       \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

constexpr int MAX_DEVICES = 64;

// Scratch blocks of finished calls, kept per device for later calls to take
// at the same size (a build or a prediction asks for the same sizes each
// time).  A block carries the stream it was last used on and an event
// recorded there when it came back: a call on the same stream takes it at
// once (the stream runs its work in order), a call on another stream once
// the event has completed.  Up to SCRATCH_KEEP bytes are kept.  Every kernel
// that uses a call's scratch runs on that call's stream.  (The
// stream-ordered pool this replaces spent 0.3-0.6 ms of host time in every
// allocation and free of a large block, during which the device idled.)
constexpr size_t SCRATCH_KEEP = 16ull << 30;

struct ScratchBlock {
    void *p;
    hipStream_t stream;
    hipEvent_t ev;
};

struct ScratchCache {
    std::mutex mu;
    std::multimap<size_t, ScratchBlock> blocks;  // size -> block
    std::vector<hipEvent_t> spare;               // events of taken blocks
    size_t bytes = 0;
};

ScratchCache &scratch_cache(int dev) {
    static ScratchCache caches[MAX_DEVICES];
    return caches[dev >= 0 && dev < MAX_DEVICES ? dev : 0];
}

// Returns every cached block of device dev to the device (after its last
// user's work).
void scratch_cache_clear(int dev) {
    ScratchCache &c = scratch_cache(dev);
    std::lock_guard<std::mutex> lock(c.mu);
    for (auto &b : c.blocks) {
        (void)hipEventSynchronize(b.second.ev);
        (void)hipFree(b.second.p);
        (void)hipEventDestroy(b.second.ev);
    }
    c.blocks.clear();
    c.bytes = 0;
}

hipError_t scratch_take(void **p, size_t bytes, hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev >= 0 && dev < MAX_DEVICES) {
        ScratchCache &c = scratch_cache(dev);
        std::lock_guard<std::mutex> lock(c.mu);
        auto range = c.blocks.equal_range(bytes);
        for (auto it = range.first; it != range.second; ++it) {
            bool ready = it->second.stream == s;
            if (!ready) {
                const hipError_t q = hipEventQuery(it->second.ev);
                ready = q == hipSuccess;
                // "not ready" is an answer, not a failure: keep it from being
                // reported by the next launch check's hipGetLastError
                if (q == hipErrorNotReady) (void)hipGetLastError();
            }
            if (ready) {
                *p = it->second.p;
                c.spare.push_back(it->second.ev);
                c.bytes -= bytes;
                c.blocks.erase(it);
                return hipSuccess;
            }
        }
    }
    hipError_t e = hipMalloc(p, bytes);
    if ((e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) && dev >= 0 &&
        dev < MAX_DEVICES) {
        (void)hipGetLastError();
        scratch_cache_clear(dev);
        e = hipMalloc(p, bytes);
    }
    return e;
}

// p (bytes long) is no longer used by work enqueued after this point; work
// already enqueued on s may still use it.
void scratch_give(void *p, size_t bytes, hipStream_t s) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= MAX_DEVICES) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
        return;
    }
    ScratchCache &c = scratch_cache(dev);
    std::lock_guard<std::mutex> lock(c.mu);
    hipEvent_t ev = nullptr;
    if (!c.spare.empty()) {
        ev = c.spare.back();
        c.spare.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
        (void)hipFree(p);
        return;
    }
    if (hipEventRecord(ev, s) != hipSuccess) {
        // an event never recorded reads as complete: wait for the stream
        // instead, so that no other stream takes the block too early
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s);
    }
    // over the limit: cached blocks go back to the device, smallest first
    while (!c.blocks.empty() && c.bytes + bytes > SCRATCH_KEEP) {
        auto it = c.blocks.begin();
        (void)hipEventSynchronize(it->second.ev);
        (void)hipFree(it->second.p);
        c.spare.push_back(it->second.ev);
        c.bytes -= it->first;
        c.blocks.erase(it);
    }
    c.blocks.emplace(bytes, ScratchBlock{p, s, ev});
    c.bytes += bytes;
}

// Arrays of freed models, kept per device (up to ARRAY_CACHE_KEEP bytes) for
// later builds to take at the same size: a build-and-free cycle then neither
// maps nor unmaps memory (hipFree after kernels have touched the memory costs
// milliseconds).  A failed allocation returns the cache to the device first.
constexpr size_t ARRAY_CACHE_KEEP = 16ull << 30;

struct ArrayCache {
    std::mutex mu;
    std::multimap<size_t, void *> blocks;  // size -> block
    size_t bytes = 0;
};

ArrayCache &array_cache(int dev) {
    static ArrayCache caches[MAX_DEVICES];
    return caches[dev >= 0 && dev < MAX_DEVICES ? dev : 0];
}

void array_cache_clear(int dev) {
    ArrayCache &c = array_cache(dev);
    std::lock_guard<std::mutex> lock(c.mu);
    for (auto &b : c.blocks) (void)hipFree(b.second);
    c.blocks.clear();
    c.bytes = 0;
}

hipError_t array_alloc(void **p, size_t bytes) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev >= 0 && dev < MAX_DEVICES) {
        ArrayCache &c = array_cache(dev);
        std::lock_guard<std::mutex> lock(c.mu);
        auto it = c.blocks.find(bytes);
        if (it != c.blocks.end()) {
            *p = it->second;
            c.bytes -= bytes;
            c.blocks.erase(it);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(p, bytes);
    if ((e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) && dev >= 0 &&
        dev < MAX_DEVICES) {
        (void)hipGetLastError();
        array_cache_clear(dev);
        e = hipMalloc(p, bytes);
    }
    return e;
}

// p (bytes long, from array_alloc on device dev) is no longer used by any work.
void array_release(int dev, void *p, size_t bytes) {
    if (dev >= 0 && dev < MAX_DEVICES) {
        ArrayCache &c = array_cache(dev);
        std::lock_guard<std::mutex> lock(c.mu);
        if (c.bytes + bytes <= ARRAY_CACHE_KEEP) {
            c.blocks.emplace(bytes, p);
            c.bytes += bytes;
            return;
        }
    }
    (void)hipFree(p);
}

// Device scratch owned by one call: given back to the scratch cache (after
// the work enqueued on the call's stream) when the holder goes out of scope.
struct Scratch {
    hipStream_t stream = nullptr;
    std::vector<std::pair<void *, size_t>> blocks;
    ~Scratch() {
        for (auto &b : blocks) scratch_give(b.first, b.second, stream);
    }
    // Gives p back before the holder ends (work enqueued on the stream
    // before this call may still use it).
    void release(void *p) {
        for (auto &b : blocks)
            if (b.first == p) {
                scratch_give(b.first, b.second, stream);
                b = blocks.back();
                blocks.pop_back();
                return;
            }
    }
    hipError_t alloc(void **p, size_t bytes) {
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~(size_t)255;
        const hipError_t e = scratch_take(p, bytes, stream);
        if (e == hipSuccess) blocks.emplace_back(*p, bytes);
        return e;
    }
};

}  // namespace

namespace {

void **model_array(fmg_model *M, int idx);

void free_model(fmg_model *M) {
    if (!M) return;
    // The arrays go back to the device's cache; nothing may still read them
    // when a later build takes them.
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != M->device) (void)hipSetDevice(M->device);
    (void)hipDeviceSynchronize();
    for (int a = 0; a < MA_COUNT; ++a) {
        void **p = model_array(M, a);
        if (*p) array_release(M->device, *p, M->arr_bytes[a]);
        *p = nullptr;
    }
    if (M->pred_fb) array_release(M->device, M->pred_fb, M->fb_bytes);
    M->pred_fb = nullptr;
    if (cur >= 0 && cur != M->device) (void)hipSetDevice(cur);
    for (void *h : M->host)
        if (h) (void)hipHostFree(h);
    if (M->timing)
        for (int e = 0; e < EV_COUNT; ++e) {
            if (M->evb[e]) (void)hipEventDestroy(M->evb[e]);
            if (M->evp[e]) (void)hipEventDestroy(M->evp[e]);
        }
    delete M;
}

int kernel_code(const fmg_hyper &h) {
    if (h.kernel == FMG_KERNEL_RBF) return KC_RBF;
    if (h.kernel != FMG_KERNEL_MATERN) return -1;
    if (h.nu == 0.5) return KC_M12;
    if (h.nu == 1.5) return KC_M32;
    if (h.nu == 2.5) return KC_M52;
    return -1;
}

void record(fmg_model *M, hipEvent_t *ev, int idx, hipStream_t s) {
    if (M->timing) (void)hipEventRecord(ev[idx], s);
}

// Allocate one of the model's device arrays (idx < MA_COUNT: a movable
// array whose size is recorded for offloading).
fmg_status model_alloc(fmg_model *M, int idx, void **p, size_t bytes, const char *what) {
    if (bytes == 0) bytes = 16;
    hipError_t e = array_alloc(p, bytes);
    if (e != hipSuccess) return hip_fail(e, what);
    M->bytes += bytes;
    if (idx >= 0 && idx < MA_COUNT) M->arr_bytes[idx] = bytes;
    else M->fb_bytes = bytes;
    return FMG_OK;
}

void **model_array(fmg_model *M, int idx) {
    switch (idx) {
    case MA_X: return &M->X;
    case MA_N: return (void **)&M->N;
    case MA_C: return &M->C;
    case MA_XP: return &M->Xp;
    case MA_Y: return &M->Y;
    case MA_PERM: return (void **)&M->perm;
    case MA_XPP: return &M->Xpp;
    case MA_TC: return &M->tile_c;
    case MA_TR: return (void **)&M->tile_r;
    case MA_CELL: return (void **)&M->cell;
    case MA_KEYS: return (void **)&M->keys;
    case MA_BOX: return (void **)&M->box;
    case MA_SC: return &M->sup_c;
    case MA_SR: return (void **)&M->sup_r;
    case MA_GC: return &M->grp_c;
    case MA_GR: return (void **)&M->grp_r;
    default: return (void **)&M->mu;
    }
}

// Screening geometry for a precision mode and dimension.
bool screen_geom(int prec, int d, ScreenGeom *g) {
    if (prec == FMG_PREC_MIXED) {
        if (d + 3 > 64) return false;
        *g = ScreenGeom{SCREEN_BF16, 64, 2, 128};
        return true;
    }
    const int kp = (int)round_up(d + 1, 16);
    if (kp > 64) return false;
    *g = ScreenGeom{SCREEN_F32, kp, kp / 4, kp * 4};
    return true;
}

}  // namespace

namespace fmg {

void clear_error() { g_err.clear(); }

fmg_status set_error(fmg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

namespace {

// Screen splits of a prediction: enough (split, query-block) pairs to fill
// the device when the batch is small, bounded by the pool capacity.
int64_t predict_splits(const fmg_model *M, int64_t m_pad, const PredictWs *ws) {
    const int64_t qblocks = m_pad / SCREEN_QPB;
    int64_t splits = (512 + qblocks - 1) / qblocks;
    int64_t cap = PREDICT_MAX_SPLITS;
    if (ws) cap = ws->pool_rows / m_pad < cap ? ws->pool_rows / m_pad : cap;
    // at least 16 tiles of candidates per split
    const int64_t min_chunk = 16 * SCREEN_TILE;
    const int64_t by_size = M->n_pad / min_chunk > 0 ? M->n_pad / min_chunk : 1;
    if (splits > cap) splits = cap;
    if (splits > by_size) splits = by_size;
    return splits < 1 ? 1 : splits;
}

int64_t ws_pool_rows(int64_t max_m) {
    const int64_t m_pad = round_up(max_m, SCREEN_QPB);
    const int64_t qblocks = m_pad / SCREEN_QPB;
    int64_t splits = (512 + qblocks - 1) / qblocks;
    if (splits > PREDICT_MAX_SPLITS) splits = PREDICT_MAX_SPLITS;
    if (splits < 1) splits = 1;
    return splits * m_pad;
}

}  // namespace

uint64_t predict_ws_bytes(int64_t max_m) {
    return predict_ws_span(max_m, ws_pool_rows(max_m));
}

void predict_ws_carve(PredictWs *ws, void *base, int64_t max_m, int64_t pool_rows) {
    *ws = PredictWs{};
    const int64_t m_pad = round_up(max_m, SCREEN_QPB);
    char *p = (char *)base;
    auto take = [&p](uint64_t bytes) {
        void *q = p;
        p += ws_align(bytes);
        return q;
    };
    ws->base = base;
    ws->Zq = take((uint64_t)m_pad * WS_ROW_BYTES);
    ws->ez = (double *)take((uint64_t)max_m * 8);
    ws->nzz = (double *)take((uint64_t)max_m * 8);
    ws->pool = (uint64_t *)take((uint64_t)pool_rows * SCREEN_CAP * 8);
    ws->cand = (uint64_t *)take((uint64_t)pool_rows * SCREEN_CMAX * 8);
    ws->tq = (float *)take((uint64_t)pool_rows * 4);
    ws->fbl = (int32_t *)take((uint64_t)max_m * 4);
    ws->nn = (int32_t *)take((uint64_t)max_m * 4);
    ws->fbc = (int32_t *)take(16);
    ws->nn_key = (uint64_t *)take((uint64_t)NN_SPLIT_ENTRIES * 8);
    ws->nn_idx = (int32_t *)take((uint64_t)NN_SPLIT_ENTRIES * 4);
    ws->max_m = max_m;
    ws->pool_rows = pool_rows;
    ws->bytes = predict_ws_span(max_m, pool_rows);
}

fmg_status predict_ws_alloc(PredictWs *ws, int64_t max_m) {
    *ws = PredictWs{};
    if (max_m < 1) return fail(FMG_E_INVALID_ARG, "workspace for %lld queries", (long long)max_m);
    const int64_t m_pad = round_up(max_m, SCREEN_QPB);
    const int64_t rows = ws_pool_rows(max_m);
    void *base = nullptr;
    hipError_t e = hipMalloc(&base, predict_ws_span(max_m, rows));
    if (e != hipSuccess) return hip_fail(e, "prediction workspace");
    predict_ws_carve(ws, base, max_m, rows);
    // Query rows past a batch are read by the screen: keep them finite.
    e = hipMemset(ws->Zq, 0, (size_t)m_pad * WS_ROW_BYTES);
    if (e != hipSuccess) {
        predict_ws_free(ws);
        return hip_fail(e, "hipMemset");
    }
    return FMG_OK;
}

void predict_ws_free(PredictWs *ws) {
    if (ws->base) (void)hipFree(ws->base);
    *ws = PredictWs{};
}

fmg_status predict_run(fmg_model *M, const void *Z, int64_t m, void *out, int32_t *nn_out,
                       hipStream_t s, const PredictWs *ws) {
    if (!M->resident)
        return fail(FMG_E_BUSY, "the model is offloaded to host memory (not admitted)");
    if (ws && m > ws->max_m)
        return fail(FMG_E_INVALID_ARG, "batch of %lld queries exceeds the workspace (%lld)",
                    (long long)m, (long long)ws->max_m);
    const bool f64 = M->prec == FMG_PREC_FP64;
    Scratch tmp;
    tmp.stream = s;
    record(M, M->evp, EV_START, s);
    uint32_t *qperm = nullptr;  // pruned screens: queries in pivot order (also the gather's order)
    int32_t *nn = nn_out;
    if (!nn) {
        if (ws)
            nn = ws->nn;
        else
            HIPCHK(tmp.alloc((void **)&nn, (size_t)m * 4), "scratch");
    }
    if (f64) {
        record(M, M->evp, EV_PREP, s);
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = M->n;
        ea.d = M->d;
        ea.Qc = Z;
        ea.nq = m;
        ea.loo = 0;
        ea.k = 1;
        ea.out = nn;
        ea.out_stride = 1;
        if (ws) {
            ea.nn_key = ws->nn_key;
            ea.nn_idx = ws->nn_idx;
        } else {
            HIPCHK(tmp.alloc((void **)&ea.nn_key, (size_t)NN_SPLIT_ENTRIES * 8), "scratch");
            HIPCHK(tmp.alloc((void **)&ea.nn_idx, (size_t)NN_SPLIT_ENTRIES * 4), "scratch");
        }
        HIPCHK(launch_exact_topk(true, ea, m, s), "exact search");
        for (int e = EV_SCREEN; e <= EV_FALLBACK; ++e) record(M, M->evp, e, s);
    } else {
        const ScreenGeom &g = M->geom;
        const int64_t m_pad = round_up(m, SCREEN_QPB);
        // Large direct batches on a model with a pivot order take the pruned
        // screen: queries sorted by nearest pivot, one column range.
        const bool prune = !ws && M->perm && m >= PREDICT_PRUNE_MIN;
        int64_t splits = prune ? 1 : predict_splits(M, m_pad, ws);
        int64_t chunk = round_up((M->n_pad + splits - 1) / splits, SCREEN_TILE);
        splits = (M->n_pad + chunk - 1) / chunk;
        const int c = M->c_query;
        void *Zq = nullptr;
        double *ez = nullptr, *nzz = nullptr;
        uint64_t *pool = nullptr, *cand = nullptr;
        float *tq = nullptr;
        int32_t *fbl = nullptr, *fbc = nullptr;
        if (ws) {
            Zq = ws->Zq;
            ez = ws->ez;
            nzz = ws->nzz;
            pool = ws->pool;
            cand = ws->cand;
            tq = ws->tq;
            fbl = ws->fbl;
            fbc = ws->fbc;
        } else {
            HIPCHK(tmp.alloc(&Zq, (size_t)m_pad * g.row_bytes), "scratch");
            HIPCHK(tmp.alloc((void **)&ez, (size_t)m * 8), "scratch");
            HIPCHK(tmp.alloc((void **)&nzz, (size_t)m * 8), "scratch");
            HIPCHK(tmp.alloc((void **)&pool, (size_t)splits * m_pad * SCREEN_CAP * 8),
                   "screen pool");
            HIPCHK(tmp.alloc((void **)&cand, (size_t)splits * m * c * 8), "scratch");
            HIPCHK(tmp.alloc((void **)&tq, (size_t)splits * m * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&fbl, (size_t)m * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&fbc, 4), "scratch");
        }
        HIPCHK(launch_prep_rows(g, (const float *)Z, m, m_pad, M->d, M->mu, Zq, nullptr, ez, nzz,
                                nullptr, nullptr, s),
               "query rows");
        record(M, M->evp, EV_PREP, s);
        HIPCHK(launch_zero_u32(fbc, 1, s), "zero");
        ScreenArgs sa{};
        sa.Q = Zq;
        sa.P = M->Xp;
        sa.m = m;
        sa.m_pad = m_pad;
        sa.n = M->n;
        sa.n_pad = M->n_pad;
        sa.col_chunk = chunk;
        sa.splits = (int)splits;
        sa.loo = 0;
        sa.c = c;
        sa.pool = pool;
        sa.cand = cand;
        sa.tq = tq;
        if (prune) {
            uint32_t *ka = nullptr, *kb = nullptr, *va = nullptr;
            void *sort_tmp = nullptr, *Zq2 = nullptr;
            float *nzq = nullptr;
            int32_t *rot = nullptr;
            size_t sort_bytes = 0;
            HIPCHK(prune_query_sort_bytes(M->n, m, &sort_bytes), "sort size");
            HIPCHK(tmp.alloc((void **)&qperm, (size_t)m * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&ka, (size_t)m * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&kb, (size_t)m * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&va, (size_t)m * 4), "scratch");
            HIPCHK(tmp.alloc(&sort_tmp, sort_bytes), "scratch");
            HIPCHK(tmp.alloc(&Zq2, (size_t)m_pad * g.row_bytes), "scratch");
            HIPCHK(tmp.alloc((void **)&nzq, (size_t)m_pad * 4), "scratch");
            HIPCHK(tmp.alloc((void **)&rot, (size_t)(m_pad / SCREEN_QPB) * 4), "scratch");
            HIPCHK(launch_prune_queries((const float *)M->X, M->n, (const float *)Z, m, M->d, M->mu,
                                        sort_tmp, sort_bytes, M->cell + prune_pivots(M->n) + 1,
                                        M->box, ka, kb, va, qperm, g, Zq, nzz, m_pad, Zq2, nzq,
                                        M->keys, rot, s),
                   "query order");
            sa.Q = Zq2;
            sa.P = M->Xpp;
            sa.prune = 1;
            sa.tile_c = M->tile_c;
            sa.tile_r = M->tile_r;
            sa.sup_c = M->sup_c;
            sa.sup_r = M->sup_r;
            sa.grp_c = M->grp_c;
            sa.grp_r = M->grp_r;
            sa.nzq = nzq;
            sa.acc_coef = M->acc_coef;
            sa.nx_max = M->nx_max;
            sa.rot_tab = rot;
        }
        if (prune) record(M, M->evp, EV_PREP, s);  // the query order counts as ingest
        HIPCHK(launch_screen(g, sa, s), "screen");
        record(M, M->evp, EV_SCREEN, s);
        RerankArgs ra{};
        if (prune) {  // screen rows and indices are in pivot order
            ra.order = qperm;
            ra.cand_idx = M->perm;
            ra.n_idx = M->n;
        }
        ra.cand = cand;
        ra.tq = tq;
        ra.splits = (int)splits;
        ra.c = c;
        ra.m = m;
        ra.X = M->X;
        ra.Zc = Z;
        ra.d = M->d;
        ra.nzq = nzz;
        ra.eq = ez;
        ra.e_max = M->e_max;
        ra.acc_coef = M->acc_coef;
        ra.nx_max = M->nx_max;
        ra.k = 1;
        ra.self_first = 0;
        ra.out = nn;
        ra.out_stride = 1;
        ra.fb_list = fbl;
        ra.fb_count = fbc;
        HIPCHK(launch_rerank(ra, s), "re-rank");
        record(M, M->evp, EV_RERANK, s);
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = M->n;
        ea.d = M->d;
        ea.Qc = Z;
        ea.list = fbl;
        ea.count = fbc;
        ea.loo = 0;
        ea.k = 1;
        ea.out = nn;
        ea.out_stride = 1;
        HIPCHK(launch_exact_topk(false, ea, m, s), "exact rescan");
        HIPCHK(launch_accum(fbc, M->pred_fb, s), "count");
        record(M, M->evp, EV_FALLBACK, s);
    }
    GatherArgs ga{};
    ga.order = qperm;
    ga.X = M->X;
    ga.Z = Z;
    ga.nn = nn;
    ga.N = M->N;
    ga.C = M->C;
    ga.m = m;
    ga.zrows = m;
    ga.crows = M->n;
    ga.d = M->d;
    ga.ell = M->ell;
    ga.k = M->k;
    ga.kc = M->kc;
    ga.inv_rho = M->inv_rho;
    ga.amp = M->amp;
    ga.out = out;
    HIPCHK(launch_gather(f64, ga, s), "gather");
    record(M, M->evp, EV_LAST, s);
    if (M->timing) M->pred_recorded = true;
    return FMG_OK;
}

// Model files (fastmuygps_save / fastmuygps_load): an 8-byte tag, the
// format number, the model's parameters field by field at their native
// widths and byte order, the byte count of every array (0 where the model
// has none), then the arrays present, in array order.
constexpr char MODEL_TAG[8] = {'F', 'M', 'G', 'M', 'O', 'D', 'E', 'L'};
constexpr uint32_t MODEL_FORMAT = 1;

struct FileW {
    FILE *f;
    bool ok = true;
    template <class T>
    void field(T &v) {
        if (ok && fwrite(&v, sizeof v, 1, f) != 1) ok = false;
    }
    template <class T>
    void put(const T &v) {
        T c = v;
        field(c);
    }
    void bytes(const void *p, size_t n) {
        if (ok && n && fwrite(p, 1, n, f) != n) ok = false;
    }
};

struct FileR {
    FILE *f;
    bool ok = true;
    template <class T>
    void field(T &v) {
        if (ok && fread(&v, sizeof v, 1, f) != 1) ok = false;
    }
    template <class T>
    void get(T &v) {
        field(v);
    }
    void bytes(void *p, size_t n) {
        if (ok && n && fread(p, 1, n, f) != n) ok = false;
    }
};

// The parameters a prediction needs, in file order (io: FileW or FileR).
template <class IO>
void model_fields(fmg_model *M, IO &io) {
    io.field(M->n);
    io.field(M->d);
    io.field(M->ell);
    io.field(M->k);
    io.field(M->hyper.kernel);
    io.field(M->hyper.nu);
    io.field(M->hyper.length_scale);
    io.field(M->hyper.noise_var);
    io.field(M->hyper.amplitude);
    io.field(M->prec);
    io.field(M->flags);
    io.field(M->kc);
    io.field(M->inv_rho);
    io.field(M->amp);
    int32_t self = M->self_inc ? 1 : 0;
    io.field(self);
    M->self_inc = self != 0;
    io.field(M->geom.mode);
    io.field(M->geom.kp);
    io.field(M->geom.ksteps);
    io.field(M->geom.row_bytes);
    io.field(M->n_pad);
    io.field(M->e_max);
    io.field(M->nx_max);
    io.field(M->acc_coef);
    io.field(M->c_build);
    io.field(M->c_query);
    io.field(M->nonpd);
    io.field(M->build_fb);
    int32_t arrays = MA_COUNT;
    io.field(arrays);
    if (arrays != MA_COUNT) io.ok = false;
}

fmg_status model_offload(fmg_model *M, bool idle) {
    if (!M->resident) return FMG_OK;
    if (!idle) HIPCHK(hipDeviceSynchronize(), "sync");
    for (int a = 0; a < MA_COUNT; ++a) {
        void **p = model_array(M, a);
        if (!*p || M->host[a]) continue;  // host copies kept from an earlier offload
        void *h = nullptr;
        HIPCHK(hipHostMalloc(&h, M->arr_bytes[a], hipHostMallocDefault), "pinned host memory");
        M->host[a] = h;
        HIPCHK(hipMemcpy(h, *p, M->arr_bytes[a], hipMemcpyDeviceToHost), "offload copy");
    }
    for (int a = 0; a < MA_COUNT; ++a) {
        void **p = model_array(M, a);
        if (!*p) continue;
        if (idle)
            array_release(M->device, *p, M->arr_bytes[a]);
        else
            HIPCHK(hipFree(*p), "hipFree");
        *p = nullptr;
        M->bytes -= M->arr_bytes[a];
    }
    M->resident = false;
    return FMG_OK;
}

fmg_status model_restore(fmg_model *M, bool keep_host) {
    if (M->resident) return FMG_OK;
    for (int a = 0; a < MA_COUNT; ++a) {
        if (!M->host[a]) continue;
        void **p = model_array(M, a);
        hipError_t e = array_alloc(p, M->arr_bytes[a]);
        if (e != hipSuccess) {
            // undo: the model stays offloaded
            for (int b = 0; b < a; ++b) {
                void **q = model_array(M, b);
                if (M->host[b] && *q) {
                    (void)hipFree(*q);
                    *q = nullptr;
                    M->bytes -= M->arr_bytes[b];
                }
            }
            return hip_fail(e, "restore");
        }
        M->bytes += M->arr_bytes[a];
        HIPCHK(hipMemcpy(*p, M->host[a], M->arr_bytes[a], hipMemcpyHostToDevice), "restore copy");
    }
    if (!keep_host)
        for (int a = 0; a < MA_COUNT; ++a) {
            if (M->host[a]) (void)hipHostFree(M->host[a]);
            M->host[a] = nullptr;
        }
    M->resident = true;
    return FMG_OK;
}

}  // namespace fmg

extern "C" {

const char *fastmuygps_last_error(void) { return g_err.c_str(); }

const char *fastmuygps_version(void) { return "fastmuygps-gfx950 0.1"; }

fmg_status fastmuygps_debug_exp_nonpos(const double *x, double *y, int64_t n, void *stream) {
    g_err.clear();
    if (n < 0) return fail(FMG_E_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0) return FMG_OK;
    if (!x || !y) return fail(FMG_E_INVALID_ARG, "x and y must not be null");
    HIPCHK(launch_exp_nonpos64(x, y, n, (hipStream_t)stream), "exp kernel");
    return FMG_OK;
}

fmg_status fastmuygps_debug_exp_nonpos32(const float *x, float *y, int64_t n, void *stream) {
    g_err.clear();
    if (n < 0) return fail(FMG_E_INVALID_ARG, "n = %lld < 0", (long long)n);
    if (n == 0) return FMG_OK;
    if (!x || !y) return fail(FMG_E_INVALID_ARG, "x and y must not be null");
    HIPCHK(launch_exp_nonpos32(x, y, n, (hipStream_t)stream), "exp kernel");
    return FMG_OK;
}

fmg_status fastmuygps_release_cached(void) {
    g_err.clear();
    int dev = 0;
    HIPCHK(hipGetDevice(&dev), "hipGetDevice");
    HIPCHK(hipDeviceSynchronize(), "sync");
    if (dev >= 0 && dev < MAX_DEVICES) {
        array_cache_clear(dev);
        scratch_cache_clear(dev);
    }
    return FMG_OK;
}

void fastmuygps_free(fmg_model *model) { free_model(model); }

fmg_status fastmuygps_build(const void *X, const void *Y, int64_t n, int32_t d, int32_t ell,
                            int32_t k, const fmg_hyper *hyper, fmg_precision prec,
                            uint32_t flags, void *stream, fmg_model **out) {
    g_err.clear();
    if (!out) return fail(FMG_E_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!X || !Y || !hyper) return fail(FMG_E_INVALID_ARG, "X, Y and hyper must not be null");
    if (prec != FMG_PREC_FP64 && prec != FMG_PREC_FP32 && prec != FMG_PREC_MIXED)
        return fail(FMG_E_INVALID_ARG, "unknown precision %d", (int)prec);
    const bool self_inc = (flags & FMG_FLAG_SELF_INCLUSIVE) != 0;
    if (n < 2 || n > 2147483647LL) return fail(FMG_E_INVALID_ARG, "n = %lld out of range", (long long)n);
    if (d < 1) return fail(FMG_E_INVALID_ARG, "d = %d must be >= 1", d);
    if (ell < 1 || ell > 16) return fail(FMG_E_INVALID_ARG, "ell = %d must be in [1, 16]", ell);
    if (k < 1 || k > 256) return fail(FMG_E_INVALID_ARG, "k = %d must be in [1, 256]", k);
    if (k > 64 && prec == FMG_PREC_MIXED)
        return fail(FMG_E_UNSUPPORTED, "k = %d > 64 needs FP64 or FP32 precision", k);
    if (k > 64 && precompute_wide_lds_bytes(prec == FMG_PREC_FP64, k, d) > PRECOMPUTE_WIDE_LDS_MAX)
        return fail(FMG_E_UNSUPPORTED, "k = %d, d = %d: the neighbourhood factor does not fit "
                                       "160 KB of LDS", k, d);
    if (!self_inc && k > n - 1)
        return fail(FMG_E_INVALID_ARG, "leave-one-out needs k <= n-1 (k=%d, n=%lld)", k, (long long)n);
    if (self_inc && k > n)
        return fail(FMG_E_INVALID_ARG, "self-inclusive needs k <= n (k=%d, n=%lld)", k, (long long)n);
    if (!(hyper->length_scale > 0.0) || !std::isfinite(hyper->length_scale))
        return fail(FMG_E_INVALID_ARG, "length_scale must be positive and finite");
    if (!(hyper->noise_var >= 0.0) || !std::isfinite(hyper->noise_var))
        return fail(FMG_E_INVALID_ARG, "noise_var must be >= 0 and finite");
    const int kc = kernel_code(*hyper);
    if (kc < 0) return fail(FMG_E_INVALID_ARG, "kernel must be RBF or Matern with nu in {0.5, 1.5, 2.5}");
    ScreenGeom geom{};
    if (prec != FMG_PREC_FP64 && !screen_geom(prec, d, &geom))
        return fail(FMG_E_UNSUPPORTED, "d = %d too large for the %s screen", d,
                    prec == FMG_PREC_MIXED ? "BF16" : "FP32");

    hipStream_t s = (hipStream_t)stream;
    fmg_model *M = new fmg_model();
    M->n = n;
    M->d = d;
    M->ell = ell;
    M->k = k;
    M->hyper = *hyper;
    M->prec = prec;
    M->flags = flags;
    M->kc = kc;
    M->inv_rho = 1.0 / hyper->length_scale;
    M->amp = hyper->amplitude > 0.0 ? hyper->amplitude : 1.0;
    M->self_inc = self_inc;
    M->geom = geom;
    (void)hipGetDevice(&M->device);
    const bool f64 = prec == FMG_PREC_FP64;
    const size_t esz = f64 ? 8 : 4;
    fmg_status st;
    Scratch tmp;
    tmp.stream = s;

#define MCHK(expr)                  \
    do {                            \
        fmg_status s_ = (expr);     \
        if (s_ != FMG_OK) {         \
            free_model(M);          \
            return s_;              \
        }                           \
    } while (0)
#define HCHK(expr, what)                      \
    do {                                      \
        hipError_t e_ = (expr);               \
        if (e_ != hipSuccess) {               \
            free_model(M);                    \
            return hip_fail(e_, what);        \
        }                                     \
    } while (0)

    if (flags & FMG_FLAG_TIMING) {
        M->timing = true;
        for (int e = 0; e < EV_COUNT; ++e) {
            HCHK(hipEventCreate(&M->evb[e]), "hipEventCreate");
            HCHK(hipEventCreate(&M->evp[e]), "hipEventCreate");
        }
    }
    // X carries 64 zero elements past its last row: kernels may read a fixed
    // number of coordinates past the end of a row.
    MCHK(model_alloc(M, MA_X, &M->X, ((size_t)n * d + 64) * esz, "model X"));
    MCHK(model_alloc(M, MA_N, (void **)&M->N, (size_t)n * k * 4, "model N"));
    MCHK(model_alloc(M, MA_C, &M->C, (size_t)n * k * ell * esz, "model C"));
    MCHK(model_alloc(M, MA_Y, &M->Y, (size_t)n * ell * esz, "model Y"));
    MCHK(model_alloc(M, -1, (void **)&M->pred_fb, 8, "counters"));
    HCHK(hipMemsetAsync(M->pred_fb, 0, 8, s), "hipMemsetAsync");
    record(M, M->evb, EV_START, s);
    HCHK(hipMemcpyAsync(M->X, X, (size_t)n * d * esz, hipMemcpyDeviceToDevice, s), "copy X");
    HCHK(hipMemcpyAsync(M->Y, Y, (size_t)n * ell * esz, hipMemcpyDeviceToDevice, s), "copy Y");
    HCHK(hipMemsetAsync((char *)M->X + (size_t)n * d * esz, 0, 64 * esz, s), "hipMemsetAsync");

    // Inputs must be finite.
    int *flag = nullptr;
    HCHK(tmp.alloc((void **)&flag, 4), "scratch");
    HCHK(hipMemsetAsync(flag, 0, 4, s), "hipMemsetAsync");
    HCHK(launch_finite_check(X, f64, n * (int64_t)d, flag, s), "finite check");
    HCHK(launch_finite_check(Y, f64, n * (int64_t)ell, flag, s), "finite check");
    const int kk = self_inc ? k - 1 : k;  // neighbours found by search
    // The screened paths read the flag with the screening rows' maxima (one
    // synchronisation, after the pivot order has been enqueued); the others
    // read it now.
    const bool screened = !f64 && kk > 0;
    int hflag = 0;
    if (!screened) {
        HCHK(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s), "copy flag");
        HCHK(hipStreamSynchronize(s), "sync");
        if (hflag) {
            free_model(M);
            return fail(FMG_E_INVALID_ARG, "X or Y holds a non-finite value");
        }
    }
    unsigned long long *mx = nullptr;  // maxima of the rounding radii and squared norms
    // Reads the input flag and the maxima, and sets the certificate's
    // constants (FP32 and MIXED).
    auto read_maxima = [&]() -> fmg_status {
        unsigned long long hmx[2] = {0, 0};
        hipError_t e = hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(hmx, mx, 16, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "copy maxima");
        if (hflag) return fail(FMG_E_INVALID_ARG, "X or Y holds a non-finite value");
        memcpy(&M->e_max, &hmx[0], 8);
        memcpy(&M->nx_max, &hmx[1], 8);
        const double u = std::ldexp(1.0, -23);
        const double nt = 2.0 * geom.kp;
        M->acc_coef = nt * u / (1.0 - nt * u);
        M->c_query = 16;
        return FMG_OK;
    };
    // Screening rows (FP32 and MIXED): the candidate side is kept by the
    // model for the queries' search, the query side serves the build.
    int64_t n_pad = 0;
    bool prune = false;
    void *Xq = nullptr;
    double *ex = nullptr, *nzx = nullptr;
    if (kk == 0) {
        record(M, M->evb, EV_PREP, s);
        HCHK(launch_self_rows(M->N, n, s), "self rows");
        for (int e = EV_SCREEN; e <= EV_FALLBACK; ++e) record(M, M->evb, e, s);
    } else if (f64) {
        record(M, M->evb, EV_PREP, s);
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = n;
        ea.d = d;
        ea.Qc = M->X;
        ea.nq = n;
        ea.loo = 1;
        ea.k = kk;
        ea.self_first = self_inc;
        ea.out = M->N;
        ea.out_stride = k;
        HCHK(tmp.alloc((void **)&ea.nn_key, (size_t)NN_SPLIT_ENTRIES * 8), "scratch");
        HCHK(tmp.alloc((void **)&ea.nn_idx, (size_t)NN_SPLIT_ENTRIES * 4), "scratch");
        HCHK(launch_exact_topk(true, ea, n, s), "exact search");
        for (int e = EV_SCREEN; e <= EV_FALLBACK; ++e) record(M, M->evb, e, s);
    } else {
        // A pruned screen takes whole super-tiles of candidate rows.
        prune = !(flags & FMG_FLAG_NO_PRUNE) && prune_pivots(n) > 1 && d <= 64 &&
                round_up(n, SCREEN_SUPER_ROWS) / SCREEN_SUPER_ROWS <= SCREEN_SUPER_MAX;
        n_pad = round_up(n, prune ? SCREEN_SUPER_ROWS : SCREEN_QPB);
        M->n_pad = n_pad;
        MCHK(model_alloc(M, MA_MU, (void **)&M->mu, (size_t)d * 4, "model mu"));
        if (flags & FMG_FLAG_NO_CENTER)
            HCHK(hipMemsetAsync(M->mu, 0, (size_t)d * 4, s), "hipMemsetAsync");
        else {
            double *part = nullptr;
            HCHK(tmp.alloc((void **)&part, (size_t)col_mean_blocks(n) * d * 8), "scratch");
            HCHK(launch_col_mean(M->X, false, n, d, M->mu, part, s), "column mean");
        }
        MCHK(model_alloc(M, MA_XP, &M->Xp, (size_t)n_pad * geom.row_bytes, "model screen rows"));
        HCHK(tmp.alloc(&Xq, (size_t)n_pad * geom.row_bytes), "scratch");
        HCHK(tmp.alloc((void **)&ex, (size_t)n * 8), "scratch");
        HCHK(tmp.alloc((void **)&nzx, (size_t)n * 8), "scratch");
        HCHK(tmp.alloc((void **)&mx, 16), "scratch");
        HCHK(hipMemsetAsync(mx, 0, 16, s), "hipMemsetAsync");
        HCHK(launch_prep_rows(geom, (const float *)M->X, n, n_pad, d, M->mu, Xq, M->Xp, ex, nzx,
                              mx, mx + 1, s),
             "screen rows");
        record(M, M->evb, EV_PREP, s);
    }
    if (kk > 64 && !f64) {
        // Neighbourhoods wider than a wavefront: pooled exact search (the
        // screening rows above still serve the queries' nearest-point search).
        MCHK(read_maxima());
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = n;
        ea.d = d;
        ea.Qc = M->X;
        ea.nq = n;
        ea.loo = 1;
        ea.k = kk;
        ea.self_first = self_inc;
        ea.out = M->N;
        ea.out_stride = k;
        HCHK(launch_exact_topk(false, ea, n, s), "exact search");
        for (int e = EV_SCREEN; e <= EV_FALLBACK; ++e) record(M, M->evb, e, s);
    } else if (kk > 0 && !f64) {
        // Candidates per row: 2k for the BF16 screen; k + 8 for the FP32
        // screen, or 2k (at most SCREEN_CMAX) in up to four dimensions, where
        // many points cluster tightly and the screen's error bound is a
        // large fraction of the k-th distance, so that k + 8 candidates would
        // often leave rows uncertified (each such row is rescanned exactly).
        M->c_build = prec == FMG_PREC_MIXED ? 2 * kk
                     : d <= 4              ? (2 * kk < SCREEN_CMAX ? 2 * kk : SCREEN_CMAX)
                                           : kk + 8;
        if (M->c_build < kk + 8 && kk + 8 <= SCREEN_CMAX) M->c_build = kk + 8;
        const int c = M->c_build;
        uint64_t *pool = nullptr, *cand = nullptr;
        float *tq = nullptr;
        int32_t *fbl = nullptr, *fbc = nullptr;
        HCHK(tmp.alloc((void **)&pool, (size_t)n_pad * SCREEN_CAP * 8), "screen pool");
        HCHK(tmp.alloc((void **)&cand, (size_t)n * c * 8), "scratch");
        HCHK(tmp.alloc((void **)&tq, (size_t)n * 4), "scratch");
        HCHK(tmp.alloc((void **)&fbl, (size_t)n * 4), "scratch");
        HCHK(tmp.alloc((void **)&fbc, 4), "scratch");
        HCHK(hipMemsetAsync(fbc, 0, 4, s), "hipMemsetAsync");
        ScreenArgs sa{};
        sa.Q = Xq;
        sa.P = M->Xp;
        sa.m = n;
        sa.m_pad = n_pad;
        sa.n = n;
        sa.n_pad = n_pad;
        sa.col_chunk = n_pad;
        sa.splits = 1;
        sa.loo = 1;
        sa.c = c;
        sa.pool = pool;
        sa.cand = cand;
        sa.tq = tq;
        // Tile pruning: screen the self-join in nearest-pivot order, skipping
        // tiles whose bounding balls no query of a wavefront can reach; the
        // re-rank takes the rows in the same order and maps the candidates'
        // indices back.
        uint32_t *perm = nullptr;
        if (prune) {
            uint32_t *ka = nullptr, *va = nullptr;
            void *sort_tmp = nullptr, *Xq2 = nullptr;
            float *nzq = nullptr;
            size_t sort_bytes = 0;
            const int npiv = prune_pivots(n);
            const size_t tiles = (size_t)(n_pad / SCREEN_TILE);
            HCHK(prune_sort_bytes(n, &sort_bytes), "sort size");
            MCHK(model_alloc(M, MA_PERM, (void **)&M->perm, (size_t)n * 4, "model order"));
            MCHK(model_alloc(M, MA_XPP, &M->Xpp, (size_t)n_pad * geom.row_bytes, "model rows"));
            MCHK(model_alloc(M, MA_TC, &M->tile_c, tiles * geom.row_bytes, "model tiles"));
            MCHK(model_alloc(M, MA_TR, (void **)&M->tile_r, tiles * 4, "model tiles"));
            MCHK(model_alloc(M, MA_CELL, (void **)&M->cell, (size_t)(2 * npiv + 1) * 4,
                             "model cells"));
            MCHK(model_alloc(M, MA_KEYS, (void **)&M->keys, (size_t)n * 4, "model keys"));
            MCHK(model_alloc(M, MA_BOX, (void **)&M->box, 128 * 4, "model box"));
            const size_t nsup = (size_t)(n_pad / SCREEN_SUPER_ROWS);
            MCHK(model_alloc(M, MA_SC, &M->sup_c, nsup * geom.row_bytes, "model super-tiles"));
            MCHK(model_alloc(M, MA_SR, (void **)&M->sup_r, nsup * 4, "model super-tiles"));
            const size_t ngrp = (size_t)(n_pad / SCREEN_GROUP_ROWS);
            MCHK(model_alloc(M, MA_GC, &M->grp_c, ngrp * geom.row_bytes, "model tile groups"));
            MCHK(model_alloc(M, MA_GR, (void **)&M->grp_r, ngrp * 4, "model tile groups"));
            perm = M->perm;
            HCHK(tmp.alloc((void **)&ka, (size_t)n * 4), "scratch");
            HCHK(tmp.alloc((void **)&va, (size_t)n * 4), "scratch");
            HCHK(tmp.alloc(&sort_tmp, sort_bytes), "scratch");
            HCHK(tmp.alloc(&Xq2, (size_t)n_pad * geom.row_bytes), "scratch");
            HCHK(tmp.alloc((void **)&nzq, (size_t)n_pad * 4), "scratch");
            HCHK(launch_prune_order((const float *)M->X, n, d, M->mu, sort_tmp, sort_bytes,
                                    M->cell + npiv + 1, M->box, ka, M->keys, va, perm, s),
                 "pivot order");
            HCHK(launch_cell_starts(M->keys, n, npiv, M->cell, s), "cell starts");
            HCHK(launch_prune_rows(geom, Xq, M->Xp, nzx, perm, n, n_pad, d, Xq2, M->Xpp, nzq,
                                   M->tile_c, M->tile_r, M->grp_c, M->grp_r, M->sup_c,
                                   M->sup_r, s),
                 "pruning rows");
            MCHK(read_maxima());
            sa.Q = Xq2;
            sa.P = M->Xpp;
            sa.prune = 1;
            sa.tile_c = M->tile_c;
            sa.tile_r = M->tile_r;
            sa.sup_c = M->sup_c;
            sa.sup_r = M->sup_r;
            sa.grp_c = M->grp_c;
            sa.grp_r = M->grp_r;
            sa.nzq = nzq;
            sa.acc_coef = M->acc_coef;
            sa.nx_max = M->nx_max;
        }
        if (prune)
            record(M, M->evb, EV_PREP, s);  // the pivot order counts as ingest
        else
            MCHK(read_maxima());
        HCHK(launch_screen(geom, sa, s), "screen");
        record(M, M->evb, EV_SCREEN, s);
        RerankArgs ra{};
        if (prune) {  // screen rows and indices are in pivot order
            ra.order = perm;
            ra.cand_idx = perm;
            ra.n_idx = n;
        }
        ra.cand = cand;
        ra.tq = tq;
        ra.splits = 1;
        ra.c = c;
        ra.m = n;
        ra.X = M->X;
        ra.Zc = M->X;
        ra.d = d;
        ra.nzq = nzx;
        ra.eq = ex;
        ra.e_max = M->e_max;
        ra.acc_coef = M->acc_coef;
        ra.nx_max = M->nx_max;
        ra.k = kk;
        ra.self_first = self_inc;
        ra.out = M->N;
        ra.out_stride = k;
        ra.fb_list = fbl;
        ra.fb_count = fbc;
        HCHK(launch_rerank(ra, s), "re-rank");
        record(M, M->evb, EV_RERANK, s);
        // the screen's pools and candidate lists are dead after the re-rank:
        // return them while the device still works (a large free costs
        // milliseconds of host time)
        tmp.release(pool);
        tmp.release(cand);
        int hfb = 0;
        HCHK(hipMemcpyAsync(&hfb, fbc, 4, hipMemcpyDeviceToHost, s), "copy count");
        HCHK(hipStreamSynchronize(s), "sync");
        M->build_fb = hfb;
        if (hfb > 0) {
            ExactArgs ea{};
            ea.X = M->X;
            ea.n = n;
            ea.d = d;
            ea.Qc = M->X;
            ea.list = fbl;
            ea.count = fbc;
            ea.loo = 1;
            ea.k = kk;
            ea.self_first = self_inc;
            ea.out = M->N;
            ea.out_stride = k;
            HCHK(launch_exact_topk(false, ea, hfb, s), "exact rescan");
        }
        record(M, M->evb, EV_FALLBACK, s);
    }

    int32_t *status = nullptr;
    unsigned long long *nbad = nullptr;
    HCHK(tmp.alloc((void **)&status, (size_t)n * 4), "scratch");
    HCHK(tmp.alloc((void **)&nbad, 8), "scratch");
    HCHK(hipMemsetAsync(nbad, 0, 8, s), "hipMemsetAsync");
    PrecomputeArgs pa{};
    pa.X = M->X;  // the model's padded copy
    pa.Y = Y;
    pa.n = n;
    pa.d = d;
    pa.ell = ell;
    pa.k = k;
    pa.N = M->N;
    pa.C = M->C;
    pa.status = status;
    pa.kc = kc;
    pa.inv_rho = M->inv_rho;
    pa.amp = M->amp;
    pa.noise = hyper->noise_var;
    pa.order = M->perm;  // pivot order of a pruned screen: nearby points run together
    const bool refine = prec == FMG_PREC_MIXED && !(flags & FMG_FLAG_NO_REFINE);
    HCHK(launch_precompute(f64, refine, pa, s), "precompute");
    record(M, M->evb, EV_LAST, s);
    HCHK(launch_count_nonzero(status, n, nbad, s), "count");
    unsigned long long hbad = 0;
    HCHK(hipMemcpyAsync(&hbad, nbad, 8, hipMemcpyDeviceToHost, s), "copy count");
    HCHK(hipStreamSynchronize(s), "sync");
    M->nonpd = (int64_t)hbad;
    if (M->timing) {
        for (int e = 1; e < EV_COUNT; ++e) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, M->evb[e - 1], M->evb[e]);
            M->build_ms[e] = ms;
        }
        float tot = 0.f;
        (void)hipEventElapsedTime(&tot, M->evb[EV_START], M->evb[EV_LAST]);
        M->build_ms[0] = tot;
    }
#undef MCHK
#undef HCHK
    *out = M;
    if (M->nonpd > 0)
        return fail(FMG_E_NOT_PD, "%lld neighbourhood matrices were not positive definite",
                    (long long)M->nonpd);
    return FMG_OK;
}

fmg_status fastmuygps_predict(const fmg_model *model, const void *Z, int64_t m, void *out,
                              int32_t *nn_out, void *stream) {
    g_err.clear();
    if (!model) return fail(FMG_E_INVALID_ARG, "model is null");
    if (m < 0) return fail(FMG_E_INVALID_ARG, "m = %lld < 0", (long long)m);
    if (m == 0) return FMG_OK;
    if (m > 2147483647LL) return fail(FMG_E_INVALID_ARG, "m too large");
    if (!Z || !out) return fail(FMG_E_INVALID_ARG, "Z and out must not be null");
    return predict_run(const_cast<fmg_model *>(model), Z, m, out, nn_out, (hipStream_t)stream,
                       nullptr);
}

fmg_status fastmuygps_predict_muygps(const fmg_model *model, const void *Z, int64_t m, void *out,
                                     int32_t *nbr_out, void *stream) {
    g_err.clear();
    if (!model) return fail(FMG_E_INVALID_ARG, "model is null");
    if (m < 0) return fail(FMG_E_INVALID_ARG, "m = %lld < 0", (long long)m);
    if (m == 0) return FMG_OK;
    if (m > 2147483647LL) return fail(FMG_E_INVALID_ARG, "m too large");
    if (!Z || !out) return fail(FMG_E_INVALID_ARG, "Z and out must not be null");
    fmg_model *M = const_cast<fmg_model *>(model);
    if (!M->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = M->prec == FMG_PREC_FP64;
    const int k = M->k;
    const size_t esz = f64 ? 8 : 4;
    Scratch tmp;
    tmp.stream = s;
    int32_t *nb = nbr_out;
    if (!nb) HIPCHK(tmp.alloc((void **)&nb, (size_t)m * k * 4), "scratch");

    // 1. The query's own k nearest training points (nothing excluded); wider
    // neighbourhoods than a wavefront take the pooled exact search.
    if (f64 || k > 64) {
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = M->n;
        ea.d = M->d;
        ea.Qc = Z;
        ea.nq = m;
        ea.loo = 0;
        ea.k = k;
        ea.out = nb;
        ea.out_stride = k;
        HIPCHK(launch_exact_topk(f64, ea, m, s), "exact search");
    } else {
        const ScreenGeom &g = M->geom;
        const int64_t m_pad = round_up(m, SCREEN_QPB);
        int64_t splits = predict_splits(M, m_pad, nullptr);
        if (splits > 8) splits = 8;
        const int64_t chunk = round_up((M->n_pad + splits - 1) / splits, SCREEN_TILE);
        splits = (M->n_pad + chunk - 1) / chunk;
        const int c = M->prec == FMG_PREC_MIXED ? 2 * k : k + 8;
        void *Zq = nullptr;
        double *ez = nullptr, *nzz = nullptr;
        uint64_t *pool = nullptr, *cand = nullptr;
        float *tq = nullptr;
        int32_t *fbl = nullptr, *fbc = nullptr;
        HIPCHK(tmp.alloc(&Zq, (size_t)m_pad * g.row_bytes), "scratch");
        HIPCHK(tmp.alloc((void **)&ez, (size_t)m * 8), "scratch");
        HIPCHK(tmp.alloc((void **)&nzz, (size_t)m * 8), "scratch");
        HIPCHK(tmp.alloc((void **)&pool, (size_t)splits * m_pad * SCREEN_CAP * 8), "screen pool");
        HIPCHK(tmp.alloc((void **)&cand, (size_t)splits * m * c * 8), "scratch");
        HIPCHK(tmp.alloc((void **)&tq, (size_t)splits * m * 4), "scratch");
        HIPCHK(tmp.alloc((void **)&fbl, (size_t)m * 4), "scratch");
        HIPCHK(tmp.alloc((void **)&fbc, 4), "scratch");
        HIPCHK(launch_prep_rows(g, (const float *)Z, m, m_pad, M->d, M->mu, Zq, nullptr, ez, nzz,
                                nullptr, nullptr, s),
               "query rows");
        HIPCHK(launch_zero_u32((uint32_t *)fbc, 1, s), "zero");
        ScreenArgs sa{};
        sa.Q = Zq;
        sa.P = M->Xp;
        sa.m = m;
        sa.m_pad = m_pad;
        sa.n = M->n;
        sa.n_pad = M->n_pad;
        sa.col_chunk = chunk;
        sa.splits = (int)splits;
        sa.loo = 0;
        sa.c = c;
        sa.pool = pool;
        sa.cand = cand;
        sa.tq = tq;
        HIPCHK(launch_screen(g, sa, s), "screen");
        RerankArgs ra{};
        ra.cand = cand;
        ra.tq = tq;
        ra.splits = (int)splits;
        ra.c = c;
        ra.m = m;
        ra.X = M->X;
        ra.Zc = Z;
        ra.d = M->d;
        ra.nzq = nzz;
        ra.eq = ez;
        ra.e_max = M->e_max;
        ra.acc_coef = M->acc_coef;
        ra.nx_max = M->nx_max;
        ra.k = k;
        ra.self_first = 0;
        ra.out = nb;
        ra.out_stride = k;
        ra.fb_list = fbl;
        ra.fb_count = fbc;
        HIPCHK(launch_rerank(ra, s), "re-rank");
        ExactArgs ea{};
        ea.X = M->X;
        ea.n = M->n;
        ea.d = M->d;
        ea.Qc = Z;
        ea.list = fbl;
        ea.count = fbc;
        ea.loo = 0;
        ea.k = k;
        ea.out = nb;
        ea.out_stride = k;
        HIPCHK(launch_exact_topk(false, ea, m, s), "exact rescan");
    }

    // 2. Per-query coefficients K(X_N*, X_N*)^{-1} Y(X_N*), centred on z.
    void *Cz = nullptr;
    int32_t *stq = nullptr;
    HIPCHK(tmp.alloc(&Cz, (size_t)m * k * M->ell * esz), "scratch");
    HIPCHK(tmp.alloc((void **)&stq, (size_t)m * 4), "scratch");
    PrecomputeArgs pa{};
    pa.X = M->X;
    pa.Y = M->Y;
    pa.n = m;
    pa.d = M->d;
    pa.ell = M->ell;
    pa.k = k;
    pa.N = nb;
    pa.C = Cz;
    pa.status = stq;
    pa.kc = M->kc;
    pa.inv_rho = M->inv_rho;
    pa.amp = M->amp;
    pa.noise = M->hyper.noise_var;
    pa.Ctr = f64 ? nullptr : Z;
    const bool refine = M->prec == FMG_PREC_MIXED && !(M->flags & FMG_FLAG_NO_REFINE);
    HIPCHK(launch_precompute(f64, refine, pa, s), "precompute");

    // 3. mu(z) = K(z, X_N*) . C_z
    GatherArgs ga{};
    ga.X = M->X;
    ga.Z = Z;
    ga.N = nb;
    ga.C = Cz;
    ga.m = m;
    ga.zrows = m;
    ga.crows = m;
    ga.d = M->d;
    ga.ell = M->ell;
    ga.k = k;
    ga.kc = M->kc;
    ga.inv_rho = M->inv_rho;
    ga.amp = M->amp;
    ga.out = out;
    HIPCHK(launch_gather(f64, ga, s), "gather");
    return FMG_OK;
}

fmg_status fastmuygps_loo_predict(const fmg_model *model, const int32_t *rows, int64_t b,
                                  void *out, void *stream) {
    g_err.clear();
    if (!model) return fail(FMG_E_INVALID_ARG, "model is null");
    if (b < 0) return fail(FMG_E_INVALID_ARG, "b = %lld < 0", (long long)b);
    if (b == 0) return FMG_OK;
    if (b > 2147483647LL) return fail(FMG_E_INVALID_ARG, "b too large");
    if (!rows || !out) return fail(FMG_E_INVALID_ARG, "rows and out must not be null");
    const fmg_model *M = model;
    if (!M->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    GatherArgs ga{};
    ga.X = M->X;
    ga.Z = M->X;
    ga.zrow = rows;
    ga.nn = rows;
    ga.N = M->N;
    ga.C = M->C;
    ga.m = b;
    ga.zrows = M->n;
    ga.crows = M->n;
    ga.d = M->d;
    ga.ell = M->ell;
    ga.k = M->k;
    ga.kc = M->kc;
    ga.inv_rho = M->inv_rho;
    ga.amp = M->amp;
    ga.out = out;
    HIPCHK(launch_gather(M->prec == FMG_PREC_FP64, ga, (hipStream_t)stream), "gather");
    return FMG_OK;
}

fmg_status fastmuygps_loo_loss(const fmg_model *model, const int32_t *rows, int64_t b,
                               const fmg_hyper *hyper, double *loss, void *stream) {
    g_err.clear();
    if (!model || !rows || !hyper || !loss) return fail(FMG_E_INVALID_ARG, "null argument");
    if (b < 1 || b > 2147483647LL) return fail(FMG_E_INVALID_ARG, "b = %lld out of range", (long long)b);
    fmg_model *M = const_cast<fmg_model *>(model);
    if (M->self_inc)
        return fail(FMG_E_INVALID_ARG, "the loss needs leave-one-out neighbourhoods (the model "
                                       "was built self-inclusive)");
    if (!(hyper->length_scale > 0.0) || !std::isfinite(hyper->length_scale))
        return fail(FMG_E_INVALID_ARG, "length_scale must be positive and finite");
    if (!(hyper->noise_var >= 0.0) || !std::isfinite(hyper->noise_var))
        return fail(FMG_E_INVALID_ARG, "noise_var must be >= 0 and finite");
    const int kc = kernel_code(*hyper);
    if (kc < 0) return fail(FMG_E_INVALID_ARG, "kernel must be RBF or Matern with nu in {0.5, 1.5, 2.5}");
    if (!M->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = M->prec == FMG_PREC_FP64;
    const size_t esz = f64 ? 8 : 4;
    const int d = M->d, k = M->k, ell = M->ell;
    const double amp = hyper->amplitude > 0.0 ? hyper->amplitude : 1.0;
    Scratch tmp;
    tmp.stream = s;
    void *Xb = nullptr, *Yb = nullptr, *Cb = nullptr, *mu = nullptr;
    int32_t *Nb = nullptr, *st = nullptr;
    int *bad = nullptr;
    double *part = nullptr, *sum = nullptr;
    HIPCHK(tmp.alloc(&Xb, (size_t)b * d * esz), "scratch");
    HIPCHK(tmp.alloc(&Yb, (size_t)b * ell * esz), "scratch");
    HIPCHK(tmp.alloc(&Cb, (size_t)b * k * ell * esz), "scratch");
    HIPCHK(tmp.alloc(&mu, (size_t)b * ell * esz), "scratch");
    HIPCHK(tmp.alloc((void **)&Nb, (size_t)b * k * 4), "scratch");
    HIPCHK(tmp.alloc((void **)&st, (size_t)b * 4), "scratch");
    HIPCHK(tmp.alloc((void **)&bad, 4), "scratch");
    HIPCHK(tmp.alloc((void **)&part, (size_t)sq_err_blocks(b * ell) * 8), "scratch");
    HIPCHK(tmp.alloc((void **)&sum, 8), "scratch");
    HIPCHK(launch_zero_u32(bad, 1, s), "zero");
    HIPCHK(launch_batch_rows(f64, M->X, M->N, M->Y, rows, b, M->n, d, k, ell, Xb, Nb, Yb, bad, s),
           "batch rows");
    // C_i(theta) for the batch rows, over their (theta-independent) lists.
    PrecomputeArgs pa{};
    pa.X = M->X;
    pa.Y = M->Y;
    pa.n = b;
    pa.d = d;
    pa.ell = ell;
    pa.k = k;
    pa.N = Nb;
    pa.C = Cb;
    pa.status = st;
    pa.kc = kc;
    pa.inv_rho = 1.0 / hyper->length_scale;
    pa.amp = amp;
    pa.noise = hyper->noise_var;
    pa.Ctr = f64 ? nullptr : Xb;
    const bool refine = M->prec == FMG_PREC_MIXED && !(M->flags & FMG_FLAG_NO_REFINE);
    HIPCHK(launch_precompute(f64, refine, pa, s), "precompute");
    // Leave-one-out predictions K_theta(x_i, X_N(i)) . C_i(theta).
    GatherArgs ga{};
    ga.X = M->X;
    ga.Z = Xb;
    ga.N = Nb;
    ga.C = Cb;
    ga.m = b;
    ga.zrows = b;
    ga.crows = b;
    ga.d = d;
    ga.ell = ell;
    ga.k = k;
    ga.kc = kc;
    ga.inv_rho = pa.inv_rho;
    ga.amp = amp;
    ga.out = mu;
    HIPCHK(launch_gather(f64, ga, s), "gather");
    HIPCHK(launch_sq_err(f64, Yb, mu, b * (int64_t)ell, part, sum, s), "squared errors");
    double hsum = 0.0;
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hsum, sum, 8, hipMemcpyDeviceToHost, s), "copy loss");
    HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "copy flag");
    HIPCHK(hipStreamSynchronize(s), "sync");
    if (hbad) return fail(FMG_E_INVALID_ARG, "a row index is outside [0, n)");
    *loss = hsum / ((double)b * ell);
    return FMG_OK;
}

fmg_status fastmuygps_loo_loss_grad(const fmg_model *model, const int32_t *rows, int64_t b,
                                    const fmg_hyper *hyper, double *loss, double *grad,
                                    void *stream) {
    g_err.clear();
    if (!model || !rows || !hyper || !loss || !grad) return fail(FMG_E_INVALID_ARG, "null argument");
    if (b < 1 || b > 2147483647LL) return fail(FMG_E_INVALID_ARG, "b = %lld out of range", (long long)b);
    const fmg_model *M = model;
    if (M->self_inc)
        return fail(FMG_E_INVALID_ARG, "the loss needs leave-one-out neighbourhoods (the model "
                                       "was built self-inclusive)");
    if (!(hyper->length_scale > 0.0) || !std::isfinite(hyper->length_scale))
        return fail(FMG_E_INVALID_ARG, "length_scale must be positive and finite");
    if (!(hyper->noise_var >= 0.0) || !std::isfinite(hyper->noise_var))
        return fail(FMG_E_INVALID_ARG, "noise_var must be >= 0 and finite");
    const int kc = kernel_code(*hyper);
    if (kc < 0) return fail(FMG_E_INVALID_ARG, "kernel must be RBF or Matern with nu in {0.5, 1.5, 2.5}");
    if (M->k > 64)
        return fail(FMG_E_UNSUPPORTED, "k = %d: the gradient holds one neighbour per lane (k <= 64)",
                    M->k);
    if (loo_grad_lds_bytes(M->k, M->d) > 65536)
        return fail(FMG_E_UNSUPPORTED, "k = %d, d = %d: the gradient's staged rows exceed 64 KB",
                    M->k, M->d);
    if (!M->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    hipStream_t s = (hipStream_t)stream;
    Scratch tmp;
    tmp.stream = s;
    double *terms = nullptr, *part = nullptr, *sums = nullptr;
    int *bad = nullptr;
    HIPCHK(tmp.alloc((void **)&terms, (size_t)b * 3 * 8), "scratch");
    HIPCHK(tmp.alloc((void **)&part, (size_t)loo_grad_blocks(b) * 3 * 8), "scratch");
    HIPCHK(tmp.alloc((void **)&sums, 3 * 8), "scratch");
    HIPCHK(tmp.alloc((void **)&bad, 4), "scratch");
    HIPCHK(launch_zero_u32(bad, 1, s), "zero");
    GradArgs ga{};
    ga.X = M->X;
    ga.Y = M->Y;
    ga.N = M->N;
    ga.rows = rows;
    ga.b = b;
    ga.n = M->n;
    ga.d = M->d;
    ga.ell = M->ell;
    ga.k = M->k;
    ga.kc = kc;
    ga.inv_rho = 1.0 / hyper->length_scale;
    ga.amp = hyper->amplitude > 0.0 ? hyper->amplitude : 1.0;
    ga.noise = hyper->noise_var;
    ga.terms = terms;
    ga.bad = bad;
    HIPCHK(launch_loo_grad(M->prec == FMG_PREC_FP64, ga, part, sums, s), "loss gradient");
    double h[3] = {0.0, 0.0, 0.0};
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(h, sums, 3 * 8, hipMemcpyDeviceToHost, s), "copy sums");
    HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s), "copy flag");
    HIPCHK(hipStreamSynchronize(s), "sync");
    if (hbad) return fail(FMG_E_INVALID_ARG, "a row index is outside [0, n)");
    const double scale = 1.0 / ((double)b * M->ell);
    *loss = h[0] * scale;
    grad[0] = h[1] * scale;
    grad[1] = h[2] * scale;
    return FMG_OK;
}

fmg_status fastmuygps_info(const fmg_model *model, fmg_info *info) {
    g_err.clear();
    if (!model || !info) return fail(FMG_E_INVALID_ARG, "null argument");
    memset(info, 0, sizeof *info);
    info->n = model->n;
    info->d = model->d;
    info->ell = model->ell;
    info->k = model->k;
    info->precision = model->prec;
    info->screen_cands = model->c_build;
    info->query_cands = model->c_query;
    info->nonpd_rows = model->nonpd;
    info->build_fallback_rows = model->build_fb;
    info->device_bytes = model->bytes;
    HIPCHK(hipDeviceSynchronize(), "sync");
    unsigned long long v = 0;
    HIPCHK(hipMemcpy(&v, model->pred_fb, 8, hipMemcpyDeviceToHost), "copy counter");
    info->predict_fallback_rows = (int64_t)v;
    return FMG_OK;
}

fmg_status fastmuygps_save(const fmg_model *model, const char *path) {
    g_err.clear();
    if (!model || !path) return fail(FMG_E_INVALID_ARG, "null argument");
    fmg_model *M = const_cast<fmg_model *>(model);
    HIPCHK(hipDeviceSynchronize(), "sync");
    FILE *f = fopen(path, "wb");
    if (!f) return fail(FMG_E_IO, "cannot open %s for writing", path);
    FileW w{f};
    w.bytes(MODEL_TAG, sizeof MODEL_TAG);
    w.put(MODEL_FORMAT);
    model_fields(M, w);
    uint64_t sizes[MA_COUNT];
    for (int a = 0; a < MA_COUNT; ++a) {
        const bool present = *model_array(M, a) != nullptr || M->host[a] != nullptr;
        sizes[a] = present ? (uint64_t)M->arr_bytes[a] : 0;
        w.put(sizes[a]);
    }
    std::vector<char> buf;
    for (int a = 0; a < MA_COUNT && w.ok; ++a) {
        if (sizes[a] == 0) continue;
        const void *src = M->host[a];
        if (!src) {
            buf.resize(sizes[a]);
            const hipError_t e =
                hipMemcpy(buf.data(), *model_array(M, a), sizes[a], hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                fclose(f);
                return hip_fail(e, "copy to host");
            }
            src = buf.data();
        }
        w.bytes(src, sizes[a]);
    }
    const bool closed = fclose(f) == 0;
    if (!w.ok || !closed) return fail(FMG_E_IO, "writing %s failed", path);
    return FMG_OK;
}

fmg_status fastmuygps_load(const char *path, fmg_model **out) {
    g_err.clear();
    if (!path || !out) return fail(FMG_E_INVALID_ARG, "null argument");
    *out = nullptr;
    FILE *f = fopen(path, "rb");
    if (!f) return fail(FMG_E_IO, "cannot open %s", path);
    FileR r{f};
    char tag[sizeof MODEL_TAG];
    uint32_t format = 0;
    r.bytes(tag, sizeof tag);
    r.get(format);
    if (!r.ok || memcmp(tag, MODEL_TAG, sizeof tag) != 0 || format != MODEL_FORMAT) {
        fclose(f);
        return fail(FMG_E_IO, "%s is not a model file of format %u", path, MODEL_FORMAT);
    }
    fmg_model *M = new fmg_model();
    auto bad = [&](fmg_status st) {
        fclose(f);
        free_model(M);
        return st;
    };
    (void)hipGetDevice(&M->device);
    model_fields(M, r);
    uint64_t sizes[MA_COUNT];
    for (int a = 0; a < MA_COUNT; ++a) r.get(sizes[a]);
    const bool shape_ok = M->n >= 1 && M->d >= 1 && M->ell >= 1 && M->ell <= 16 && M->k >= 1 &&
                          M->k <= 256 && M->k <= M->n && M->n_pad >= 0 &&
                          (M->prec == FMG_PREC_FP64 || M->prec == FMG_PREC_FP32 ||
                           M->prec == FMG_PREC_MIXED) &&
                          kernel_code(M->hyper) == M->kc && sizes[MA_X] > 0 &&
                          sizes[MA_N] >= (uint64_t)M->n * M->k * 4 && sizes[MA_C] > 0;
    bool sizes_ok = true;
    uint64_t body = 0;
    for (int a = 0; a < MA_COUNT; ++a) {
        sizes_ok = sizes_ok && sizes[a] <= (1ull << 40);
        body += sizes[a];
    }
    if (!r.ok || !shape_ok || !sizes_ok) {
        fail(FMG_E_IO, "%s: malformed model header", path);
        return bad(FMG_E_IO);
    }
    // the arrays must fill the rest of the file exactly (checked before any
    // allocation, so that a damaged header cannot ask for absurd sizes)
    const long here = ftell(f);
    if (here < 0 || fseek(f, 0, SEEK_END) != 0) {
        fail(FMG_E_IO, "%s: cannot seek", path);
        return bad(FMG_E_IO);
    }
    const long end = ftell(f);
    if (end < here || (uint64_t)(end - here) != body || fseek(f, here, SEEK_SET) != 0) {
        fail(FMG_E_IO, "%s holds %lld bytes of arrays where its header names %llu", path,
             (long long)(end - here), (unsigned long long)body);
        return bad(FMG_E_IO);
    }
    std::vector<char> buf;
    for (int a = 0; a < MA_COUNT; ++a) {
        if (sizes[a] == 0) continue;
        buf.resize(sizes[a]);
        r.bytes(buf.data(), sizes[a]);
        if (!r.ok) {
            fail(FMG_E_IO, "%s is truncated", path);
            return bad(FMG_E_IO);
        }
        void **p = model_array(M, a);
        const fmg_status st = model_alloc(M, a, p, sizes[a], "model array");
        if (st != FMG_OK) return bad(st);
        const hipError_t e = hipMemcpy(*p, buf.data(), sizes[a], hipMemcpyHostToDevice);
        if (e != hipSuccess) return bad(hip_fail(e, "copy to device"));
    }
    if (fgetc(f) != EOF) {
        fail(FMG_E_IO, "%s has bytes past the last array", path);
        return bad(FMG_E_IO);
    }
    fclose(f);
    const fmg_status st = model_alloc(M, -1, (void **)&M->pred_fb, 8, "counters");
    if (st != FMG_OK) {
        free_model(M);
        return st;
    }
    const hipError_t e = hipMemset(M->pred_fb, 0, 8);
    if (e != hipSuccess) {
        free_model(M);
        return hip_fail(e, "hipMemset");
    }
    *out = M;
    return FMG_OK;
}

fmg_status fastmuygps_neighbors(const fmg_model *model, int32_t *dev_out, void *stream) {
    g_err.clear();
    if (!model || !dev_out) return fail(FMG_E_INVALID_ARG, "null argument");
    if (!model->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    HIPCHK(hipMemcpyAsync(dev_out, model->N, (size_t)model->n * model->k * 4,
                          hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "copy N");
    return FMG_OK;
}

fmg_status fastmuygps_coeffs(const fmg_model *model, void *dev_out, void *stream) {
    g_err.clear();
    if (!model || !dev_out) return fail(FMG_E_INVALID_ARG, "null argument");
    if (!model->resident) return fail(FMG_E_BUSY, "the model is offloaded to host memory");
    const size_t esz = model->prec == FMG_PREC_FP64 ? 8 : 4;
    HIPCHK(hipMemcpyAsync(dev_out, model->C, (size_t)model->n * model->k * model->ell * esz,
                          hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "copy C");
    return FMG_OK;
}

fmg_status fastmuygps_timings(const fmg_model *model, fmg_timings *t) {
    g_err.clear();
    if (!model || !t) return fail(FMG_E_INVALID_ARG, "null argument");
    if (!model->timing) return fail(FMG_E_INVALID_ARG, "model was built without FMG_FLAG_TIMING");
    memset(t, 0, sizeof *t);
    t->build_prep_ms = model->build_ms[EV_PREP];
    t->build_screen_ms = model->build_ms[EV_SCREEN];
    t->build_rerank_ms = model->build_ms[EV_RERANK];
    t->build_fallback_ms = model->build_ms[EV_FALLBACK];
    t->build_precompute_ms = model->build_ms[EV_LAST];
    t->build_total_ms = model->build_ms[0];
    if (model->pred_recorded) {
        HIPCHK(hipEventSynchronize(model->evp[EV_LAST]), "event sync");
        double v[EV_COUNT] = {0};
        for (int e = 1; e < EV_COUNT; ++e) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, model->evp[e - 1], model->evp[e]), "elapsed");
            v[e] = ms;
        }
        float tot = 0.f;
        HIPCHK(hipEventElapsedTime(&tot, model->evp[EV_START], model->evp[EV_LAST]), "elapsed");
        t->predict_prep_ms = v[EV_PREP];
        t->predict_screen_ms = v[EV_SCREEN];
        t->predict_rerank_ms = v[EV_RERANK];
        t->predict_fallback_ms = v[EV_FALLBACK];
        t->predict_gather_ms = v[EV_LAST];
        t->predict_total_ms = tot;
    }
    return FMG_OK;
}

}  // extern "C"
