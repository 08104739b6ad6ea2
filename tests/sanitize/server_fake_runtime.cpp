// Host-only implementations behind the server's thread-sanitizer build: the
// HIP stand-in of fake_hip/hip/hip_runtime.h, and fake versions of the
// library functions the server calls (prediction, workspaces, residency,
// error text).  The fake prediction of query q, response c of a model is
// (c + 1) * sum_j Z[q][j] + n, summed in order in the model's precision, so
// the driver can check every served row.  Test infrastructure only.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fastmuygps.h"
#include "fmg_internal.h"

struct FakeStream {
    std::mutex mu;
    bool capturing = false;
    FakeGraph *graph = nullptr;
};
struct FakeEvent {
    std::mutex mu;
    uint64_t seq = 0;
};
struct FakeGraph {
    std::vector<std::function<void()>> ops;
};

void fake_hip_enqueue(hipStream_t s, std::function<void()> op) {
    if (s) {
        std::lock_guard<std::mutex> l(s->mu);
        if (s->capturing) {
            s->graph->ops.push_back(std::move(op));
            return;
        }
    }
    op();
}

const char *hipGetErrorString(hipError_t) { return "fake HIP error"; }
hipError_t hipGetDevice(int *dev) {
    *dev = 0;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t bytes) {
    *p = calloc(1, bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) {
    free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) { return hipMalloc(p, bytes); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMemGetInfo(size_t *free_bytes, size_t *total_bytes) {
    *free_bytes = *total_bytes = (size_t)64 << 30;
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind) {
    memcpy(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind,
                          hipStream_t s) {
    fake_hip_enqueue(s, [dst, src, bytes] { memcpy(dst, src, bytes); });
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new FakeStream();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
    *e = new FakeEvent();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    std::lock_guard<std::mutex> l(e->mu);
    e->seq += 1;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::lock_guard<std::mutex> l(e->mu);
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    std::lock_guard<std::mutex> l(s->mu);
    if (s->capturing) return hipErrorInvalidValue;
    s->capturing = true;
    s->graph = new FakeGraph();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    std::lock_guard<std::mutex> l(s->mu);
    if (!s->capturing) return hipErrorInvalidValue;
    s->capturing = false;
    *g = s->graph;
    s->graph = nullptr;
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t g, hipGraphNode_t *, char *,
                               size_t) {
    *ge = new FakeGraph(*g);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ge, hipStream_t) {
    for (auto &op : ge->ops) op();
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ge) {
    delete ge;
    return hipSuccess;
}

namespace {
thread_local std::string g_err;
std::mutex g_viol_mu;
int g_violations = 0;
}  // namespace

// Calls of the fake prediction on a model that was not resident.
int fake_violations() {
    std::lock_guard<std::mutex> l(g_viol_mu);
    return g_violations;
}

extern "C" const char *fastmuygps_last_error(void) { return g_err.c_str(); }

namespace fmg {

fmg_status set_error(fmg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

uint64_t predict_ws_bytes(int64_t max_m) { return 4096 + (uint64_t)max_m * 16; }

fmg_status predict_ws_alloc(PredictWs *ws, int64_t max_m) {
    ws->bytes = predict_ws_bytes(max_m);
    ws->base = calloc(1, ws->bytes);
    ws->max_m = max_m;
    return ws->base ? FMG_OK : FMG_E_OOM;
}

void predict_ws_free(PredictWs *ws) {
    free(ws->base);
    ws->base = nullptr;
}

template <typename T>
void fake_predict(const T *Z, int64_t m, int d, int ell, int64_t n, T *out) {
    for (int64_t q = 0; q < m; ++q) {
        T s = 0;
        for (int j = 0; j < d; ++j) s += Z[q * d + j];
        for (int c = 0; c < ell; ++c) out[q * ell + c] = (T)(c + 1) * s + (T)n;
    }
}

fmg_status predict_run(fmg_model *M, const void *Z, int64_t m, void *out, int32_t *,
                       hipStream_t s, const PredictWs *ws) {
    if (!M->resident) {
        std::lock_guard<std::mutex> l(g_viol_mu);
        ++g_violations;
        return set_error(FMG_E_DEVICE, "prediction on a model that is not resident");
    }
    if (ws && m > ws->max_m) return set_error(FMG_E_INVALID_ARG, "batch beyond the workspace");
    const int d = M->d, ell = M->ell;
    const int64_t n = M->n;
    const bool f64 = M->prec == FMG_PREC_FP64;
    fake_hip_enqueue(s, [=] {
        if (f64)
            fake_predict((const double *)Z, m, d, ell, n, (double *)out);
        else
            fake_predict((const float *)Z, m, d, ell, n, (float *)out);
    });
    return FMG_OK;
}

fmg_status model_offload(fmg_model *M, bool) {
    M->resident = false;
    return FMG_OK;
}

fmg_status model_restore(fmg_model *M, bool) {
    M->resident = true;
    return FMG_OK;
}

}  // namespace fmg
