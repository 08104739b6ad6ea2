// Allocation-free prediction (fastmuygps_predict_noalloc): the prediction of
// fastmuygps_predict with every scratch buffer carved from one static device
// array per GPU instead of the stream-ordered pool.  For callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc.
//
// The array, `scratch`, is a file-scope __device__ variable, so every GPU the
// library runs on holds its own copy (NOALLOC_BYTES, about 87 MiB) until the
// process ends.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress, with
// that device current, and only that address is used.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fmg_internal.h"

namespace {

constexpr int64_t NOALLOC_MAX_M = FMG_NOALLOC_MAX_M;
// Screen pool rows: a batch of m queries gets min(32, rows / m_pad) candidate
// splits, so up to 1,024 queries keep the 16+ splits a small batch needs to
// fill the device, and 4,096 queries still take four.
constexpr int64_t NOALLOC_POOL_ROWS = 4 * NOALLOC_MAX_M;
constexpr uint64_t NOALLOC_BYTES = fmg::predict_ws_span(NOALLOC_MAX_M, NOALLOC_POOL_ROWS);

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_addr[MAX_DEVICES];  // device address of `scratch` on each device

}  // namespace

// Every allocation-free prediction on a GPU works in that GPU's copy.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// The device address of the current device's copy of `scratch` (dev must be
// current).  Looked up once per device and kept.
fmg_status scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fmg::set_error(FMG_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s",
                                  dev, hipGetErrorString(e));
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return FMG_OK;
}

}  // namespace

extern "C" {

uint64_t fastmuygps_noalloc_scratch_bytes(void) { return NOALLOC_BYTES; }

fmg_status fastmuygps_predict_noalloc(const fmg_model *model, const void *Z, int64_t m,
                                      void *out, int32_t *nn_out, void *stream) {
    fmg::clear_error();
    if (!model) return fmg::set_error(FMG_E_INVALID_ARG, "model is null");
    if (m < 0) return fmg::set_error(FMG_E_INVALID_ARG, "m = %lld < 0", (long long)m);
    if (m > NOALLOC_MAX_M)
        return fmg::set_error(FMG_E_INVALID_ARG,
                              "m = %lld exceeds the allocation-free limit of %lld queries "
                              "per call (split the batch, or use fastmuygps_predict)",
                              (long long)m, (long long)NOALLOC_MAX_M);
    if (m == 0) return FMG_OK;
    if (!Z || !out) return fmg::set_error(FMG_E_INVALID_ARG, "Z and out must not be null");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fmg::set_error(FMG_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fmg::set_error(FMG_E_UNSUPPORTED, "device %d beyond the %d this call serves", dev,
                              MAX_DEVICES);
    if (dev != model->device)
        return fmg::set_error(FMG_E_INVALID_ARG,
                              "the model lives on device %d but device %d is current",
                              model->device, dev);
    void *base = nullptr;
    fmg_status st = scratch_address(dev, &base);
    if (st != FMG_OK) return st;
    fmg::PredictWs ws;
    fmg::predict_ws_carve(&ws, base, NOALLOC_MAX_M, NOALLOC_POOL_ROWS);
    return fmg::predict_run(const_cast<fmg_model *>(model), Z, m, out, nn_out,
                            (hipStream_t)stream, &ws);
}

}  // extern "C"
