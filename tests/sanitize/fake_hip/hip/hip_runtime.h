// Host-only stand-in for the part of the HIP runtime API that the request
// server (fmg_server.hip) and the library's internal headers use, so that the
// server's host logic (admission, swapping, coalescing, graph bookkeeping,
// latency statistics, request parts) builds with g++ and a thread sanitizer
// on a machine without a GPU.  "Device" memory is host memory.  A stream runs
// each operation when it is enqueued, or records it while the stream is being
// captured; a graph replays what was recorded.  Events complete at once.
// Test infrastructure only: nothing of the library links it.
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>

typedef enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorMemoryAllocation = 2,
    hipErrorNotReady = 600,
} hipError_t;

typedef enum {
    hipMemcpyHostToHost = 0,
    hipMemcpyHostToDevice = 1,
    hipMemcpyDeviceToHost = 2,
    hipMemcpyDeviceToDevice = 3,
} hipMemcpyKind;

typedef enum { hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;

struct FakeStream;
struct FakeEvent;
struct FakeGraph;
typedef FakeStream *hipStream_t;
typedef FakeEvent *hipEvent_t;
typedef FakeGraph *hipGraph_t;
typedef FakeGraph *hipGraphExec_t;
typedef struct hipGraphNode *hipGraphNode_t;

#define hipStreamNonBlocking 0x01
#define hipEventDisableTiming 0x02
#define hipHostMallocDefault 0x0

const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *dev);
hipError_t hipSetDevice(int dev);
hipError_t hipGetLastError();
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags);
hipError_t hipHostFree(void *p);
hipError_t hipMemGetInfo(size_t *free_bytes, size_t *total_bytes);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind kind);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind,
                          hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *ge, hipGraph_t g, hipGraphNode_t *err_node,
                               char *log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t ge, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t ge);

// Runs op on stream s now, or records it while s is being captured.
void fake_hip_enqueue(hipStream_t s, std::function<void()> op);
