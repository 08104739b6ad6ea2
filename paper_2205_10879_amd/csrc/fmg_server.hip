// Request server of the library: resident models within an HBM budget and a
// continuous-batching loop over several in-flight slots.
//
//   submit  -> per-model FIFO of requests (host buffers, arrival time)
//   dispatcher thread: whenever a slot is free, coalesce the queued requests
//       of one admitted model (round robin over models) up to max_batch
//       queries, gather them into the slot's pinned buffer, and enqueue on
//       the slot's stream: copy in, prediction (Algorithm 2, prediction
//       loop) with the slot's preallocated workspace, copy out, event;
//   completer thread: waits for slots in launch order, scatters the results
//       to the requests' host buffers, records latencies, frees the slot.
// Batches of different slots overlap on the device.  With graphs enabled
// the enqueued sequence of a batch is captured once per (model, slot,
// batch-size bucket) and replayed; the queries past the batch in a bucket
// repeat its last query and their results are dropped.  Models that do not
// fit the budget wait in pinned host memory; with swap_idle, a waiting model
// with requests is swapped in for idle resident ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "fastmuygps.h"
#include "fmg_internal.h"

using namespace fmg;

struct fmg_request {
    int32_t model = -1;
    const void *Z = nullptr;
    void *out = nullptr;
    int32_t B = 0;
    int64_t arrival_ns = 0;
    double latency_ms = 0.0;
    fmg_status status = FMG_OK;
    bool done = false;
    std::mutex mu;
    std::condition_variable cv;
    // A request of more than max_batch queries is queued as parts of at most
    // max_batch queries each; the parts point at their parent (the ticket),
    // which counts the parts still running and completes with the last.
    fmg_request *parent = nullptr;
    int parts = 0;
};

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr int SLOT_MAX_D = 64;
constexpr int SLOT_MAX_ELL = 16;

// What completing a request (or a part) finished: the whole request, with
// its status, latency and arrival, or nothing yet (parts still running).
struct Finished {
    bool whole = false;
    fmg_status status = FMG_OK;
    double ms = 0.0;
    int64_t arrival_ns = 0;
};

// Marks r done with status st at t_done and wakes its waiter.  A part folds
// its status into its parent and is deleted here (nobody waits on a part);
// the parent completes with its last part.  Neither r nor its parent may be
// used after this call: the waiter deletes a completed request.
Finished finish(fmg_request *r, fmg_status st, int64_t t_done) {
    Finished f;
    fmg_request *const p = r->parent;
    fmg_request *const w = p ? p : r;  // the request that may complete
    if (p) delete r;
    std::lock_guard<std::mutex> l(w->mu);
    if (p) {
        if (st != FMG_OK && w->status == FMG_OK) w->status = st;
        if (--w->parts > 0) return f;
    } else {
        w->status = st;
    }
    w->latency_ms = (double)(t_done - w->arrival_ns) * 1e-6;
    f.whole = true;
    f.status = w->status;
    f.ms = w->latency_ms;
    f.arrival_ns = w->arrival_ns;
    w->done = true;
    w->cv.notify_all();
    return f;
}

struct ServerModel {
    fmg_model *M = nullptr;
    uint64_t footprint = 0;
    bool admitted = false;
    bool removed = false;
    bool loading = false;      // being swapped in (budget reserved, not yet admitted)
    int64_t last_use = 0;      // ns: last dispatch (least recently used is swapped out first)
    int64_t admitted_at = 0;   // ns
    int running = 0;  // slots holding a batch of this model
    std::deque<fmg_request *> queue;
    size_t esz = 4;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void *Zh = nullptr, *Oh = nullptr;  // pinned host staging
    void *Zd = nullptr, *Od = nullptr;
    PredictWs ws;
    bool busy = false;
    int32_t model = -1;
    int64_t count = 0;
    fmg_status launch_status = FMG_OK;
    std::vector<fmg_request *> reqs;
    std::map<std::pair<int32_t, int64_t>, hipGraphExec_t> graphs;
};

int64_t bucket_of(int64_t m, int64_t max_batch) {
    int64_t b = m <= 4096 ? (m + 255) / 256 * 256 : (m + 2047) / 2048 * 2048;
    return b < max_batch ? b : max_batch;
}

}  // namespace

struct fmg_server {
    uint64_t budget = 0;
    fmg_server_opts opts{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work;      // dispatcher: requests or slots
    std::condition_variable cv_inflight;  // completer: launched slots
    std::condition_variable cv_idle;      // removal and destruction: model drained
    std::deque<ServerModel> models;  // ids index it; references stay valid
    std::deque<int32_t> waiting;  // models waiting for admission, first come first
    std::vector<Slot> slots;
    std::deque<int> inflight;
    uint64_t ws_bytes = 0, resident = 0, peak = 0;
    int rr = 0;
    bool stop = false;
    bool dispatch_done = false;
    std::thread dispatcher, completer;
    // statistics
    std::vector<double> lat;
    int64_t n_req = 0, n_q = 0, n_batch = 0, n_swaps = 0;
    int64_t t_first = 0, t_last = 0;

    void note_resident() { peak = std::max(peak, resident); }
    void dispatch_loop();
    void complete_loop();
    fmg_status launch(Slot &sl, ServerModel &sm, int64_t m);
    void admit_waiting();
    bool swap_in(std::unique_lock<std::mutex> &l);
};

// A resident model is swapped out only after it has been resident this long
// (a quantum against thrashing when every model has a stream of requests).
constexpr int64_t SWAP_MIN_RESIDENT_NS = 50'000'000;

// Swap policy (opts.swap_idle): the first waiting model with queued requests
// is brought in, swapping out idle resident models (no queued or running
// batch), least recently used first, until it fits the budget.  The budget
// accounting changes under the lock; the copies run without it (the
// completer keeps finishing other slots' batches), in the dispatcher thread.
// The swapped-out models join the waiting list and come back the same way
// when requests for them arrive.  Returns whether a swap was made.
bool fmg_server::swap_in(std::unique_lock<std::mutex> &l) {
    int w = -1;
    for (int32_t id : waiting) {
        const ServerModel &sm = models[id];
        if (!sm.removed && !sm.loading && !sm.queue.empty()) {
            w = id;
            break;
        }
    }
    if (w < 0) return false;
    const int64_t t = now_ns();
    const uint64_t need = models[w].footprint;
    std::vector<int32_t> idle;
    for (int32_t id = 0; id < (int32_t)models.size(); ++id) {
        const ServerModel &sm = models[id];
        if (sm.admitted && !sm.removed && sm.queue.empty() && sm.running == 0 &&
            t - sm.admitted_at >= SWAP_MIN_RESIDENT_NS)
            idle.push_back(id);
    }
    std::sort(idle.begin(), idle.end(),
              [&](int32_t x, int32_t y) { return models[x].last_use < models[y].last_use; });
    uint64_t res = resident;
    std::vector<int32_t> out;
    for (int32_t id : idle) {
        if (res + need <= budget) break;
        out.push_back(id);
        res -= models[id].footprint;
    }
    if (res + need > budget) return false;
    // Their graphs hold the device addresses of the arrays that are about to
    // move: drop them (none is in flight: the models are idle, and only this
    // thread launches or captures graphs).
    for (int32_t id : out) {
        ServerModel &sm = models[id];
        sm.admitted = false;
        resident -= sm.footprint;
        waiting.push_back(id);
        for (Slot &sl : slots)
            for (auto it = sl.graphs.begin(); it != sl.graphs.end();) {
                if (it->first.first == id) {
                    (void)hipGraphExecDestroy(it->second);
                    it = sl.graphs.erase(it);
                } else {
                    ++it;
                }
            }
    }
    ServerModel &in = models[w];
    in.loading = true;
    resident += need;
    waiting.erase(std::find(waiting.begin(), waiting.end(), w));
    l.unlock();
    fmg_status st = FMG_OK;
    for (int32_t id : out) {
        fmg_status so = model_offload(models[id].M, true);
        if (so != FMG_OK) st = so;
    }
    if (st == FMG_OK) st = model_restore(in.M, true);
    l.lock();
    in.loading = false;
    if (st != FMG_OK) {  // stays waiting; the swapped-out models wait as well
        resident -= need;
        waiting.push_front(w);
        return false;
    }
    in.admitted = true;
    in.admitted_at = now_ns();
    n_swaps += 1;
    note_resident();
    return true;
}

fmg_status fmg_server::launch(Slot &sl, ServerModel &sm, int64_t m) {
    fmg_model *M = sm.M;
    const size_t esz = sm.esz;
    const bool graphs = opts.use_graphs != 0;
    const int64_t mb = graphs ? bucket_of(m, opts.max_batch) : m;
    auto enqueue = [&]() -> fmg_status {
        hipError_t e = hipMemcpyAsync(sl.Zd, sl.Zh, (size_t)mb * M->d * esz,
                                      hipMemcpyHostToDevice, sl.stream);
        if (e != hipSuccess) return set_error(FMG_E_DEVICE, "copy in: %s", hipGetErrorString(e));
        fmg_status st = predict_run(M, sl.Zd, mb, sl.Od, nullptr, sl.stream, &sl.ws);
        if (st != FMG_OK) return st;
        e = hipMemcpyAsync(sl.Oh, sl.Od, (size_t)mb * M->ell * esz, hipMemcpyDeviceToHost,
                           sl.stream);
        if (e != hipSuccess) return set_error(FMG_E_DEVICE, "copy out: %s", hipGetErrorString(e));
        return FMG_OK;
    };
    fmg_status st = FMG_OK;
    if (!graphs) {
        st = enqueue();
    } else {
        const auto key = std::make_pair(sl.model, mb);
        auto it = sl.graphs.find(key);
        if (it == sl.graphs.end()) {
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess)
                return set_error(FMG_E_DEVICE, "begin capture: %s", hipGetErrorString(e));
            st = enqueue();
            e = hipStreamEndCapture(sl.stream, &g);
            if (st != FMG_OK) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess)
                return set_error(FMG_E_DEVICE, "end capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess)
                return set_error(FMG_E_DEVICE, "instantiate: %s", hipGetErrorString(e));
            it = sl.graphs.emplace(key, ge).first;
        }
        hipError_t e = hipGraphLaunch(it->second, sl.stream);
        if (e != hipSuccess) return set_error(FMG_E_DEVICE, "graph launch: %s", hipGetErrorString(e));
    }
    if (st != FMG_OK) return st;
    hipError_t e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return set_error(FMG_E_DEVICE, "event: %s", hipGetErrorString(e));
    return FMG_OK;
}

void fmg_server::dispatch_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> l(mu);
    for (;;) {
        int free_slot = -1;
        for (size_t i = 0; i < slots.size(); ++i)
            if (!slots[i].busy) {
                free_slot = (int)i;
                break;
            }
        int pick = -1;
        if (free_slot >= 0) {
            const int nm = (int)models.size();
            for (int t = 0; t < nm; ++t) {
                const int id = (rr + t) % nm;
                const ServerModel &sm = models[id];
                if (sm.admitted && !sm.removed && !sm.queue.empty()) {
                    pick = id;
                    break;
                }
            }
        }
        if (free_slot >= 0 && opts.swap_idle && !waiting.empty() && swap_in(l)) continue;
        if (pick < 0) {
            if (stop) break;
            if (opts.swap_idle && !waiting.empty())
                cv_work.wait_for(l, std::chrono::milliseconds(5));  // models may turn idle
            else
                cv_work.wait(l);
            continue;
        }
        rr = (pick + 1) % (int)models.size();
        ServerModel &sm = models[pick];
        sm.last_use = now_ns();
        Slot &sl = slots[free_slot];
        sl.busy = true;
        sl.model = pick;
        sl.reqs.clear();
        int64_t m = 0;
        while (!sm.queue.empty() && m + sm.queue.front()->B <= opts.max_batch) {
            sl.reqs.push_back(sm.queue.front());
            m += sm.queue.front()->B;
            sm.queue.pop_front();
        }
        sl.count = m;
        sm.running += 1;
        l.unlock();
        // Gather the requests' queries into the slot's pinned buffer.
        const size_t row = (size_t)sm.M->d * sm.esz;
        size_t off = 0;
        for (fmg_request *r : sl.reqs) {
            memcpy((char *)sl.Zh + off, r->Z, (size_t)r->B * row);
            off += (size_t)r->B * row;
        }
        // A graph predicts a whole bucket.  The rows past the batch repeat its
        // last query: left as they were, they would hold an earlier batch's
        // bytes, possibly of another model's dtype (FP64 bytes read as FP32
        // can be NaN or Inf, which fail the certificate and take the exact
        // rescan).  Their results are dropped.
        if (opts.use_graphs && m > 0) {
            const int64_t mb = bucket_of(m, opts.max_batch);
            const char *last = (const char *)sl.Zh + (size_t)(m - 1) * row;
            for (int64_t t = m; t < mb; ++t) memcpy((char *)sl.Zh + (size_t)t * row, last, row);
        }
        sl.launch_status = launch(sl, sm, m);
        l.lock();
        inflight.push_back(free_slot);
        cv_inflight.notify_one();
    }
    dispatch_done = true;
    cv_inflight.notify_all();
}

void fmg_server::complete_loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> l(mu);
    for (;;) {
        if (inflight.empty()) {
            if (dispatch_done) break;
            cv_inflight.wait(l);
            continue;
        }
        const int si = inflight.front();
        Slot &sl = slots[si];
        ServerModel &sm = models[sl.model];
        l.unlock();
        fmg_status st = sl.launch_status;
        if (st == FMG_OK) {
            hipError_t e = hipEventSynchronize(sl.done);
            if (e != hipSuccess) st = FMG_E_DEVICE;
        }
        const size_t row = (size_t)sm.M->ell * sm.esz;
        size_t off = 0;
        if (st == FMG_OK)
            for (fmg_request *r : sl.reqs) {
                memcpy(r->out, (const char *)sl.Oh + off, (size_t)r->B * row);
                off += (size_t)r->B * row;
            }
        const int64_t t = now_ns();
        l.lock();
        for (fmg_request *r : sl.reqs) {
            if (st == FMG_OK) n_q += r->B;
            const Finished fin = finish(r, st, t);  // r is gone after this
            if (fin.whole && fin.status == FMG_OK) {
                lat.push_back(fin.ms);
                n_req += 1;
                if (t_first == 0 || fin.arrival_ns < t_first) t_first = fin.arrival_ns;
                t_last = std::max(t_last, t);
            }
        }
        if (st == FMG_OK) n_batch += 1;
        sl.reqs.clear();
        sl.busy = false;
        sm.running -= 1;
        inflight.pop_front();
        cv_work.notify_one();
        cv_idle.notify_all();
    }
}

// Admit waiting models, first come first, while the budget allows (called
// with the lock held).
void fmg_server::admit_waiting() {
    while (!waiting.empty()) {
        ServerModel &sm = models[waiting.front()];
        if (sm.removed) {
            waiting.pop_front();
            continue;
        }
        if (resident + sm.footprint > budget) break;
        if (model_restore(sm.M, opts.swap_idle != 0) != FMG_OK) break;
        sm.admitted = true;
        sm.admitted_at = now_ns();
        resident += sm.footprint;
        note_resident();
        waiting.pop_front();
        cv_work.notify_one();
    }
}

extern "C" {

fmg_status fastmuygps_server_create(uint64_t hbm_budget, const fmg_server_opts *opts,
                                    fmg_server **out) {
    if (!out) return set_error(FMG_E_INVALID_ARG, "out is null");
    *out = nullptr;
    fmg_server_opts o{3, 16384, 1, 0};
    if (opts) {
        o = *opts;
        if (o.slots == 0) o.slots = 3;
        if (o.max_batch == 0) o.max_batch = 16384;
    }
    if (o.slots < 1 || o.slots > 8) return set_error(FMG_E_INVALID_ARG, "slots = %d", o.slots);
    if (o.max_batch < 1 || o.max_batch > 65536)
        return set_error(FMG_E_INVALID_ARG, "max_batch = %d", o.max_batch);
    fmg_server *S = new fmg_server();
    S->opts = o;
    (void)hipGetDevice(&S->device);
    if (hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        hbm_budget = fr;
    }
    S->budget = hbm_budget;
    const uint64_t per_slot = predict_ws_bytes(o.max_batch) +
                              (uint64_t)o.max_batch * (SLOT_MAX_D + SLOT_MAX_ELL) * 8;
    if (per_slot * o.slots > hbm_budget) {
        delete S;
        return set_error(FMG_E_OOM, "slot workspaces (%llu bytes) exceed the budget",
                         (unsigned long long)(per_slot * o.slots));
    }
    S->slots.resize(o.slots);
    auto fail_create = [&](fmg_status st) {
        fastmuygps_server_destroy(S);
        return st;
    };
    for (Slot &sl : S->slots) {
        const size_t zb = (size_t)o.max_batch * SLOT_MAX_D * 8;
        const size_t ob = (size_t)o.max_batch * SLOT_MAX_ELL * 8;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
            return fail_create(set_error(FMG_E_DEVICE, "stream or event creation failed"));
        if (hipHostMalloc(&sl.Zh, zb, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.Oh, ob, hipHostMallocDefault) != hipSuccess)
            return fail_create(set_error(FMG_E_OOM, "pinned staging buffers"));
        memset(sl.Zh, 0, zb);  // rows past a batch stay finite
        if (hipMalloc(&sl.Zd, zb) != hipSuccess || hipMalloc(&sl.Od, ob) != hipSuccess)
            return fail_create(set_error(FMG_E_OOM, "slot buffers"));
        fmg_status st = predict_ws_alloc(&sl.ws, o.max_batch);
        if (st != FMG_OK) return fail_create(st);
        S->ws_bytes += zb + ob + sl.ws.bytes;
    }
    S->resident = S->ws_bytes;
    S->note_resident();
    S->dispatcher = std::thread([S] { S->dispatch_loop(); });
    S->completer = std::thread([S] { S->complete_loop(); });
    *out = S;
    return FMG_OK;
}

fmg_status fastmuygps_server_add_model(fmg_server *S, fmg_model *M, int32_t *id) {
    if (!S || !M || !id) return set_error(FMG_E_INVALID_ARG, "null argument");
    if (M->timing)
        return set_error(FMG_E_INVALID_ARG, "models built with FMG_FLAG_TIMING cannot be served");
    if (M->d > SLOT_MAX_D || M->ell > SLOT_MAX_ELL)
        return set_error(FMG_E_INVALID_ARG, "d or ell beyond the slot buffers");
    if (!M->resident) return set_error(FMG_E_INVALID_ARG, "the model is offloaded");
    std::unique_lock<std::mutex> l(S->mu);
    for (const ServerModel &o : S->models)
        if (o.M == M && !o.removed) return set_error(FMG_E_INVALID_ARG, "model already added");
    ServerModel sm;
    sm.M = M;
    sm.footprint = M->bytes;
    sm.esz = M->prec == FMG_PREC_FP64 ? 8 : 4;
    if (S->ws_bytes + sm.footprint > S->budget)
        return set_error(FMG_E_OOM, "model of %llu bytes exceeds the budget",
                         (unsigned long long)sm.footprint);
    *id = (int32_t)S->models.size();
    if (S->waiting.empty() && S->resident + sm.footprint <= S->budget) {
        sm.admitted = true;
        sm.admitted_at = now_ns();
        S->resident += sm.footprint;
        S->note_resident();
        S->models.push_back(sm);
        return FMG_OK;
    }
    fmg_status st = model_offload(M);
    if (st != FMG_OK) return st;
    S->models.push_back(sm);
    S->waiting.push_back(*id);
    return set_error(FMG_E_BUSY, "model waits for admission (budget)");
}

fmg_status fastmuygps_server_remove_model(fmg_server *S, int32_t id) {
    if (!S) return set_error(FMG_E_INVALID_ARG, "server is null");
    std::unique_lock<std::mutex> l(S->mu);
    if (id < 0 || id >= (int32_t)S->models.size() || S->models[id].removed)
        return set_error(FMG_E_INVALID_ARG, "unknown model id %d", id);
    {
        ServerModel &sm = S->models[id];
        if (!sm.admitted && !S->opts.swap_idle) {
            // never admitted: fail its queued requests
            const int64_t t = now_ns();
            for (fmg_request *r : sm.queue) finish(r, FMG_E_BUSY, t);
            sm.queue.clear();
        }
    }
    S->cv_idle.wait(l, [&] {
        const ServerModel &sm = S->models[id];
        return sm.queue.empty() && sm.running == 0 && !sm.loading;
    });
    ServerModel &sm = S->models[id];
    sm.removed = true;
    fmg_status st = FMG_OK;
    if (sm.admitted) {
        S->resident -= sm.footprint;
        sm.admitted = false;
    } else {
        st = model_restore(sm.M);  // hand it back resident when memory allows
    }
    S->admit_waiting();
    return st;
}

fmg_status fastmuygps_server_submit(fmg_server *S, int32_t id, const void *Z_host, int32_t B,
                                    void *out_host, int64_t arrival_ns, fmg_ticket *ticket) {
    if (!S || !Z_host || !out_host || !ticket) return set_error(FMG_E_INVALID_ARG, "null argument");
    *ticket = nullptr;
    if (B < 1) return set_error(FMG_E_INVALID_ARG, "B = %d < 1", B);
    const int32_t mb = S->opts.max_batch;
    fmg_request *r = new fmg_request();
    r->model = id;
    r->Z = Z_host;
    r->out = out_host;
    r->B = B;
    r->arrival_ns = arrival_ns > 0 ? arrival_ns : now_ns();
    {
        std::lock_guard<std::mutex> l(S->mu);
        if (id < 0 || id >= (int32_t)S->models.size() || S->models[id].removed || S->stop) {
            delete r;
            return set_error(FMG_E_INVALID_ARG, "unknown model id %d", id);
        }
        ServerModel &sm = S->models[id];
        if (B <= mb) {
            sm.queue.push_back(r);
        } else {
            // parts of at most max_batch queries, queued back to back
            const size_t zrow = (size_t)sm.M->d * sm.esz, orow = (size_t)sm.M->ell * sm.esz;
            r->parts = (B + mb - 1) / mb;
            for (int32_t s0 = 0; s0 < B; s0 += mb) {
                fmg_request *q = new fmg_request();
                q->model = id;
                q->Z = (const char *)Z_host + (size_t)s0 * zrow;
                q->out = (char *)out_host + (size_t)s0 * orow;
                q->B = B - s0 < mb ? B - s0 : mb;
                q->arrival_ns = r->arrival_ns;
                q->parent = r;
                sm.queue.push_back(q);
            }
        }
    }
    S->cv_work.notify_one();
    *ticket = r;
    return FMG_OK;
}

fmg_status fastmuygps_server_wait(fmg_ticket r, double *latency_ms) {
    if (!r) return set_error(FMG_E_INVALID_ARG, "ticket is null");
    fmg_status st;
    {
        std::unique_lock<std::mutex> l(r->mu);
        r->cv.wait(l, [&] { return r->done; });
        st = r->status;
        if (latency_ms) *latency_ms = r->latency_ms;
    }
    delete r;
    if (st != FMG_OK) return set_error(st, "request failed (status %d)", (int)st);
    return FMG_OK;
}

fmg_status fastmuygps_server_stats(fmg_server *S, fmg_server_stats *st) {
    if (!S || !st) return set_error(FMG_E_INVALID_ARG, "null argument");
    std::lock_guard<std::mutex> l(S->mu);
    memset(st, 0, sizeof *st);
    st->requests = S->n_req;
    st->queries = S->n_q;
    st->batches = S->n_batch;
    if (!S->lat.empty()) {
        std::vector<double> v(S->lat);
        std::sort(v.begin(), v.end());
        // nearest-rank percentiles
        auto pct = [&](double p) {
            size_t r = (size_t)std::ceil(p / 100.0 * (double)v.size());
            if (r < 1) r = 1;
            return v[r - 1];
        };
        st->p50_ms = pct(50.0);
        st->p99_ms = pct(99.0);
        double sum = 0.0;
        for (double x : v) sum += x;
        st->mean_ms = sum / (double)v.size();
        st->max_ms = v.back();
    }
    st->wall_s = S->t_last > S->t_first ? (double)(S->t_last - S->t_first) * 1e-9 : 0.0;
    st->queries_per_s = st->wall_s > 0.0 ? (double)S->n_q / st->wall_s : 0.0;
    st->hbm_resident = S->resident;
    st->hbm_peak = S->peak;
    st->swaps = S->n_swaps;
    for (const ServerModel &sm : S->models) {
        if (sm.removed) continue;
        if (sm.admitted) st->models_resident += 1;
        else st->models_waiting += 1;
    }
    return FMG_OK;
}

fmg_status fastmuygps_server_reset_stats(fmg_server *S) {
    if (!S) return set_error(FMG_E_INVALID_ARG, "server is null");
    std::lock_guard<std::mutex> l(S->mu);
    S->lat.clear();
    S->n_req = S->n_q = S->n_batch = S->n_swaps = 0;
    S->t_first = S->t_last = 0;
    return FMG_OK;
}

void fastmuygps_server_destroy(fmg_server *S) {
    if (!S) return;
    {
        std::unique_lock<std::mutex> l(S->mu);
        const int64_t t = now_ns();
        if (!S->opts.swap_idle)
            for (ServerModel &sm : S->models) {
                if (sm.admitted) continue;
                for (fmg_request *r : sm.queue) finish(r, FMG_E_BUSY, t);
                sm.queue.clear();
            }
        // admitted models (and, when swapping, waiting ones): let the loop
        // finish their queues
        S->cv_idle.wait(l, [&] {
            for (const ServerModel &sm : S->models)
                if (!sm.queue.empty() || sm.running > 0 || sm.loading) return false;
            return true;
        });
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->dispatcher.joinable()) S->dispatcher.join();
    if (S->completer.joinable()) S->completer.join();
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        for (auto &kv : sl.graphs) (void)hipGraphExecDestroy(kv.second);
        predict_ws_free(&sl.ws);
        if (sl.Zd) (void)hipFree(sl.Zd);
        if (sl.Od) (void)hipFree(sl.Od);
        if (sl.Zh) (void)hipHostFree(sl.Zh);
        if (sl.Oh) (void)hipHostFree(sl.Oh);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (ServerModel &sm : S->models)
        if (!sm.removed && !sm.M->resident) (void)model_restore(sm.M);
    delete S;
}

}  // extern "C"
