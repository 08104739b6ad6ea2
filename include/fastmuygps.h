/*
 * fastmuygps.h -- C ABI of the MI355X (gfx950) FastMuyGPs posterior-mean library.
 *
 * Method: Dunton, Priest, Muyskens, "Fast Gaussian Process Posterior Mean
 * Prediction via Local Cross Validation and Precomputation", arXiv 2205.10879.
 *   offline (Algorithm 2, training loop; Section 3, coefficient equation):
 *       N(i) = k nearest training points of x_i other than i (leave-one-out),
 *       C[i] = (K(X_N(i), X_N(i)) + sigma^2 I)^{-1} Y(X_N(i));
 *   online (Algorithm 2, prediction loop; Section 3, prediction equation):
 *       j = nearest training point of z,
 *       mu(z) = K(z, X_N(j)) . C[j].
 * Kernels: Matern (Section 2, Matern equation) at nu in {1/2, 3/2, 5/2}, and
 * the RBF limit nu -> infinity.
 *
 * Conventions for every call:
 *   - all arrays are row-major; all sizes are element counts;
 *   - "device pointer" means memory of the current HIP device; "host pointer"
 *     means ordinary process memory;
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream); work is enqueued on it;
 *   - no call throws; every call returns an fmg_status and, on failure,
 *     leaves a message for fastmuygps_last_error() (thread-local);
 *   - indices are int32, so n <= 2^31 - 1;
 *   - device scratch of a call (candidate pools, orders, staging) is kept by
 *     the library when the call ends (up to 16 GiB per device), tagged with
 *     the call's stream and an event recorded there, and reused by a later
 *     call that asks for the same size (at once on the same stream, once the
 *     event has completed on another); a failed allocation returns the
 *     kept blocks to the device and retries;
 *   - the device arrays of a freed model are kept by the library (up to
 *     16 GiB per device) for later builds of the same sizes; an allocation
 *     that fails returns them to the device first, and
 *     fastmuygps_release_cached() returns both caches at once.
 */
#ifndef FASTMUYGPS_H
#define FASTMUYGPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FMG_OK = 0,
    FMG_E_INVALID_ARG = 1, /* bad size, null pointer, unsupported kernel, non-finite input */
    FMG_E_OOM = 2,         /* device allocation failed */
    FMG_E_NOT_PD = 3,      /* build finished but some neighbourhood matrices were not
                              positive definite; their C rows are NaN (count in fmg_info) */
    FMG_E_DEVICE = 4,      /* a HIP runtime call failed */
    FMG_E_BUSY = 5,        /* server admission: request queued, not yet admitted */
    FMG_E_UNSUPPORTED = 6, /* valid request outside what the library implements (e.g. d too
                              large for the chosen precision) */
    FMG_E_IO = 7           /* a model file could not be opened, read or written, or is not
                              a complete model file of this library's format */
} fmg_status;

/* Arithmetic of the path.
 *   FP64 : X, Y, Z, C and means in double; exact FP64 neighbour search;
 *          FP64 assembly and Cholesky.
 *   FP32 : X, Y, Z, C and means in float; FP32 MFMA distance screen over
 *          k + 8 candidates, FP64 re-rank with an exactness certificate
 *          (rows that fail are rescanned in FP64); FP32 assembly and Cholesky.
 *   MIXED: as FP32, but the screen is BF16 MFMA with FP32 accumulation over
 *          2k candidates, and each coefficient row gets one step of iterative
 *          refinement with an FP64 residual.
 * In every mode the neighbour lists equal those of an exact FP64 search
 * (ties to the smaller index). */
typedef enum { FMG_PREC_FP64 = 0, FMG_PREC_FP32 = 1, FMG_PREC_MIXED = 2 } fmg_precision;

typedef enum { FMG_KERNEL_RBF = 0, FMG_KERNEL_MATERN = 1 } fmg_kernel;

/* Hyperparameters (Section 2, Matern equation, with the nugget added by
 * index on the training diagonal only):
 *   K(x, x') = amplitude * phi(||x - x'|| / length_scale),   x != x' by index,
 *   K(x_a, x_a) = amplitude + noise_var.
 * nu is read only for FMG_KERNEL_MATERN and must be 0.5, 1.5 or 2.5.
 * amplitude <= 0 is read as 1. */
typedef struct {
    int32_t kernel;       /* fmg_kernel */
    double nu;
    double length_scale;  /* > 0 */
    double noise_var;     /* >= 0 */
    double amplitude;
} fmg_hyper;

/* Build flags. */
#define FMG_FLAG_SELF_INCLUSIVE 0x1u /* paper-literal S_i = [i ; k-1 nearest others]
                                        (Algorithm 2) instead of leave-one-out */
#define FMG_FLAG_NO_CENTER 0x2u      /* screening uses X as given instead of X - mean(X) */
#define FMG_FLAG_NO_REFINE 0x4u      /* MIXED: skip the FP64-residual refinement */
#define FMG_FLAG_TIMING 0x8u         /* record per-phase HIP-event timings (build and the
                                        most recent predict); makes predict on this
                                        model unsafe to call from several threads */
#define FMG_FLAG_NO_PRUNE 0x10u      /* MIXED: screen every candidate tile in the build
                                        (by default the training points are ordered by
                                        nearest pivot and tiles that no query of a
                                        wavefront can take are skipped; results are
                                        identical either way) */

typedef struct fmg_model fmg_model;

typedef struct {
    int64_t n;
    int32_t d, ell, k;
    int32_t precision;        /* fmg_precision */
    int32_t screen_cands;     /* candidates kept per training row by the screen (c) */
    int32_t query_cands;      /* candidates kept per query by the screen (c') */
    int64_t nonpd_rows;       /* rows whose neighbourhood matrix was not PD */
    int64_t build_fallback_rows; /* training rows rescanned exactly after the certificate */
    int64_t predict_fallback_rows; /* queries rescanned exactly, summed over all predicts
                                      (reading it synchronises the device) */
    uint64_t device_bytes;    /* device memory held by the model */
} fmg_info;

/* Per-phase times in milliseconds from HIP events (FMG_FLAG_TIMING). */
typedef struct {
    double build_prep_ms, build_screen_ms, build_rerank_ms, build_fallback_ms,
        build_precompute_ms, build_total_ms;
    double predict_prep_ms, predict_screen_ms, predict_rerank_ms, predict_fallback_ms,
        predict_gather_ms, predict_total_ms;
} fmg_timings;

/* Offline training: neighbour lists and coefficient rows (Algorithm 2,
 * training loop; Section 3, coefficient equation).
 *   X   : device pointer, [n, d], double for FP64, float otherwise.
 *   Y   : device pointer, [n, ell], same dtype as X.
 *   n   : training points, 2 <= n < 2^31 (LOO needs 1 <= k <= n-1,
 *         SELF needs 1 <= k <= n).
 *   d   : 1 <= d <= 64 (FP32), 61 (MIXED), any (FP64).
 *   ell : responses per point, 1 <= ell <= 16.
 *   k   : neighbours, 1 <= k <= 256.  Up to 64 a wavefront owns one
 *         neighbourhood (one neighbour per lane); wider neighbourhoods take an
 *         exact FP64-distance search for every training point and one
 *         workgroup per factorisation with the packed factor in LDS, so they
 *         need FP64 or FP32 precision and
 *         esz * (k (d+1) + k (k+1)/2 + 513) <= 160 KB (esz = 8 for FP64,
 *         4 for FP32); otherwise FMG_E_UNSUPPORTED.
 * X and Y are only read during the call; the model keeps its own copies of
 * what prediction needs (X, Y, the neighbour lists N [n,k] and C [n,k,ell]).
 * The call returns when the model is complete (it synchronises `stream`).
 * Errors: FMG_E_INVALID_ARG (sizes, null pointers, length_scale <= 0,
 * noise_var < 0, nu not supported, non-finite X or Y), FMG_E_UNSUPPORTED,
 * FMG_E_OOM, FMG_E_DEVICE.  FMG_E_NOT_PD still returns a usable model in
 * *out (the affected C rows are NaN). */
fmg_status fastmuygps_build(const void *X, const void *Y, int64_t n, int32_t d, int32_t ell,
                            int32_t k, const fmg_hyper *hyper, fmg_precision prec,
                            uint32_t flags, void *stream, fmg_model **out);

/* Online prediction (Algorithm 2, prediction loop; Section 3, prediction
 * equation): nearest training point j of every query, then
 * mu(z) = K(z, X_N(j)) . C[j].
 *   Z      : device pointer, [m, d], dtype of the model's X.
 *   out    : device pointer, [m, ell], dtype of the model's X.
 *   nn_out : optional device pointer, [m] int32, receives j (NULL to skip).
 *   m = 0 is a no-op.  Asynchronous on `stream`; scratch memory is
 *   allocated stream-ordered and released on the same stream.  The model is
 *   not modified (unless built with FMG_FLAG_TIMING), so predictions on
 *   several streams may run concurrently.
 * Errors: FMG_E_INVALID_ARG (null model or pointer, m < 0), FMG_E_OOM,
 * FMG_E_DEVICE. */
fmg_status fastmuygps_predict(const fmg_model *model, const void *Z, int64_t m, void *out,
                              int32_t *nn_out, void *stream);

/* Allocation-free prediction, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Computes exactly what fastmuygps_predict computes (same
 * kernels; neighbour index and means bit-identical), but every scratch buffer
 * comes from one static device array that the library holds on each GPU it
 * runs on until the process ends (fastmuygps_noalloc_scratch_bytes(), about
 * 87 MiB); no hipMalloc, hipFree or allocating library routine is called.
 *   Z, out, nn_out : as in fastmuygps_predict (caller-owned device memory).
 *   m              : 0 <= m <= FMG_NOALLOC_MAX_M queries per call (m = 0 is
 *                    a no-op); split larger batches.
 * The model must live on the current device.  The array keeps the last
 * call's contents; every buffer that must start cleared is cleared by a
 * kernel on `stream` (no memset).  All calls on one GPU share its array, so
 * calls that overlap on one GPU (different streams or host threads without
 * ordering between them) race: order them on one stream or synchronise.
 * Errors: FMG_E_INVALID_ARG (null model or pointer, m < 0,
 * m > FMG_NOALLOC_MAX_M, model on another device), FMG_E_BUSY (model
 * offloaded by a server), FMG_E_DEVICE. */
#define FMG_NOALLOC_MAX_M 4096
fmg_status fastmuygps_predict_noalloc(const fmg_model *model, const void *Z, int64_t m,
                                      void *out, int32_t *nn_out, void *stream);
/* Bytes of the static scratch array fastmuygps_predict_noalloc uses on each
 * device. */
uint64_t fastmuygps_noalloc_scratch_bytes(void);

/* MuyGPs prediction of novel points (Section 2.1, MuyGPs prediction
 * equation): the per-query method whose training-data part FastMuyGPs
 * precomputes.  For every query z:
 *   N*(z) = the k nearest training points of z (exact, ties to the smaller
 *           index; the screen, re-rank and certificate of the build, with
 *           the build's candidate count; for k > 64 and in FP64 the exact
 *           FP64-distance search),
 *   mu(z) = K(z, X_N*) (K(X_N*, X_N*) + sigma^2 I)^{-1} Y(X_N*),
 * with the model's k, kernel, hyperparameters and precision (a k x k solve
 * per query, refined in MIXED as in the build).
 *   Z       : device pointer [m, d], dtype of the model's X.
 *   out     : device pointer [m, ell], dtype of the model's X.
 *   nbr_out : optional device pointer [m, k] int32, receives N*(z) (NULL to
 *             skip).
 * Asynchronous on `stream`; scratch is stream-ordered.  A query whose
 * neighbourhood matrix is not positive definite gets NaN means.
 * Errors: FMG_E_INVALID_ARG (null model or pointer, m < 0), FMG_E_BUSY
 * (model offloaded by a server), FMG_E_OOM, FMG_E_DEVICE. */
fmg_status fastmuygps_predict_muygps(const fmg_model *model, const void *Z, int64_t m, void *out,
                                     int32_t *nbr_out, void *stream);

/* Leave-one-out predictions of training points (Section 2.1: the MuyGPs
 * prediction of x_i from its neighbours X_N(i), whose squared errors the
 * MuyGPs loss Q(theta) averages over a batch): with the model's neighbour
 * lists and coefficients this is K(x_i, X_N(i)) . C[i] (Section 3,
 * coefficient equation), no solve needed.  In self-inclusive models
 * (FMG_FLAG_SELF_INCLUSIVE) the set S_i contains i itself.
 *   rows : device pointer [b] int32 of training-point indices; an index
 *          outside [0, n) yields NaN for that row.
 *   out  : device pointer [b, ell], dtype of the model's X.
 * Asynchronous on `stream`.  Errors: FMG_E_INVALID_ARG, FMG_E_BUSY,
 * FMG_E_DEVICE. */
fmg_status fastmuygps_loo_predict(const fmg_model *model, const int32_t *rows, int64_t b,
                                  void *out, void *stream);

/* Loss of MuyGPs hyperparameter training (Algorithm 1; Section 2.1, loss
 * Q(theta)): the mean over a batch B of training rows, and over the ell
 * responses, of (Y(x_i) - Yhat_theta(x_i | X_N(i)))^2, where the
 * leave-one-out prediction uses the model's neighbour lists (they do not
 * depend on theta: the kernels are isotropic) and coefficient rows solved
 * again under `hyper`, in the model's precision.  An optimiser over theta
 * (e.g. L-BFGS-B on the host) calls this once per candidate theta.
 *   rows : device pointer [b] int32, b >= 1, training-point indices.
 *   loss : host pointer, receives Q(theta); NaN when a batch row's
 *          neighbourhood matrix is not positive definite under theta.
 * Synchronises `stream`.  Errors: FMG_E_INVALID_ARG (null pointers, b < 1,
 * a row outside [0, n), invalid hyperparameters, a self-inclusive model),
 * FMG_E_BUSY, FMG_E_OOM, FMG_E_DEVICE. */
fmg_status fastmuygps_loo_loss(const fmg_model *model, const int32_t *rows, int64_t b,
                               const fmg_hyper *hyper, double *loss, void *stream);

/* Loss of MuyGPs hyperparameter training and its gradient (Algorithm 1;
 * Section 2.1, loss Q(theta)), for a gradient-based optimiser over theta
 * (e.g. L-BFGS-B on the host).  Q is the mean over the batch rows and the
 * ell responses of the squared leave-one-out error, with the model's
 * neighbour lists (independent of theta) and the local systems solved again
 * under `hyper`; the gradient is exact (differentiated through the solve,
 * dK^{-1} = -K^{-1} dK K^{-1}).  Everything runs in FP64 whatever the model
 * precision (FP32 inputs widened exactly), so for FP32 and MIXED models the
 * loss can differ from fastmuygps_loo_loss by that path's rounding.
 *   rows : device pointer [b] int32, b >= 1, training-point indices.
 *   loss : host pointer, receives Q(theta).
 *   grad : host pointer [2], receives dQ/d length_scale and dQ/d noise_var
 *          (amplitude and kernel are held fixed).
 * Loss and gradient are NaN when a batch row's matrix is not positive
 * definite under theta.  Synchronises `stream`.  Errors: FMG_E_INVALID_ARG
 * (null pointers, b < 1, a row outside [0, n), invalid hyperparameters, a
 * self-inclusive model), FMG_E_UNSUPPORTED (k > 64, or (k+1)(d+1) +
 * k(k+1)/2 + 128 doubles exceed 64 KB), FMG_E_BUSY, FMG_E_OOM,
 * FMG_E_DEVICE. */
fmg_status fastmuygps_loo_loss_grad(const fmg_model *model, const int32_t *rows, int64_t b,
                                    const fmg_hyper *hyper, double *loss, double *grad,
                                    void *stream);

/* Model metadata (host struct).  Synchronises the device. */
fmg_status fastmuygps_info(const fmg_model *model, fmg_info *info);

/* Copy the neighbour lists N [n, k] int32 (ascending distance) into the
 * caller's device buffer. */
fmg_status fastmuygps_neighbors(const fmg_model *model, int32_t *dev_out, void *stream);

/* Copy the coefficients C [n, k, ell] (model dtype) into the caller's
 * device buffer. */
fmg_status fastmuygps_coeffs(const fmg_model *model, void *dev_out, void *stream);

/* HIP-event phase timings of the build and of the latest predict
 * (FMG_FLAG_TIMING models only; FMG_E_INVALID_ARG otherwise). */
fmg_status fastmuygps_timings(const fmg_model *model, fmg_timings *t);

/* ------------------------------------------------------------------------
 * Serving: resident models and continuous batching of query requests.
 *
 * The paper motivates prediction inside online loops (Section 1) but gives no
 * serving design; this is the library's.  A server keeps built models on the
 * device within an HBM budget and runs a request loop: requests (host query
 * buffers of uneven size) are queued per model; whenever one of `slots`
 * in-flight slots is free, all queued requests of one model, up to
 * `max_batch` queries, are coalesced into one batch, copied to the device and
 * predicted there (Algorithm 2, prediction loop) on that slot's stream, while
 * other slots' batches run.  Every slot owns its buffers (allocated at
 * creation), so a batch allocates nothing; with `use_graphs` the copy-in,
 * prediction and copy-out of a batch replay a HIP graph captured once per
 * (model, slot, batch-size bucket).  Each result is the one
 * fastmuygps_predict returns for the same query alone.
 * ------------------------------------------------------------------------ */
typedef struct fmg_server fmg_server;
typedef struct fmg_request *fmg_ticket;

typedef struct {
    int32_t slots;      /* batches in flight (one stream each), 1..8; 0 = 3 */
    int32_t max_batch;  /* queries per batch and per request, 1..65536; 0 = 16384 */
    int32_t use_graphs; /* replay captured HIP graphs per batch (1) or launch (0) */
    int32_t swap_idle;  /* 1: a waiting model with queued requests is swapped in for idle
                           resident models (no queued or running batch, resident at least
                           50 ms), least recently used first; 0: it waits for removals */
} fmg_server_opts;

typedef struct {
    int64_t requests, queries, batches; /* completed since creation or reset */
    double p50_ms, p99_ms, mean_ms, max_ms; /* request latency: arrival to results
                                               in the caller's host buffer */
    double wall_s;          /* first arrival to last completion */
    double queries_per_s;   /* queries / wall_s */
    uint64_t hbm_resident;  /* bytes: admitted models + slot workspaces */
    uint64_t hbm_peak;
    int32_t models_resident, models_waiting;
    int64_t swaps;          /* models swapped in by the swap_idle policy */
} fmg_server_stats;

/* Create a server on the current device.  hbm_budget (bytes) bounds the
 * admitted models plus the slot workspaces; 0 means the device's free memory.
 * opts may be NULL (defaults).  Errors: FMG_E_INVALID_ARG, FMG_E_OOM (the
 * slot workspaces alone exceed the budget), FMG_E_DEVICE. */
fmg_status fastmuygps_server_create(uint64_t hbm_budget, const fmg_server_opts *opts,
                                    fmg_server **out);

/* Register a built model (the caller keeps ownership and frees it after
 * removing it or destroying the server).  FMG_OK: admitted, resident.
 * FMG_E_BUSY: over budget now -- the model's arrays are moved to pinned host
 * memory and it is admitted (moved back) when a removal frees enough budget,
 * or, with swap_idle, when requests for it arrive and idle resident models
 * can make room (they move to host memory in turn and wait);
 * *id is valid and requests may be submitted meanwhile (they wait).
 * FMG_E_OOM: the model alone exceeds the budget.  FMG_E_INVALID_ARG: null
 * arguments, a model built with FMG_FLAG_TIMING, or d/ell beyond the slots. */
fmg_status fastmuygps_server_add_model(fmg_server *server, fmg_model *model, int32_t *id);

/* Unregister a model once its queued and running requests are done; its
 * budget goes to waiting models (first come, first admitted).  The model is
 * left resident on the device for the caller when memory allows.  */
fmg_status fastmuygps_server_remove_model(fmg_server *server, int32_t id);

/* Queue B queries for model `id`.  Z_host: host pointer [B, d] in the
 * model's dtype; out_host: host pointer [B, ell] in the model's dtype; both
 * stay owned by the caller and must stay valid until fastmuygps_server_wait
 * returns for this ticket.  arrival_ns: the request's scheduled arrival on
 * CLOCK_MONOTONIC in nanoseconds (latency is measured from it), 0 = now.
 * A request of more than max_batch queries is queued as consecutive parts of
 * at most max_batch queries (each batched like any request); its ticket
 * completes with the last part, its latency runs to then, and it counts as
 * one request in the statistics.  Returns at once.  Errors:
 * FMG_E_INVALID_ARG (unknown id, B < 1, null pointers). */
fmg_status fastmuygps_server_submit(fmg_server *server, int32_t id, const void *Z_host,
                                    int32_t B, void *out_host, int64_t arrival_ns,
                                    fmg_ticket *ticket);

/* Block until the request is done; releases the ticket.  latency_ms may be
 * NULL.  Returns the request's status. */
fmg_status fastmuygps_server_wait(fmg_ticket ticket, double *latency_ms);

/* Latency and throughput statistics (host struct). */
fmg_status fastmuygps_server_stats(fmg_server *server, fmg_server_stats *stats);

/* Clear the statistics (not the HBM peak). */
fmg_status fastmuygps_server_reset_stats(fmg_server *server);

/* Finish every queued request of admitted models, fail those of models never
 * admitted (FMG_E_BUSY), stop the request loop and free the slots.  Models
 * stay owned by the caller and are moved back to the device when memory
 * allows.  NULL is a no-op.  Outstanding tickets stay valid until waited on. */
void fastmuygps_server_destroy(fmg_server *server);

/* Release the model and all its device memory.  NULL is a no-op. */
void fastmuygps_free(fmg_model *model);

/* Checkpoint of a built model (the output of Algorithm 2's training loop:
 * neighbour lists and coefficient rows, with the training rows, responses
 * and screening structures that prediction reads).
 * fastmuygps_save writes the model to the file `path` (created or
 * truncated), after synchronising the device: an 8-byte tag "FMGMODEL", a
 * format number (1), the model's parameters at their native widths and byte
 * order, then its arrays.  The model is unchanged.
 * fastmuygps_load reads such a file onto the current device and returns a
 * new model in *out (owned by the caller, released with fastmuygps_free),
 * whose predictions are bitwise identical to those of the saved model; its
 * prediction fallback count starts at 0.  The file is read with the byte
 * order of the machine that wrote it.
 * Errors: FMG_E_INVALID_ARG (null pointers), FMG_E_IO (the file cannot be
 * opened, read or written; a wrong tag or format; a malformed header; a
 * truncated file or bytes past its end), FMG_E_OOM, FMG_E_DEVICE. */
fmg_status fastmuygps_save(const fmg_model *model, const char *path);
fmg_status fastmuygps_load(const char *path, fmg_model **out);

/* Message of the last failed call on this thread ("" if none).  The string
 * is owned by the library and valid until the next call on this thread. */
const char *fastmuygps_last_error(void);

/* Library version string, e.g. "fastmuygps-gfx950 0.1". */
const char *fastmuygps_version(void);

/* Diagnostic, for tests of the arithmetic: y[i] = exp(x[i]) for x[i] <= 0,
 * evaluated on the device by the FP64 exponential that the MIXED
 * refinement's residual uses for kernel values (additive range reduction
 * x = n ln2 + r with ln2 in two parts (Cody and Waite), the Taylor series of
 * exp(r) to degree 12, scaling by 2^n; it underflows to 0 below about -745).
 * x and y are device pointers [n].  Asynchronous on `stream`.  Errors:
 * FMG_E_INVALID_ARG (n < 0, null pointers), FMG_E_DEVICE. */
fmg_status fastmuygps_debug_exp_nonpos(const double *x, double *y, int64_t n, void *stream);

/* Diagnostic, for tests of the arithmetic: y[i] = exp(x[i]) for x[i] <= 0,
 * evaluated on the device by the FP32 exponential of the FP32 kernel values
 * (x log2(e) = n + f carried in two parts, 2^f from the hardware base-2
 * exponential, scaling by 2^n).  Results that are normal floats are within
 * about two units in the last place; below the smallest normal float they
 * are within that float of exp(x).  x and y are device pointers [n].
 * Asynchronous on `stream`.  Errors: FMG_E_INVALID_ARG (n < 0, null
 * pointers), FMG_E_DEVICE. */
fmg_status fastmuygps_debug_exp_nonpos32(const float *x, float *y, int64_t n, void *stream);

/* Return the device memory the library keeps cached on the current device
 * (the arrays of freed models and the freed scratch of earlier calls) to the
 * device.  Synchronises the device first; no call may be running on it.
 * Later calls allocate afresh.  FMG_E_DEVICE on a HIP error. */
fmg_status fastmuygps_release_cached(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTMUYGPS_H */
