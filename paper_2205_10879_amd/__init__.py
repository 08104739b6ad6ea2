"""FastMuyGPs posterior-mean path for MI355X (gfx950): Python binding.

Thin ctypes marshalling over the C ABI in include/fastmuygps.h (same names:
``fastmuygps_build``, ``fastmuygps_predict``, ...).  Every step of the path
runs in the HIP library ``libfastmuygps.so``; torch is used only for device
memory and streams.  The first call raises when the library has not been
built (``python -m paper_2205_10879_amd.build``); there is no fallback.

Method: Dunton, Priest, Muyskens, arXiv 2205.10879, Algorithm 2.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfastmuygps.so")

FMG_OK = 0
FMG_E_INVALID_ARG = 1
FMG_E_OOM = 2
FMG_E_NOT_PD = 3
FMG_E_DEVICE = 4
FMG_E_BUSY = 5
FMG_E_UNSUPPORTED = 6
FMG_E_IO = 7

PREC_FP64 = 0
PREC_FP32 = 1
PREC_MIXED = 2
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "mixed": PREC_MIXED}

KERNEL_RBF = 0
KERNEL_MATERN = 1

FLAG_SELF_INCLUSIVE = 0x1
FLAG_NO_CENTER = 0x2
FLAG_NO_REFINE = 0x4
FLAG_TIMING = 0x8
FLAG_NO_PRUNE = 0x10

# Public C entry points (checked by the CPU tests against include/fastmuygps.h).
EXPORTS = ("fastmuygps_build", "fastmuygps_predict", "fastmuygps_info", "fastmuygps_neighbors",
           "fastmuygps_coeffs", "fastmuygps_timings", "fastmuygps_free", "fastmuygps_last_error",
           "fastmuygps_version", "fastmuygps_predict_muygps", "fastmuygps_loo_predict",
           "fastmuygps_loo_loss", "fastmuygps_loo_loss_grad",
           "fastmuygps_server_create", "fastmuygps_server_add_model",
           "fastmuygps_server_remove_model", "fastmuygps_server_submit", "fastmuygps_server_wait",
           "fastmuygps_server_stats", "fastmuygps_server_reset_stats",
           "fastmuygps_server_destroy", "fastmuygps_release_cached",
           "fastmuygps_predict_noalloc", "fastmuygps_noalloc_scratch_bytes",
           "fastmuygps_debug_exp_nonpos", "fastmuygps_debug_exp_nonpos32",
           "fastmuygps_save", "fastmuygps_load")

# Largest batch of one fastmuygps_predict_noalloc call (FMG_NOALLOC_MAX_M).
NOALLOC_MAX_M = 4096


class FmgHyper(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("nu", ctypes.c_double),
                ("length_scale", ctypes.c_double), ("noise_var", ctypes.c_double),
                ("amplitude", ctypes.c_double)]


class FmgInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("ell", ctypes.c_int32),
                ("k", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("screen_cands", ctypes.c_int32), ("query_cands", ctypes.c_int32),
                ("nonpd_rows", ctypes.c_int64), ("build_fallback_rows", ctypes.c_int64),
                ("predict_fallback_rows", ctypes.c_int64), ("device_bytes", ctypes.c_uint64)]


class FmgTimings(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in (
        "build_prep_ms", "build_screen_ms", "build_rerank_ms", "build_fallback_ms",
        "build_precompute_ms", "build_total_ms", "predict_prep_ms", "predict_screen_ms",
        "predict_rerank_ms", "predict_fallback_ms", "predict_gather_ms", "predict_total_ms")]


class FmgServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("swap_idle", ctypes.c_int32)]


class FmgServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("wall_s", ctypes.c_double),
                ("queries_per_s", ctypes.c_double), ("hbm_resident", ctypes.c_uint64),
                ("hbm_peak", ctypes.c_uint64), ("models_resident", ctypes.c_int32),
                ("models_waiting", ctypes.c_int32), ("swaps", ctypes.c_int64)]


class FmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("fastmuygps status %d: %s" % (status, message))
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError("FastMuyGPs HIP library not built: %s is missing "
                          "(run `python -m paper_2205_10879_amd.build`)" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.fastmuygps_build.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.POINTER(FmgHyper), ctypes.c_int,
                                     ctypes.c_uint32, P, ctypes.POINTER(P)]
    lib.fastmuygps_build.restype = ctypes.c_int
    lib.fastmuygps_predict.argtypes = [P, P, ctypes.c_int64, P, P, P]
    lib.fastmuygps_predict.restype = ctypes.c_int
    lib.fastmuygps_debug_exp_nonpos.argtypes = [P, P, ctypes.c_int64, P]
    lib.fastmuygps_debug_exp_nonpos.restype = ctypes.c_int
    lib.fastmuygps_debug_exp_nonpos32.argtypes = [P, P, ctypes.c_int64, P]
    lib.fastmuygps_debug_exp_nonpos32.restype = ctypes.c_int
    lib.fastmuygps_save.argtypes = [P, ctypes.c_char_p]
    lib.fastmuygps_save.restype = ctypes.c_int
    lib.fastmuygps_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]
    lib.fastmuygps_load.restype = ctypes.c_int
    lib.fastmuygps_predict_noalloc.argtypes = [P, P, ctypes.c_int64, P, P, P]
    lib.fastmuygps_predict_noalloc.restype = ctypes.c_int
    lib.fastmuygps_noalloc_scratch_bytes.argtypes = []
    lib.fastmuygps_noalloc_scratch_bytes.restype = ctypes.c_uint64
    lib.fastmuygps_predict_muygps.argtypes = [P, P, ctypes.c_int64, P, P, P]
    lib.fastmuygps_predict_muygps.restype = ctypes.c_int
    lib.fastmuygps_loo_predict.argtypes = [P, P, ctypes.c_int64, P, P]
    lib.fastmuygps_loo_predict.restype = ctypes.c_int
    lib.fastmuygps_loo_loss.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(FmgHyper),
                                        ctypes.POINTER(ctypes.c_double), P]
    lib.fastmuygps_loo_loss.restype = ctypes.c_int
    lib.fastmuygps_loo_loss_grad.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(FmgHyper),
                                             ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double), P]
    lib.fastmuygps_loo_loss_grad.restype = ctypes.c_int
    lib.fastmuygps_info.argtypes = [P, ctypes.POINTER(FmgInfo)]
    lib.fastmuygps_info.restype = ctypes.c_int
    lib.fastmuygps_neighbors.argtypes = [P, P, P]
    lib.fastmuygps_neighbors.restype = ctypes.c_int
    lib.fastmuygps_coeffs.argtypes = [P, P, P]
    lib.fastmuygps_coeffs.restype = ctypes.c_int
    lib.fastmuygps_timings.argtypes = [P, ctypes.POINTER(FmgTimings)]
    lib.fastmuygps_timings.restype = ctypes.c_int
    lib.fastmuygps_free.argtypes = [P]
    lib.fastmuygps_free.restype = None
    lib.fastmuygps_last_error.argtypes = []
    lib.fastmuygps_last_error.restype = ctypes.c_char_p
    lib.fastmuygps_version.argtypes = []
    lib.fastmuygps_version.restype = ctypes.c_char_p
    lib.fastmuygps_release_cached.argtypes = []
    lib.fastmuygps_release_cached.restype = ctypes.c_int
    lib.fastmuygps_server_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(FmgServerOpts),
                                             ctypes.POINTER(P)]
    lib.fastmuygps_server_create.restype = ctypes.c_int
    lib.fastmuygps_server_add_model.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32)]
    lib.fastmuygps_server_add_model.restype = ctypes.c_int
    lib.fastmuygps_server_remove_model.argtypes = [P, ctypes.c_int32]
    lib.fastmuygps_server_remove_model.restype = ctypes.c_int
    lib.fastmuygps_server_submit.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, P,
                                             ctypes.c_int64, ctypes.POINTER(P)]
    lib.fastmuygps_server_submit.restype = ctypes.c_int
    lib.fastmuygps_server_wait.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.fastmuygps_server_wait.restype = ctypes.c_int
    lib.fastmuygps_server_stats.argtypes = [P, ctypes.POINTER(FmgServerStats)]
    lib.fastmuygps_server_stats.restype = ctypes.c_int
    lib.fastmuygps_server_reset_stats.argtypes = [P]
    lib.fastmuygps_server_reset_stats.restype = ctypes.c_int
    lib.fastmuygps_server_destroy.argtypes = [P]
    lib.fastmuygps_server_destroy.restype = None
    return lib


_lib_handle = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library (loaded on first use)."""
    global _lib_handle
    if _lib_handle is None:
        _lib_handle = load_library()
    return _lib_handle


def _check(status: int, allow=()):
    if status != FMG_OK and status not in allow:
        raise FmgError(status, lib().fastmuygps_last_error().decode())
    return status


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype, name: str) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def version() -> str:
    return lib().fastmuygps_version().decode()


def release_cached() -> None:
    """Return the device memory cached by the library (freed models' arrays,
    freed scratch) on the current device."""
    _check(lib().fastmuygps_release_cached())


class Model:
    """A built FastMuyGPs model (owns its device memory in the HIP library)."""

    def __init__(self, handle: ctypes.c_void_p, dtype, d: int, ell: int, k: int, n: int,
                 status: int):
        self._h = handle
        self.dtype = dtype
        self.d, self.ell, self.k, self.n = d, ell, k, n
        self.build_status = status

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise ValueError("model has been freed")
        return self._h

    def predict(self, Z: torch.Tensor, out: torch.Tensor | None = None,
                nn_out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """fastmuygps_predict: means [m, ell] for the queries Z [m, d]."""
        if Z.dim() != 2 or Z.shape[1] != self.d:
            raise ValueError("Z must be [m, %d]" % self.d)
        m = Z.shape[0]
        if out is None:
            out = torch.empty((m, self.ell), dtype=self.dtype, device=Z.device)
        nn_ptr = None
        if nn_out is not None:
            nn_ptr = _dev_ptr(nn_out, torch.int32, "nn_out")
        _check(lib().fastmuygps_predict(self.handle, _dev_ptr(Z, self.dtype, "Z"), m,
                                       _dev_ptr(out, self.dtype, "out"), nn_ptr,
                                       _stream_handle(stream)))
        return out

    def predict_noalloc(self, Z: torch.Tensor, out: torch.Tensor, nn_out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
        """fastmuygps_predict_noalloc: the prediction of `predict` with no
        device allocation (scratch in the library's static per-device array);
        at most NOALLOC_MAX_M queries per call, `out` supplied by the caller."""
        if Z.dim() != 2 or Z.shape[1] != self.d:
            raise ValueError("Z must be [m, %d]" % self.d)
        if out.dim() != 2 or out.shape[0] != Z.shape[0] or out.shape[1] != self.ell:
            raise ValueError("out must be [m, %d]" % self.ell)
        nn_ptr = None
        if nn_out is not None:
            nn_ptr = _dev_ptr(nn_out, torch.int32, "nn_out")
        _check(lib().fastmuygps_predict_noalloc(self.handle, _dev_ptr(Z, self.dtype, "Z"),
                                               Z.shape[0], _dev_ptr(out, self.dtype, "out"),
                                               nn_ptr, _stream_handle(stream)))
        return out

    def predict_muygps(self, Z: torch.Tensor, out: torch.Tensor | None = None,
                       nbr_out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """fastmuygps_predict_muygps: MuyGPs means [m, ell] (Section 2.1), each query
        solving over its own k nearest training points."""
        if Z.dim() != 2 or Z.shape[1] != self.d:
            raise ValueError("Z must be [m, %d]" % self.d)
        m = Z.shape[0]
        if out is None:
            out = torch.empty((m, self.ell), dtype=self.dtype, device=Z.device)
        nb_ptr = None
        if nbr_out is not None:
            if tuple(nbr_out.shape) != (m, self.k):
                raise ValueError("nbr_out must be [m, %d]" % self.k)
            nb_ptr = _dev_ptr(nbr_out, torch.int32, "nbr_out")
        _check(lib().fastmuygps_predict_muygps(self.handle, _dev_ptr(Z, self.dtype, "Z"), m,
                                              _dev_ptr(out, self.dtype, "out"), nb_ptr,
                                              _stream_handle(stream)))
        return out

    def loo_predict(self, rows: torch.Tensor, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
        """fastmuygps_loo_predict: leave-one-out predictions [b, ell] of training rows."""
        if rows.dim() != 1:
            raise ValueError("rows must be a 1-D int32 tensor")
        b = rows.shape[0]
        if out is None:
            out = torch.empty((b, self.ell), dtype=self.dtype, device=rows.device)
        _check(lib().fastmuygps_loo_predict(self.handle, _dev_ptr(rows, torch.int32, "rows"), b,
                                           _dev_ptr(out, self.dtype, "out"),
                                           _stream_handle(stream)))
        return out

    def loo_loss(self, rows: torch.Tensor, kernel: str = "matern", nu: float = 1.5,
                 length_scale: float = 1.0, noise_var: float = 0.0, amplitude: float = 1.0,
                 stream=None) -> float:
        """fastmuygps_loo_loss: MuyGPs loss Q(theta) over the training rows `rows`
        with the hyperparameters given here (Algorithm 1)."""
        if rows.dim() != 1:
            raise ValueError("rows must be a 1-D int32 tensor")
        if kernel not in ("rbf", "matern"):
            raise ValueError("kernel must be 'rbf' or 'matern'")
        hyper = FmgHyper(KERNEL_RBF if kernel == "rbf" else KERNEL_MATERN, float(nu),
                         float(length_scale), float(noise_var), float(amplitude))
        val = ctypes.c_double()
        _check(lib().fastmuygps_loo_loss(self.handle, _dev_ptr(rows, torch.int32, "rows"),
                                        rows.shape[0], ctypes.byref(hyper), ctypes.byref(val),
                                        _stream_handle(stream)))
        return val.value

    def loo_loss_grad(self, rows: torch.Tensor, kernel: str = "matern", nu: float = 1.5,
                      length_scale: float = 1.0, noise_var: float = 0.0,
                      amplitude: float = 1.0, stream=None):
        """fastmuygps_loo_loss_grad: Q(theta) over the training rows `rows` and its
        gradient (dQ/d length_scale, dQ/d noise_var), in FP64 (Algorithm 1).
        Returns (loss, numpy array [2])."""
        if rows.dim() != 1:
            raise ValueError("rows must be a 1-D int32 tensor")
        if kernel not in ("rbf", "matern"):
            raise ValueError("kernel must be 'rbf' or 'matern'")
        hyper = FmgHyper(KERNEL_RBF if kernel == "rbf" else KERNEL_MATERN, float(nu),
                         float(length_scale), float(noise_var), float(amplitude))
        val = ctypes.c_double()
        grad = (ctypes.c_double * 2)()
        _check(lib().fastmuygps_loo_loss_grad(self.handle, _dev_ptr(rows, torch.int32, "rows"),
                                             rows.shape[0], ctypes.byref(hyper),
                                             ctypes.byref(val), grad, _stream_handle(stream)))
        import numpy as np
        return val.value, np.array([grad[0], grad[1]])

    def fit_hyper(self, rows: torch.Tensor, kernel: str = "matern", nu: float = 1.5,
                  length_scale: float = 1.0, noise_var: float = 1e-2,
                  fit_noise: bool = True, length_scale_bounds=(1e-3, 1e3),
                  noise_bounds=(1e-8, 10.0), maxiter: int = 100) -> dict:
        """MuyGPs hyperparameter training (Algorithm 1): minimise Q(theta) over
        the batch `rows` with L-BFGS-B on the host, in log(length_scale) and
        log(noise_var), each step one fastmuygps_loo_loss_grad on the device.
        Returns the fitted values, the final loss and gradient, and the
        optimiser's counts.  The model's own coefficients are not changed."""
        import numpy as np
        from scipy.optimize import minimize

        def objective(u):
            rho = float(np.exp(u[0]))
            s2 = float(np.exp(u[1])) if fit_noise else float(noise_var)
            q, g = self.loo_loss_grad(rows, kernel, nu, rho, s2)
            if not np.isfinite(q) or not np.all(np.isfinite(g)):
                return 1e300, np.zeros_like(u)  # not positive definite here: back off
            gu = [g[0] * rho] + ([g[1] * s2] if fit_noise else [])
            return q, np.array(gu)

        u0 = [np.log(length_scale)] + ([np.log(noise_var)] if fit_noise else [])
        bounds = [tuple(np.log(length_scale_bounds))]
        if fit_noise:
            bounds.append(tuple(np.log(noise_bounds)))
        res = minimize(objective, np.array(u0, dtype=np.float64), jac=True, method="L-BFGS-B",
                       bounds=bounds, options={"maxiter": int(maxiter)})
        rho = float(np.exp(res.x[0]))
        s2 = float(np.exp(res.x[1])) if fit_noise else float(noise_var)
        q, g = self.loo_loss_grad(rows, kernel, nu, rho, s2)
        return {"length_scale": rho, "noise_var": s2, "loss": q, "grad": g,
                "iterations": int(res.nit), "evaluations": int(res.nfev),
                "success": bool(res.success), "message": str(res.message)}

    def info(self) -> dict:
        inf = FmgInfo()
        _check(lib().fastmuygps_info(self.handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in FmgInfo._fields_}

    def save(self, path: str) -> None:
        """fastmuygps_save: write the model to a file (synchronises the device)."""
        _check(lib().fastmuygps_save(self.handle, os.fsencode(path)))

    def neighbors(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.n, self.k), dtype=torch.int32, device="cuda")
        _check(lib().fastmuygps_neighbors(self.handle, ctypes.c_void_p(out.data_ptr()),
                                         _stream_handle(stream)))
        return out

    def coeffs(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.n, self.k, self.ell), dtype=self.dtype, device="cuda")
        _check(lib().fastmuygps_coeffs(self.handle, ctypes.c_void_p(out.data_ptr()),
                                      _stream_handle(stream)))
        return out

    def timings(self) -> dict:
        t = FmgTimings()
        _check(lib().fastmuygps_timings(self.handle, ctypes.byref(t)))
        return {name: getattr(t, name) for name, _ in FmgTimings._fields_}

    def free(self):
        if self._h:
            lib().fastmuygps_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fastmuygps_build(X: torch.Tensor, Y: torch.Tensor, k: int, kernel: str = "matern",
                     nu: float = 1.5, length_scale: float = 1.0, noise_var: float = 0.0,
                     amplitude: float = 1.0, precision: str = "fp32", flags: int = 0,
                     stream=None, allow_not_pd: bool = False) -> Model:
    """fastmuygps_build(X, y, k, kernel, hyperparams) -> model (Algorithm 2, training)."""
    prec = PRECISIONS[precision]
    dtype = torch.float64 if prec == PREC_FP64 else torch.float32
    if X.dim() != 2:
        raise ValueError("X must be [n, d]")
    if Y.dim() == 1:
        Y = Y[:, None]
    n, d = X.shape
    if Y.shape[0] != n:
        raise ValueError("Y must have n rows")
    ell = Y.shape[1]
    hyper = FmgHyper(KERNEL_RBF if kernel == "rbf" else KERNEL_MATERN, float(nu),
                     float(length_scale), float(noise_var), float(amplitude))
    if kernel not in ("rbf", "matern"):
        raise ValueError("kernel must be 'rbf' or 'matern'")
    h = ctypes.c_void_p()
    st = lib().fastmuygps_build(_dev_ptr(X, dtype, "X"), _dev_ptr(Y.contiguous(), dtype, "Y"), n,
                               d, ell, int(k), ctypes.byref(hyper), prec, int(flags),
                               _stream_handle(stream), ctypes.byref(h))
    _check(st, allow=(FMG_E_NOT_PD,) if allow_not_pd else ())
    return Model(h, dtype, d, ell, int(k), n, st)


def fastmuygps_load(path: str) -> Model:
    """fastmuygps_load: a model saved by Model.save, on the current device."""
    h = ctypes.c_void_p()
    _check(lib().fastmuygps_load(os.fsencode(path), ctypes.byref(h)))
    inf = FmgInfo()
    st = lib().fastmuygps_info(h, ctypes.byref(inf))
    if st != FMG_OK:
        lib().fastmuygps_free(h)
        _check(st)
    dtype = torch.float64 if inf.precision == PREC_FP64 else torch.float32
    return Model(h, dtype, inf.d, inf.ell, inf.k, inf.n,
                 FMG_E_NOT_PD if inf.nonpd_rows > 0 else FMG_OK)


def fastmuygps_predict(model: Model, Z: torch.Tensor, out=None, nn_out=None, stream=None):
    """fastmuygps_predict(model, Z) -> means (Algorithm 2, prediction)."""
    return model.predict(Z, out=out, nn_out=nn_out, stream=stream)


def fastmuygps_predict_noalloc(model: Model, Z: torch.Tensor, out, nn_out=None, stream=None):
    """fastmuygps_predict_noalloc(model, Z, out): prediction without device
    allocation, at most NOALLOC_MAX_M queries."""
    return model.predict_noalloc(Z, out, nn_out=nn_out, stream=stream)


def noalloc_scratch_bytes() -> int:
    """Bytes of the static device array the allocation-free prediction uses."""
    return int(lib().fastmuygps_noalloc_scratch_bytes())


def fastmuygps_info(model: Model) -> dict:
    return model.info()


def fastmuygps_free(model: Model) -> None:
    model.free()



class Ticket:
    """A submitted request; ``wait()`` returns (means, latency_ms)."""

    def __init__(self, handle: ctypes.c_void_p, Z, out):
        self._h = handle
        self._keep = (Z, out)  # the host buffers must outlive the request

    def wait(self):
        if self._h is None:
            raise ValueError("ticket already waited on")
        lat = ctypes.c_double()
        h, self._h = self._h, None
        st = lib().fastmuygps_server_wait(h, ctypes.byref(lat))
        _check(st)
        return self._keep[1], lat.value


class Server:
    """fastmuygps_server_*: resident models and continuous batching of requests
    (host numpy query arrays) over several in-flight slots."""

    def __init__(self, hbm_budget: int = 0, slots: int = 3, max_batch: int = 16384,
                 use_graphs: bool = True, swap_idle: bool = False):
        opts = FmgServerOpts(int(slots), int(max_batch), 1 if use_graphs else 0,
                             1 if swap_idle else 0)
        h = ctypes.c_void_p()
        _check(lib().fastmuygps_server_create(int(hbm_budget), ctypes.byref(opts),
                                             ctypes.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self._models = {}

    def add_model(self, model: Model) -> tuple:
        """Returns (id, admitted); a model that does not fit waits (admitted False)."""
        mid = ctypes.c_int32()
        st = lib().fastmuygps_server_add_model(self._h, model.handle, ctypes.byref(mid))
        _check(st, allow=(FMG_E_BUSY,))
        self._models[mid.value] = model
        return mid.value, st == FMG_OK

    def remove_model(self, mid: int) -> None:
        _check(lib().fastmuygps_server_remove_model(self._h, int(mid)))
        self._models.pop(mid, None)

    def submit(self, mid: int, Z, arrival_ns: int = 0) -> Ticket:
        import numpy as np
        model = self._models[mid]
        dt = np.float64 if model.dtype == torch.float64 else np.float32
        Z = np.ascontiguousarray(Z, dtype=dt)
        if Z.ndim != 2 or Z.shape[1] != model.d:
            raise ValueError("Z must be [B, %d]" % model.d)
        out = np.empty((Z.shape[0], model.ell), dtype=dt)
        t = ctypes.c_void_p()
        _check(lib().fastmuygps_server_submit(self._h, int(mid), Z.ctypes.data, Z.shape[0],
                                             out.ctypes.data, int(arrival_ns), ctypes.byref(t)))
        return Ticket(t, Z, out)

    def stats(self) -> dict:
        st = FmgServerStats()
        _check(lib().fastmuygps_server_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in FmgServerStats._fields_}

    def reset_stats(self) -> None:
        _check(lib().fastmuygps_server_reset_stats(self._h))

    def close(self) -> None:
        if self._h:
            lib().fastmuygps_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
