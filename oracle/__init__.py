"""FastMuyGPs FP64 CPU oracle (ctypes wrapper around fmg_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain, sequential FP64 statement of the
FastMuyGPs posterior-mean path (Dunton, Priest, Muyskens, arXiv 2205.10879,
Algorithm 2 and the equations of Sections 2-3).  Only tests/,
``__graft_entry__.smoke()`` and the cpu_baseline leg of ``bench.py`` may
import it.  It shares no code with the HIP library and never imports it.

Every function takes float64 numpy arrays (FP32 inputs are widened exactly by
the caller) and returns numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RBF = 0
MATERN = 1
MODE_LOO = 0
MODE_SELF = 1


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc: -O2, no FMA contraction, no fast-math."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        dbl = ctypes.c_double
        lib.oracle_sqdist.argtypes = [P, P, i32]
        lib.oracle_sqdist.restype = dbl
        lib.oracle_phi.argtypes = [dbl, i32, dbl, dbl, dbl]
        lib.oracle_phi.restype = dbl
        lib.oracle_neighborhood.argtypes = [P, i64, i32, i64, i32, i32, P]
        lib.oracle_neighborhood.restype = i32
        lib.oracle_nearest.argtypes = [P, i64, i32, P, P]
        lib.oracle_nearest.restype = i64
        lib.oracle_cholesky.argtypes = [P, i32]
        lib.oracle_cholesky.restype = i32
        lib.oracle_cholesky_solve.argtypes = [P, i32, P, P, i32]
        lib.oracle_cholesky_solve.restype = None
        lib.oracle_assemble.argtypes = [P, i32, P, i32, i32, dbl, dbl, dbl, dbl, P]
        lib.oracle_assemble.restype = None
        lib.oracle_build.argtypes = [P, P, i64, i32, i32, i32, i32, dbl, dbl, dbl, dbl, i32,
                                     P, i64, P, P, P, i32]
        lib.oracle_build.restype = i64
        lib.oracle_nearest_batch.argtypes = [P, i64, i32, P, i64, P, P, i32]
        lib.oracle_nearest_batch.restype = None
        lib.oracle_mean.argtypes = [P, i32, i32, i32, i32, dbl, dbl, dbl, P, P, P, P]
        lib.oracle_mean.restype = None
        lib.oracle_mean_batch.argtypes = [P, i32, i32, i32, i32, dbl, dbl, dbl, P, i64, P, P,
                                          P, i32]
        lib.oracle_mean_batch.restype = None
        lib.oracle_muygps_batch.argtypes = [P, P, i64, i32, i32, i32, i32, dbl, dbl, dbl, dbl,
                                             P, i64, P, P, P, i32]
        lib.oracle_muygps_batch.restype = None
        lib.oracle_dphi_drho.argtypes = [dbl, i32, dbl, dbl, dbl]
        lib.oracle_dphi_drho.restype = dbl
        lib.oracle_loo_loss_grad.argtypes = [P, P, i64, i32, i32, i32, i32, dbl, dbl, dbl, dbl,
                                             P, i64, P, P, i32]
        lib.oracle_loo_loss_grad.restype = i64
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = i32
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _kernel_code(kernel: str) -> int:
    if kernel == "rbf":
        return RBF
    if kernel == "matern":
        return MATERN
    raise ValueError("kernel must be 'rbf' or 'matern'")


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def sqdist(u, v) -> float:
    u = _f64(u)
    v = _f64(v)
    return float(_load().oracle_sqdist(_ptr(u), _ptr(v), u.shape[-1]))


def phi(D, kernel="matern", nu=1.5, rho=1.0, amp=1.0):
    """Kernel values from squared distances D (any shape)."""
    lib = _load()
    D = np.asarray(D, dtype=np.float64)
    out = np.empty_like(D)
    kc = _kernel_code(kernel)
    flat_in = D.reshape(-1)
    flat_out = out.reshape(-1)
    for e in range(flat_in.size):
        flat_out[e] = lib.oracle_phi(float(flat_in[e]), kc, float(nu), float(rho), float(amp))
    return out


def dphi_drho(D, kernel="matern", nu=1.5, rho=1.0, amp=1.0):
    """Derivative of the kernel values with respect to the length scale, from
    squared distances D (any shape)."""
    lib = _load()
    D = np.asarray(D, dtype=np.float64)
    out = np.empty_like(D)
    kc = _kernel_code(kernel)
    flat_in = D.reshape(-1)
    flat_out = out.reshape(-1)
    for e in range(flat_in.size):
        flat_out[e] = lib.oracle_dphi_drho(float(flat_in[e]), kc, float(nu), float(rho),
                                           float(amp))
    return out


def neighborhood(X, i: int, k: int, mode: int = MODE_LOO):
    X = _f64(X)
    n, d = X.shape
    out = np.empty(k, dtype=np.int32)
    rc = _load().oracle_neighborhood(_ptr(X), n, d, int(i), int(k), int(mode), _ptr(out))
    if rc != 0:
        raise ValueError("too few training points for k")
    return out


def nearest(X, Z, nthreads: int = 0):
    """Nearest training index and squared distance of every row of Z."""
    X = _f64(X)
    Z = _f64(np.atleast_2d(Z))
    n, d = X.shape
    m = Z.shape[0]
    nn = np.empty(m, dtype=np.int64)
    dm = np.empty(m, dtype=np.float64)
    _load().oracle_nearest_batch(_ptr(X), n, d, _ptr(Z), m, _ptr(nn), _ptr(dm), int(nthreads))
    return nn, dm


def cholesky(K):
    """Lower Cholesky factor (numpy array) or None when not positive definite."""
    A = _f64(K).copy()
    k = A.shape[0]
    rc = _load().oracle_cholesky(_ptr(A), k)
    if rc != 0:
        return None
    return np.tril(A)


def cholesky_solve(L, Y):
    """Solve L L^T C = Y for Y of shape [k] or [k, ell]."""
    L = _f64(L)
    Y = _f64(Y)
    k = L.shape[0]
    Y2 = Y.reshape(k, -1)
    ell = Y2.shape[1]
    Y2 = np.ascontiguousarray(Y2)
    C = np.empty_like(Y2)
    lib = _load()
    for c in range(ell):
        ycol = np.ascontiguousarray(Y2[:, c])
        ccol = np.empty(k)
        lib.oracle_cholesky_solve(_ptr(L), k, _ptr(ycol), _ptr(ccol), 1)
        C[:, c] = ccol
    return C.reshape(Y.shape)


def assemble(X, nb, kernel="matern", nu=1.5, rho=1.0, noise=0.0, amp=1.0):
    X = _f64(X)
    nb = np.ascontiguousarray(nb, dtype=np.int32)
    k = nb.shape[0]
    K = np.empty((k, k))
    _load().oracle_assemble(_ptr(X), X.shape[1], _ptr(nb), k, _kernel_code(kernel), float(nu),
                            float(rho), float(noise), float(amp), _ptr(K))
    return K


def build_model(X, Y, k: int, kernel="matern", nu=1.5, rho=1.0, noise=0.0, amp=1.0,
                mode: int = MODE_LOO, rows=None, nthreads: int = 0):
    """Offline training (Algorithm 2).  Returns (N [r,k] int32, C [r,k,ell], status [r])."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    n, d = X.shape
    ell = Y.shape[1]
    if rows is None:
        r = n
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        r = rows_arr.shape[0]
    nb = np.empty((r, k), dtype=np.int32)
    C = np.empty((r, k, ell), dtype=np.float64)
    st = np.empty(r, dtype=np.int32)
    _load().oracle_build(_ptr(X), _ptr(Y), n, d, ell, int(k), _kernel_code(kernel), float(nu),
                         float(rho), float(noise), float(amp), int(mode),
                         _ptr(rows_arr) if rows_arr is not None else None, r, _ptr(nb),
                         _ptr(C), _ptr(st), int(nthreads))
    return nb, C, st


def means(X, Z, nb_rows, C_rows, kernel="matern", nu=1.5, rho=1.0, amp=1.0, nthreads: int = 0):
    """Posterior means of the queries Z, query t using nb_rows[t] and C_rows[t]."""
    X = _f64(X)
    Z = _f64(np.atleast_2d(Z))
    nb_rows = np.ascontiguousarray(nb_rows, dtype=np.int32)
    C_rows = _f64(C_rows)
    m = Z.shape[0]
    k = nb_rows.shape[1]
    ell = C_rows.shape[2]
    out = np.empty((m, ell))
    _load().oracle_mean_batch(_ptr(X), X.shape[1], ell, k, _kernel_code(kernel), float(nu),
                              float(rho), float(amp), _ptr(Z), m, _ptr(nb_rows), _ptr(C_rows),
                              _ptr(out), int(nthreads))
    return out


def predict(X, Y, Z, k: int, kernel="matern", nu=1.5, rho=1.0, noise=0.0, amp=1.0,
            mode: int = MODE_LOO, model=None, nthreads: int = 0):
    """Full FastMuyGPs prediction (Algorithm 2, online part) for queries Z.

    When `model` = (N, C, status) for every training row is given it is used;
    otherwise only the rows that are some query's nearest point are trained
    (the sampled oracle).  Returns (means [m, ell], nn [m], dmin [m]).
    """
    nn, dm = nearest(X, Z, nthreads)
    if model is not None:
        N, C, _ = model
        nb_rows = N[nn]
        C_rows = C[nn]
    else:
        uniq, inv = np.unique(nn, return_inverse=True)
        N, C, _ = build_model(X, Y, k, kernel, nu, rho, noise, amp, mode, rows=uniq,
                              nthreads=nthreads)
        nb_rows = N[inv]
        C_rows = C[inv]
    mu = means(X, Z, nb_rows, C_rows, kernel, nu, rho, amp, nthreads)
    return mu, nn, dm


def muygps_predict(X, Y, Z, k: int, kernel="matern", nu=1.5, rho=1.0, noise=0.0, amp=1.0,
                   nthreads: int = 0):
    """MuyGPs prediction of novel points (Section 2.1): for each query its own k
    nearest training points N*, then K(z, X_N*) K(X_N*, X_N*)^{-1} Y(X_N*).
    Returns (means [m, ell], N* [m, k] int32, status [m])."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    Z = _f64(np.atleast_2d(Z))
    n, d = X.shape
    ell = Y.shape[1]
    m = Z.shape[0]
    nb = np.empty((m, k), dtype=np.int32)
    out = np.empty((m, ell))
    st = np.empty(m, dtype=np.int32)
    _load().oracle_muygps_batch(_ptr(X), _ptr(Y), n, d, ell, int(k), _kernel_code(kernel),
                                float(nu), float(rho), float(noise), float(amp), _ptr(Z), m,
                                _ptr(nb), _ptr(out), _ptr(st), int(nthreads))
    return out, nb, st


def loo_loss_grad(X, Y, rows, k: int, kernel="matern", nu=1.5, rho=1.0, noise=0.0, amp=1.0,
                  nthreads: int = 0):
    """Leave-one-out loss Q(theta) of MuyGPs training over the batch `rows`
    (Algorithm 1; Section 2.1) and its gradient with respect to
    (length scale, noise variance).  Returns (Q, grad [2], terms [b, 3],
    status [b]); terms are the unnormalised per-row (loss, d/drho, d/dsigma^2),
    Q and grad their sums over b * ell."""
    X = _f64(X)
    Y = _f64(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    n, d = X.shape
    ell = Y.shape[1]
    b = rows.shape[0]
    terms = np.empty((b, 3))
    st = np.empty(b, dtype=np.int32)
    _load().oracle_loo_loss_grad(_ptr(X), _ptr(Y), n, d, ell, int(k), _kernel_code(kernel),
                                 float(nu), float(rho), float(noise), float(amp), _ptr(rows), b,
                                 _ptr(terms), _ptr(st), int(nthreads))
    tot = terms.sum(axis=0) / (b * ell)
    return float(tot[0]), tot[1:].copy(), terms, st
