"""Helpers shared by the GPU parity tests: tolerance definitions and oracle
comparisons.  The oracle (FP64, CPU) always receives exactly the values the
GPU receives, widened to double."""
from __future__ import annotations

import math

import numpy as np

import oracle

# Relative tolerance on posterior means (max over queries and responses of
# |mu_gpu - mu_oracle| / max(|mu_oracle|, RMS(mu_oracle))).
TOL_MEAN = {"fp64": 1e-10, "fp32": 2e-4, "mixed": 2e-4}
# |RMSE_gpu / RMSE_oracle - 1| on the same queries.
TOL_RMSE = 1e-3


def rel_err(got, ref) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    rms = math.sqrt(float(np.mean(ref * ref)))
    if rms == 0.0:
        return float(np.max(np.abs(got - ref)))
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), rms)))


def rmse(mu, y) -> float:
    d = np.asarray(mu, dtype=np.float64) - np.asarray(y, dtype=np.float64)
    return math.sqrt(float(np.mean(d * d)))


def backward_error(X, Y, nb, C, kernel, nu, rho, noise):
    """Normwise backward error ||K C - Y_N|| / (||K|| ||C|| + ||Y_N||) of each
    row's coefficient solve, with K assembled by the oracle in FP64."""
    out = []
    for r in range(nb.shape[0]):
        K = oracle.assemble(X, nb[r], kernel, nu, rho, noise, 1.0)
        yN = np.asarray(Y, dtype=np.float64)[nb[r]]
        c = np.asarray(C[r], dtype=np.float64).reshape(yN.shape)
        res = K @ c - yN
        den = np.linalg.norm(K, 2) * np.linalg.norm(c) + np.linalg.norm(yN)
        out.append(np.linalg.norm(res) / den)
    return np.asarray(out)


def forward_error_bound_ok(X, Y, nb, C_gpu, C_ref, kernel, nu, rho, noise, unit, factor=50.0):
    """|C_gpu - C_ref| <= factor * kappa(K) * k * unit * max|C_ref| per row."""
    bad = []
    for r in range(nb.shape[0]):
        K = oracle.assemble(X, nb[r], kernel, nu, rho, noise, 1.0)
        kappa = np.linalg.cond(K)
        k = nb.shape[1]
        scale = max(float(np.max(np.abs(C_ref[r]))), 1e-300)
        err = float(np.max(np.abs(np.asarray(C_gpu[r], dtype=np.float64) - C_ref[r])))
        if err > factor * kappa * k * unit * scale:
            bad.append((r, err / scale, kappa))
    return bad
