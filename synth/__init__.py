"""Seeded synthetic workloads shaped like the paper's experiments.

This module only draws inputs: training features X, responses Y, queries Z,
their true responses, hyperparameters and request arrival streams.  It holds
none of the FastMuyGPs arithmetic, so both the FP64 oracle and the HIP path
consume exactly the same arrays without depending on each other.

Randomness: numpy ``Generator(PCG64(SeedSequence([220510879, cfg, role])))``
with role 0 = parameters, 1 = training set, 2 = test set, 3 = arrivals,
4 = oracle sample.  FP32 workloads are rounded to float32 here, at generation,
so every consumer sees the same values.

Workloads (the paper's datasets are not available; these stand in for their
shapes):
  cfg 1: 2-D spatial field on the unit square, Matern nu=3/2, FP64
         (stands in for the MODIS land-surface temperature set, Section 4.1).
  cfg 2: 8-D Gaussian inputs with a random-Fourier response, Matern nu=5/2,
         FP32 (n and d of the borehole emulation, Section 4.2).
  cfg 3: 40-D ten-cluster Gaussian mixture with a one-hot +-0.5 multi-response,
         RBF, mixed precision (stands in for the star/galaxy classifier,
         Section 4.3).
  cfg 5a: 3-D uniform inputs with a random-Fourier response, Matern nu=1/2;
         with eight models of the kinds above (cfg5_models) it forms the
         multi-model serving workload.
  cfg 6: the borehole flow-rate function (Section 4.2) on Latin-hypercube
         inputs, anisotropically scaled, RBF with k = 150, FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED = 220510879


def rng(cfg: int, role: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, cfg, role])))


@dataclass
class Workload:
    name: str
    X: np.ndarray          # [n, d] training features (float64 or float32)
    Y: np.ndarray          # [n, ell] training responses
    Z: np.ndarray          # [m, d] queries
    Yz: np.ndarray         # [m, ell] true responses at the queries
    k: int
    kernel: str            # "rbf" | "matern"
    nu: float
    rho: float
    noise: float
    precision: str         # "fp64" | "fp32" | "mixed"
    extra: dict = field(default_factory=dict)

    @property
    def hyper(self) -> dict:
        return dict(kernel=self.kernel, nu=self.nu, rho=self.rho, noise=self.noise)


def _fourier(rs: np.random.Generator, terms: int, d: int, scale: float):
    w = rs.normal(0.0, 1.0 / scale, size=(terms, d))
    a = rs.normal(0.0, math.sqrt(1.0 / terms), size=terms)
    b = rs.uniform(0.0, 2.0 * math.pi, size=terms)
    return w, a, b


def _fourier_eval(X, w, a, b):
    return np.cos(X.astype(np.float64) @ w.T + b) @ a


def cfg1(n: int = 10_000, m: int = 1_000, cfg: int = 1) -> Workload:
    """n points uniform on [0,1]^2, y = sin(2 pi x1) cos(2 pi x2) + N(0, 0.01^2);
    k=30, Matern nu=3/2, rho=0.1, sigma^2=1e-4, FP64.  `cfg` selects the seed
    stream (other values draw further models of the same kind)."""
    def draw(role, cnt):
        rs = rng(cfg, role)
        X = rs.uniform(0.0, 1.0, size=(cnt, 2))
        y = np.sin(2 * np.pi * X[:, 0]) * np.cos(2 * np.pi * X[:, 1])
        y = y + rs.normal(0.0, 0.01, size=cnt)
        return X, y[:, None]
    X, Y = draw(1, n)
    Z, Yz = draw(2, m)
    return Workload("cfg1-spatial2d", X, Y, Z, Yz, 30, "matern", 1.5, 0.1, 1e-4, "fp64")


def cfg2(n: int = 100_000, m: int = 100_000, cfg: int = 2) -> Workload:
    """X ~ N(0, I_8), y = sum_{64} a cos(w.x + b) + N(0, 0.05^2) with
    w ~ N(0, I/0.5^2), a ~ N(0, 1/64), b ~ U[0, 2pi); k=50, Matern nu=5/2,
    rho=1, sigma^2=1e-3, FP32.  `cfg` selects the seed stream."""
    w, a, b = _fourier(rng(cfg, 0), 64, 8, 0.5)

    def draw(role, cnt):
        rs = rng(cfg, role)
        X = rs.normal(0.0, 1.0, size=(cnt, 8)).astype(np.float32)
        y = _fourier_eval(X, w, a, b) + rs.normal(0.0, 0.05, size=cnt)
        return X, y.astype(np.float32)[:, None]
    X, Y = draw(1, n)
    Z, Yz = draw(2, m)
    return Workload("cfg2-fourier8d", X, Y, Z, Yz, 50, "matern", 2.5, 1.0, 1e-3, "fp32")


def cfg3(n: int = 1_000_000, m: int = 200_000, d: int = 40, classes: int = 10,
         cfg: int = 3) -> Workload:
    """Ten-cluster Gaussian mixture in 40-D: means ~ N(0, 4 I), unit covariance,
    labels uniform; responses are the one-hot label mapped 1 -> +0.5,
    0 -> -0.5 (ell = 10).  k=50, RBF, rho=3, sigma^2=1e-2, mixed precision.
    `cfg` selects the seed stream."""
    means = rng(cfg, 0).normal(0.0, 2.0, size=(classes, d))

    def draw(role, cnt):
        rs = rng(cfg, role)
        lab = rs.integers(0, classes, size=cnt)
        X = means[lab] + rs.normal(0.0, 1.0, size=(cnt, d))
        Y = np.full((cnt, classes), -0.5, dtype=np.float32)
        Y[np.arange(cnt), lab] = 0.5
        return X.astype(np.float32), Y, lab
    X, Y, lx = draw(1, n)
    Z, Yz, lz = draw(2, m)
    return Workload("cfg3-mixture40d", X, Y, Z, Yz, 50, "rbf", 0.0, 3.0, 1e-2, "mixed",
                    extra={"labels_train": lx, "labels_test": lz, "means": means})


def cfg5a(n: int = 5_000_000, m: int = 100_000) -> Workload:
    """X ~ U[0,1]^3, y = sum_{32} a cos(w.x + b) + N(0, 0.02^2) with
    w ~ N(0, I/0.2^2), a ~ N(0, 1/32); k=30, Matern nu=1/2, FP32.  The length
    scale and noise are not given by the workload description; rho=0.2 and
    sigma^2=4e-4 (the noise variance) are the readings used here."""
    w, a, b = _fourier(rng(5, 0), 32, 3, 0.2)

    def draw(role, cnt):
        rs = rng(5, role)
        X = rs.uniform(0.0, 1.0, size=(cnt, 3)).astype(np.float32)
        y = _fourier_eval(X, w, a, b) + rs.normal(0.0, 0.02, size=cnt)
        return X, y.astype(np.float32)[:, None]
    X, Y = draw(1, n)
    Z, Yz = draw(2, m)
    return Workload("cfg5a-fourier3d", X, Y, Z, Yz, 30, "matern", 0.5, 0.2, 4e-4, "fp32")


def cfg5_specs():
    """The eight further models of the multi-model serving workload: n
    log-uniform in [1e4, 2e6], d uniform on {2, 8, 40}, k uniform on {30, 50}
    (drawn from seed stream 50).  Returns [(n, d, k)]."""
    rs = rng(50, 0)
    n = np.floor(np.exp(rs.uniform(math.log(1e4), math.log(2e6), size=8))).astype(np.int64)
    d = rs.choice([2, 8, 40], size=8)
    k = rs.choice([30, 50], size=8)
    return [(int(n[i]), int(d[i]), int(k[i])) for i in range(8)]


def cfg5_models(m: int = 65_536, n_a: int = 5_000_000):
    """Model A (cfg5a: n = 5,000,000, d = 3, Matern nu=1/2, FP32) and the eight
    models of cfg5_specs().  Each of those takes the generator, kernel,
    precision and number of responses of the workload of its dimension: d=2
    like cfg 1 (FP64, Matern 3/2, ell 1), d=8 like cfg 2 (FP32, Matern 5/2,
    ell 1), d=40 like cfg 3 (mixed, RBF, ell 10), on seed stream 51 + i, with
    its own n and k.  m queries per model (the serving pool)."""
    out = [cfg5a(n=n_a, m=m)]
    for i, (n, d, k) in enumerate(cfg5_specs()):
        if d == 2:
            w = cfg1(n=n, m=m, cfg=51 + i)
        elif d == 8:
            w = cfg2(n=n, m=m, cfg=51 + i)
        else:
            w = cfg3(n=n, m=m, cfg=51 + i)
        w.k = k
        w.name = "cfg5-%d-%s-n%d-k%d" % (i + 1, w.name.split("-")[1], n, k)
        out.append(w)
    return out


# Borehole function (Section 4.2): parameter order, bounds, and the divisors
# that make the inputs anisotropic.
BOREHOLE_NAMES = ("r_w", "r", "T_u", "H_u", "T_l", "H_l", "L", "K_w")
BOREHOLE_LO = np.array([0.05, 100.0, 63070.0, 990.0, 63.1, 700.0, 1120.0, 9855.0])
BOREHOLE_HI = np.array([0.15, 50000.0, 115600.0, 1110.0, 116.0, 820.0, 1680.0, 12045.0])
BOREHOLE_SCALE = np.array([0.0625, 0.25, 1.0, 0.25, 0.5, 0.25, 0.125, 0.5])
BOREHOLE_VARY = (0, 1, 2, 4)  # r_w, r, T_u, T_l vary; H_u, H_l, L, K_w are held fixed
BOREHOLE_FIXED_U = 0.5        # reading: the fixed parameters sit at their mid-range


def borehole_flow(P):
    """Water flow rate (m^3/yr) through a borehole for physical parameters
    P [..., 8] in the order of BOREHOLE_NAMES (Section 4.2, borehole
    equation)."""
    P = np.asarray(P, dtype=np.float64)
    rw, r, tu, hu, tl, hl, L, kw = (P[..., j] for j in range(8))
    lg = np.log(r / rw)
    return 2.0 * np.pi * tu * (hu - hl) / (lg * (1.0 + 2.0 * L * tu / (lg * rw * rw * kw) + tu / tl))


def borehole_inputs(U):
    """GP inputs from unit-cube coordinates U [..., 8]: each coordinate divided
    by its anisotropy divisor."""
    return np.asarray(U, dtype=np.float64) / BOREHOLE_SCALE


def borehole_unit(cnt: int, rs: np.random.Generator):
    """Latin-hypercube sample of the four varying parameters in unit-cube
    coordinates (one point per stratum of each axis, independent random
    permutations, uniform within the stratum); the fixed ones at mid-range."""
    U = np.full((cnt, 8), BOREHOLE_FIXED_U)
    for j in BOREHOLE_VARY:
        U[:, j] = (rs.permutation(cnt) + rs.uniform(0.0, 1.0, size=cnt)) / cnt
    return U


def borehole(n: int = 100_000, m: int = 20_000, noise: float = 1e-6) -> Workload:
    """Borehole emulator (Section 4.2): n training and m test points, each a
    Latin-hypercube sample of (r_w, r, T_u, T_l) mapped affinely to its bounds
    with H_u, H_l, L, K_w fixed at mid-range; inputs are the unit-cube
    coordinates divided by [0.0625, 0.25, 1, 0.25, 0.5, 0.25, 0.125, 0.5]; the
    response is the flow rate minus the training mean.  RBF kernel, length
    scale 43.27, k = 150 (the paper's values); the nugget is not given and is
    a reading; FP64."""
    def draw(role, cnt):
        U = borehole_unit(cnt, rng(6, role))
        f = borehole_flow(BOREHOLE_LO + U * (BOREHOLE_HI - BOREHOLE_LO))
        return borehole_inputs(U), f, U
    X, fx, Ux = draw(1, n)
    Z, fz, Uz = draw(2, m)
    mean = float(np.mean(fx))
    return Workload("borehole-emulator8d", X, (fx - mean)[:, None], Z, (fz - mean)[:, None], 150,
                    "rbf", 0.0, 43.27, noise, "fp64",
                    extra={"response_mean": mean, "unit_train": Ux, "unit_test": Uz})


def cfg3_queries(m: int, role: int = 3, d: int = 40, classes: int = 10):
    """Fresh queries from the cfg-3 mixture (serving streams use role 3)."""
    means = rng(3, 0).normal(0.0, 2.0, size=(classes, d))
    rs = rng(3, role)
    lab = rs.integers(0, classes, size=m)
    return (means[lab] + rs.normal(0.0, 1.0, size=(m, d))).astype(np.float32)


def poisson_stream(rate: float, duration: float, bmax: int, cfg: int = 4):
    """Open-loop request stream: Poisson arrival times at `rate` per second and
    batch sizes B = floor(exp(U * ln(bmax + 1))) clipped to [1, bmax]."""
    rs = rng(cfg, 3)
    cnt = int(rate * duration * 1.2) + 16
    gaps = rs.exponential(1.0 / rate, size=cnt)
    t = np.cumsum(gaps)
    t = t[t < duration]
    u = rs.uniform(0.0, 1.0, size=t.shape[0])
    B = np.clip(np.floor(np.exp(u * math.log(bmax + 1))).astype(np.int64), 1, bmax)
    return t, B


def small(n: int, m: int, d: int, ell: int = 1, seed: int = 0, dist: str = "normal",
          dtype=np.float64):
    """Small generic inputs for parity tests.  dist: 'normal', 'uniform',
    'grid' (integer lattice points with many exact distance ties) or 'dups'
    (every training point appears twice)."""
    rs = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED, 100, seed])))
    if dist == "normal":
        X = rs.normal(size=(n, d))
        Z = rs.normal(size=(m, d))
    elif dist == "uniform":
        X = rs.uniform(size=(n, d))
        Z = rs.uniform(size=(m, d))
    elif dist == "grid":
        side = max(2, int(round(n ** (1.0 / d))) + 1)
        X = rs.integers(0, side, size=(n, d)).astype(np.float64)
        Z = rs.integers(0, side, size=(m, d)).astype(np.float64) + 0.5 * rs.integers(0, 2, size=(m, d))
    elif dist == "dups":
        half = rs.normal(size=((n + 1) // 2, d))
        X = np.concatenate([half, half])[:n]
        Z = rs.normal(size=(m, d))
    else:
        raise ValueError(dist)
    Y = rs.normal(size=(n, ell))
    return X.astype(dtype), Y.astype(dtype), Z.astype(dtype)
