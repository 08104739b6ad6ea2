"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against an independent source: brute force with
numpy, the general Matern formula through SciPy's Bessel function,
scikit-learn's kernels, explicit matrix inversion, the dense GP posterior
mean, and closed forms.  A plausible mistake anywhere in the oracle fails at
least one of them:
  - a dropped or wrong kernel term      -> Matern/Bessel, sklearn, dense-GP
  - a wrong sign, index or transpose in the Cholesky or the solves
                                         -> explicit inverse, dense-GP, LOO
  - a self-inclusive / LOO mix-up        -> LOO invariant, dense-GP(n-1)
  - nugget on cross terms or by distance -> k=1 form, duplicates, amplitude
  - wrong tie-break or off-by-one in kNN -> lexsort brute force on grids
"""
import math

import numpy as np
import pytest
from scipy import special
from sklearn.gaussian_process.kernels import RBF as SkRBF
from sklearn.gaussian_process.kernels import Matern as SkMatern

import oracle
import synth


def np_sqdist(X, q):
    return ((X - q) ** 2).sum(axis=1)


def lexsort_order(D):
    idx = np.arange(D.shape[0])
    return np.lexsort((idx, D))


def rel_err(got, ref):
    """max |got - ref| / max(|ref|, RMS(ref)): relative error that stays
    meaningful for means near zero."""
    ref = np.asarray(ref, dtype=np.float64)
    rms = math.sqrt(float(np.mean(ref * ref)))
    return float(np.max(np.abs(np.asarray(got) - ref) / np.maximum(np.abs(ref), rms)))


def sk_kernel(kernel, nu, rho):
    if kernel == "rbf":
        return SkRBF(length_scale=rho)
    return SkMatern(length_scale=rho, nu=nu)


# --------------------------------------------------------------------------------------
# Neighbour search (Algorithm 2, offline and online neighbour queries)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("dist,d", [("normal", 1), ("normal", 2), ("normal", 3), ("normal", 8),
                                    ("grid", 2), ("grid", 3), ("dups", 4)])
def test_neighbors_match_lexsort(dist, d):
    X, _, Z = synth.small(300, 40, d, seed=d + 7, dist=dist)
    for k in (1, 5, 30, 299):
        for i in (0, 17, 150, 299):
            D = np_sqdist(X, X[i])
            order = [p for p in lexsort_order(D) if p != i][:k]
            got = oracle.neighborhood(X, i, k, oracle.MODE_LOO)
            assert got.tolist() == order
            got_self = oracle.neighborhood(X, i, k, oracle.MODE_SELF)
            assert got_self[0] == i
            assert got_self[1:].tolist() == order[:k - 1]
    nn, dm = oracle.nearest(X, Z)
    for t in range(Z.shape[0]):
        D = np_sqdist(X, Z[t])
        assert nn[t] == lexsort_order(D)[0]
        # numpy may sum the d squares in another order: equal to rounding
        assert abs(dm[t] - D[nn[t]]) <= 2 * d * np.finfo(np.float64).eps * D[nn[t]]


def test_grid_ties_go_to_smaller_index():
    # Four points at the same distance from the origin, listed in scrambled order.
    X = np.array([[0.0, 0.0], [0.0, 1.0], [1.0, 0.0], [-1.0, 0.0], [0.0, -1.0], [2.0, 2.0]])
    assert oracle.neighborhood(X, 0, 3).tolist() == [1, 2, 3]
    nn, _ = oracle.nearest(X, np.array([[0.5, 0.5]]))
    assert nn[0] == 0  # (0,0), (0,1), (1,0) tie; smallest index wins
    # duplicated point: its copy is at distance 0 and is its nearest other point
    Xd = np.vstack([X, X[2:3]])
    assert oracle.neighborhood(Xd, 2, 1).tolist() == [6]
    assert oracle.neighborhood(Xd, 6, 1).tolist() == [2]


def test_too_few_points_is_an_error():
    X = np.zeros((3, 2))
    with pytest.raises(ValueError):
        oracle.neighborhood(X, 0, 3, oracle.MODE_LOO)
    assert oracle.neighborhood(X, 0, 3, oracle.MODE_SELF).tolist() == [0, 1, 2]


# --------------------------------------------------------------------------------------
# Kernels (Section 2, Matern equation and its limits)
# --------------------------------------------------------------------------------------

def matern_bessel(r, nu, rho, amp=1.0):
    """General Matern of Section 2 through the modified Bessel function K_nu,
    evaluated in log space: a 2^(1-nu)/Gamma(nu) s^nu K_nu(s), s = sqrt(2 nu) r/rho."""
    s = math.sqrt(2.0 * nu) * np.asarray(r, dtype=np.float64) / rho
    logv = (1.0 - nu) * math.log(2.0) - special.gammaln(nu) + nu * np.log(s) + \
        np.log(special.kve(nu, s)) - s
    return amp * np.exp(logv)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_matern_closed_forms_match_bessel(nu):
    rho = 0.37
    r = np.logspace(-6, math.log10(20.0), 400) * rho
    got = oracle.phi(r * r, "matern", nu, rho, 1.0)
    ref = matern_bessel(r, nu, rho)
    assert np.max(np.abs(got - ref) / ref) < 1e-13
    # sklearn's Matern is a separate implementation of the same definition
    sk = sk_kernel("matern", nu, rho)(np.zeros((1, 1)), r[:, None])[0]
    assert np.max(np.abs(got - sk) / sk) < 1e-13
    assert oracle.phi(np.array([0.0]), "matern", nu, rho, 2.5)[0] == 2.5


def test_rbf_matches_sklearn_and_is_the_matern_limit():
    rho = 1.3
    r = np.linspace(0.0, 6.0, 301) * rho
    got = oracle.phi(r * r, "rbf", 0.0, rho, 1.0)
    sk = SkRBF(length_scale=rho)(np.zeros((1, 1)), r[:, None])[0]
    assert np.max(np.abs(got - sk)) < 1e-15
    assert got[0] == 1.0
    rr = r[1:]
    errs = []
    for nu in (12.5, 25.0, 50.0):
        errs.append(np.max(np.abs(matern_bessel(rr, nu, rho) - got[1:])))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2
    # roughly 1/nu convergence
    assert errs[1] / errs[2] > 1.6


def test_unsupported_nu_is_nan():
    assert np.isnan(oracle.phi(np.array([1.0]), "matern", 0.75, 1.0, 1.0)[0])


# --------------------------------------------------------------------------------------
# Assembly and solve (Section 3, coefficient equation)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,nu", [("matern", 0.5), ("matern", 1.5), ("matern", 2.5),
                                       ("rbf", 0.0)])
def test_assembly_matches_sklearn(kernel, nu):
    X, _, _ = synth.small(64, 1, 5, seed=3)
    nb = np.array([5, 9, 0, 33, 12, 7], dtype=np.int32)
    K = oracle.assemble(X, nb, kernel, nu, 0.8, 0.05, 1.0)
    ref = sk_kernel(kernel, nu, 0.8)(X[nb]) + 0.05 * np.eye(nb.size)
    assert np.max(np.abs(K - ref)) < 1e-14
    # nugget by index only: a duplicated neighbour gets no nugget off-diagonal
    nbd = np.array([5, 5, 9], dtype=np.int32)
    Kd = oracle.assemble(X, nbd, kernel, nu, 0.8, 0.05, 1.0)
    assert Kd[0, 1] == 1.0 and Kd[0, 0] == 1.05 and Kd[1, 1] == 1.05


@pytest.mark.parametrize("k", [1, 2, 7, 30, 64])
def test_cholesky_solve_matches_explicit_inverse(k):
    rs = np.random.default_rng(k)
    A = rs.normal(size=(k, k))
    K = A @ A.T + 0.5 * np.eye(k)
    Y = rs.normal(size=(k, 3))
    L = oracle.cholesky(K)
    assert L is not None
    assert np.max(np.abs(L @ L.T - K)) < 1e-12 * np.max(np.abs(K)) * k
    C = oracle.cholesky_solve(L, Y)
    ref = np.linalg.inv(K) @ Y
    kappa = np.linalg.cond(K)
    tol = 10.0 * kappa * k * np.finfo(np.float64).eps
    assert np.max(np.abs(C - ref)) / np.max(np.abs(ref)) < tol


def test_cholesky_rejects_non_pd():
    assert oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]])) is None
    assert oracle.cholesky(np.array([[0.0]])) is None
    assert oracle.cholesky(np.array([[np.nan]])) is None


def test_duplicates_without_noise_are_flagged_not_pd():
    X = np.array([[0.0], [1.0], [1.0], [2.0], [5.0]])
    Y = np.arange(5.0)[:, None]
    N, C, st = oracle.build_model(X, Y, 3, "rbf", 0.0, 1.0, noise=0.0)
    # rows whose neighbourhood holds both copies of x=1 are singular
    for i in range(5):
        has_both = 1 in N[i] and 2 in N[i]
        assert (st[i] == 1) == has_both
        assert np.all(np.isnan(C[i])) == has_both


# --------------------------------------------------------------------------------------
# End to end (Algorithm 2) against the dense GP and MuyGPs
# --------------------------------------------------------------------------------------

def dense_gp_mean(Xtr, ytr, Z, kernel, nu, rho, noise):
    """Posterior mean of Section 2 (K(Z,X) K(X,X)^{-1} Y) with the nugget on the
    training diagonal, via sklearn kernels and a dense LU solve."""
    kf = sk_kernel(kernel, nu, rho)
    K = kf(Xtr) + noise * np.eye(Xtr.shape[0])
    return kf(Z, Xtr) @ np.linalg.solve(K, ytr)


@pytest.mark.parametrize("kernel,nu", [("matern", 1.5), ("matern", 2.5), ("rbf", 0.0),
                                       ("matern", 0.5)])
def test_k_equals_n_minus_1_is_the_dense_gp_without_j(kernel, nu):
    X, Y, Z = synth.small(120, 25, 3, ell=2, seed=11)
    rho, noise = 1.2, 1e-2
    n = X.shape[0]
    mu, nn, _ = oracle.predict(X, Y, Z, n - 1, kernel, nu, rho, noise)
    for t in range(Z.shape[0]):
        keep = np.arange(n) != nn[t]
        ref = dense_gp_mean(X[keep], Y[keep], Z[t:t + 1], kernel, nu, rho, noise)[0]
        assert rel_err(mu[t], ref) < 1e-10


def test_self_mode_with_k_equals_n_is_the_dense_gp():
    X, Y, Z = synth.small(90, 20, 2, ell=1, seed=12)
    n = X.shape[0]
    mu, _, _ = oracle.predict(X, Y, Z, n, "matern", 2.5, 0.9, 5e-3, mode=oracle.MODE_SELF)
    ref = dense_gp_mean(X, Y, Z, "matern", 2.5, 0.9, 5e-3)
    assert rel_err(mu, ref) < 1e-10


@pytest.mark.parametrize("kernel,nu", [("matern", 1.5), ("rbf", 0.0)])
def test_query_on_training_point_is_the_muygps_loo_prediction(kernel, nu):
    X, Y, _ = synth.small(400, 1, 4, ell=3, seed=13)
    k, rho, noise = 20, 1.0, 1e-2
    rows = np.array([0, 1, 57, 399])
    mu, nn, dm = oracle.predict(X, Y, X[rows], k, kernel, nu, rho, noise)
    assert nn.tolist() == rows.tolist() and np.all(dm == 0.0)
    kf = sk_kernel(kernel, nu, rho)
    for t, i in enumerate(rows):
        D = np_sqdist(X, X[i])
        nb = [p for p in lexsort_order(D) if p != i][:k]
        K = kf(X[nb]) + noise * np.eye(k)
        ref = kf(X[i:i + 1], X[nb]) @ np.linalg.solve(K, Y[nb])
        assert rel_err(mu[t], ref[0]) < 1e-12


def test_k1_closed_form():
    X, Y, Z = synth.small(200, 30, 2, ell=1, seed=14)
    rho, noise, amp = 0.7, 0.3, 1.0
    mu, nn, _ = oracle.predict(X, Y, Z, 1, "matern", 1.5, rho, noise, amp)
    N, _, _ = oracle.build_model(X, Y, 1, "matern", 1.5, rho, noise, amp)
    for t in range(Z.shape[0]):
        p = N[nn[t], 0]
        r = math.sqrt(np_sqdist(X[p:p + 1], Z[t])[0])
        s = math.sqrt(3.0) * r / rho
        ref = amp * (1 + s) * math.exp(-s) * Y[p, 0] / (amp + noise)
        assert abs(mu[t, 0] - ref) <= 4e-16 * max(abs(ref), 1e-300) + 1e-300


def test_amplitude_and_nugget_scale_together():
    X, Y, Z = synth.small(300, 40, 3, ell=2, seed=15)
    a1 = oracle.predict(X, Y, Z, 15, "matern", 2.5, 1.0, 1e-2, 1.0)[0]
    a2 = oracle.predict(X, Y, Z, 15, "matern", 2.5, 1.0, 1e-2 * 3.7, 3.7)[0]
    assert rel_err(a2, a1) < 1e-12


def test_multi_response_columns_are_independent_runs():
    X, Y, Z = synth.small(250, 30, 3, ell=3, seed=16)
    N, C, st = oracle.build_model(X, Y, 12, "rbf", 0.0, 1.0, 1e-2)
    mu = oracle.predict(X, Y, Z, 12, "rbf", 0.0, 1.0, 1e-2, model=(N, C, st))[0]
    for c in range(3):
        Nc, Cc, _ = oracle.build_model(X, Y[:, c:c + 1], 12, "rbf", 0.0, 1.0, 1e-2)
        assert np.array_equal(N, Nc)
        assert np.array_equal(C[:, :, c], Cc[:, :, 0])
        muc = oracle.predict(X, Y[:, c:c + 1], Z, 12, "rbf", 0.0, 1.0, 1e-2,
                             model=(Nc, Cc, None))[0]
        assert np.array_equal(mu[:, c], muc[:, 0])


def test_two_by_two_worked_example():
    """Three points on a line, k=2 LOO, RBF: every quantity by hand."""
    X = np.array([[0.0], [1.0], [3.0]])
    Y = np.array([[1.0], [2.0], [4.0]])
    rho, s2 = 1.0, 0.5
    N, C, st = oracle.build_model(X, Y, 2, "rbf", 0.0, rho, s2)
    assert N.tolist() == [[1, 2], [0, 2], [1, 0]]
    # row 0: neighbourhood {x=1, x=3}: K = [[1.5, e^-2], [e^-2, 1.5]]
    e = math.exp(-2.0)
    det = 1.5 * 1.5 - e * e
    c0 = (1.5 * 2.0 - e * 4.0) / det
    c1 = (-e * 2.0 + 1.5 * 4.0) / det
    assert abs(C[0, 0, 0] - c0) < 1e-15 and abs(C[0, 1, 0] - c1) < 1e-15
    # query z = 0.25 -> nearest training point 0
    mu, nn, _ = oracle.predict(X, Y, np.array([[0.25]]), 2, "rbf", 0.0, rho, s2,
                               model=(N, C, st))
    ref = math.exp(-(0.75 ** 2) / 2) * c0 + math.exp(-(2.75 ** 2) / 2) * c1
    assert nn[0] == 0 and abs(mu[0, 0] - ref) < 1e-15


def test_thread_count_does_not_change_results():
    X, Y, Z = synth.small(500, 50, 3, ell=2, seed=17)
    N1, C1, _ = oracle.build_model(X, Y, 10, "matern", 1.5, 0.5, 1e-3, nthreads=1)
    N4, C4, _ = oracle.build_model(X, Y, 10, "matern", 1.5, 0.5, 1e-3, nthreads=4)
    assert np.array_equal(N1, N4) and np.array_equal(C1, C4)


# --------------------------------------------------------------------------------------
# MuyGPs prediction of novel points (Section 2.1, MuyGPs prediction equation)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("kernel,nu", [("matern", 0.5), ("matern", 1.5), ("matern", 2.5),
                                       ("rbf", 0.0)])
def test_muygps_with_k_equals_n_is_the_dense_gp(kernel, nu):
    X, Y, Z = synth.small(110, 30, 3, ell=2, seed=31)
    rho, noise = 1.1, 1e-2
    mu, nb, st = oracle.muygps_predict(X, Y, Z, X.shape[0], kernel, nu, rho, noise)
    assert np.all(st == 0)
    assert rel_err(mu, dense_gp_mean(X, Y, Z, kernel, nu, rho, noise)) < 1e-10


@pytest.mark.parametrize("dist,d,k", [("normal", 2, 7), ("grid", 2, 9), ("dups", 3, 5)])
def test_muygps_neighbourhoods_match_lexsort(dist, d, k):
    X, Y, Z = synth.small(500, 40, d, ell=1, seed=32, dist=dist)
    _, nb, _ = oracle.muygps_predict(X, Y, Z, k, "matern", 1.5, 1.0, 1e-2)
    for t in range(Z.shape[0]):
        assert nb[t].tolist() == lexsort_order(np_sqdist(X, Z[t]))[:k].tolist()


def test_muygps_matches_an_independent_local_solve():
    X, Y, Z = synth.small(800, 25, 4, ell=3, seed=33)
    k, rho, noise = 24, 0.8, 2e-2
    mu, nb, _ = oracle.muygps_predict(X, Y, Z, k, "matern", 2.5, rho, noise)
    kf = sk_kernel("matern", 2.5, rho)
    for t in range(Z.shape[0]):
        idx = lexsort_order(np_sqdist(X, Z[t]))[:k]
        ref = kf(Z[t:t + 1], X[idx]) @ np.linalg.solve(kf(X[idx]) + noise * np.eye(k), Y[idx])
        assert rel_err(mu[t], ref[0]) < 1e-11


def test_muygps_k1_closed_form():
    X, Y, Z = synth.small(150, 20, 2, ell=1, seed=34)
    rho, noise = 0.6, 0.25
    mu, nb, _ = oracle.muygps_predict(X, Y, Z, 1, "rbf", 0.0, rho, noise)
    for t in range(Z.shape[0]):
        p = int(np.argmin(np_sqdist(X, Z[t])))
        assert nb[t, 0] == p
        ref = math.exp(-np_sqdist(X[p:p + 1], Z[t])[0] / (2 * rho * rho)) * Y[p, 0] / (1 + noise)
        assert abs(mu[t, 0] - ref) <= 4e-16 * max(abs(ref), 1e-300) + 1e-300


# --- Leave-one-out loss Q(theta) and its gradient (Algorithm 1) -----------------------

KERNELS4 = [("matern", 0.5), ("matern", 1.5), ("matern", 2.5), ("rbf", 0.0)]


@pytest.mark.parametrize("kernel,nu", KERNELS4)
def test_dphi_drho_matches_finite_differences(kernel, nu):
    # central differences of the (Bessel- and sklearn-pinned) kernel value in rho
    D = np.array([0.0, 1e-6, 0.01, 0.3, 1.0, 2.5, 9.0, 40.0])
    for rho in (0.3, 1.0, 2.7):
        h = 1e-5 * rho
        fd = (oracle.phi(D, kernel, nu, rho + h) - oracle.phi(D, kernel, nu, rho - h)) / (2 * h)
        got = oracle.dphi_drho(D, kernel, nu, rho)
        assert np.all(np.abs(got - fd) <= 1e-8 * (np.abs(fd) + 1.0 / rho))
    assert oracle.dphi_drho(np.array([0.0]), kernel, nu, 1.0)[0] == 0.0


def composed_loo_loss(X, Y, rows, k, kernel, nu, rho, noise):
    """Q(theta) composed from pinned parts: the coefficient rows of the batch
    points and their means at z = x_i, which are MuyGPs' leave-one-out
    predictions (pinned above by an independent dense solve)."""
    N, C, _ = oracle.build_model(X, Y, k, kernel, nu, rho, noise, rows=rows)
    mu = oracle.means(X, X[rows], N, C, kernel, nu, rho)
    return float(np.mean((Y[rows] - mu) ** 2))


@pytest.mark.parametrize("kernel,nu", KERNELS4)
def test_loo_loss_is_the_composed_loss(kernel, nu):
    X, Y, _ = synth.small(500, 1, 3, ell=2, seed=81)
    rows = np.random.default_rng(1).choice(500, 60, replace=False)
    q, _, terms, st = oracle.loo_loss_grad(X, Y, rows, 12, kernel, nu, 0.9, 1e-2)
    ref = composed_loo_loss(X, Y, rows, 12, kernel, nu, 0.9, 1e-2)
    assert np.all(st == 0)
    assert abs(q - ref) <= 1e-12 * ref
    assert terms.shape == (60, 3)


@pytest.mark.parametrize("kernel,nu", KERNELS4)
def test_loo_gradient_matches_finite_differences(kernel, nu):
    X, Y, _ = synth.small(400, 1, 3, ell=2, seed=82)
    Y = np.sin(2.0 * X[:, :2]) + 0.1 * Y  # smooth signal: an interior optimum in rho
    rows = np.random.default_rng(2).choice(400, 50, replace=False)
    k = 10
    for rho, noise in ((0.7, 1e-2), (1.6, 0.2)):
        q, g, _, _ = oracle.loo_loss_grad(X, Y, rows, k, kernel, nu, rho, noise)
        hr, hn = 1e-5 * rho, 1e-5 * noise
        fr = (composed_loo_loss(X, Y, rows, k, kernel, nu, rho + hr, noise)
              - composed_loo_loss(X, Y, rows, k, kernel, nu, rho - hr, noise)) / (2 * hr)
        fn = (composed_loo_loss(X, Y, rows, k, kernel, nu, rho, noise + hn)
              - composed_loo_loss(X, Y, rows, k, kernel, nu, rho, noise - hn)) / (2 * hn)
        assert abs(g[0] - fr) <= 1e-6 * abs(fr) + 1e-9 * q / rho
        assert abs(g[1] - fn) <= 1e-6 * abs(fn) + 1e-9 * q / noise


def test_loo_gradient_k1_closed_form():
    # k = 1: mu_i = phi(r_ip) y_p / (a + sigma^2), p the nearest other point
    X, Y, _ = synth.small(120, 1, 2, ell=1, seed=83)
    rho, noise = 0.8, 0.3
    rows = np.arange(0, 120, 3)
    q, g, _, _ = oracle.loo_loss_grad(X, Y, rows, 1, "matern", 2.5, rho, noise)
    sq, gr, gs = 0.0, 0.0, 0.0
    for i in rows:
        D = np_sqdist(X, X[i])
        p = [j for j in lexsort_order(D) if j != i][0]
        ph = oracle.phi(D[p], "matern", 2.5, rho)
        dph = oracle.dphi_drho(D[p], "matern", 2.5, rho)
        e = ph * Y[p, 0] / (1 + noise) - Y[i, 0]
        sq += e * e
        gr += 2 * e * dph * Y[p, 0] / (1 + noise)
        gs += 2 * e * (-ph * Y[p, 0] / (1 + noise) ** 2)
    b = len(rows)
    assert abs(q - sq / b) <= 1e-13 * (sq / b)
    assert abs(g[0] - gr / b) <= 1e-12 * abs(gr / b) + 1e-15
    assert abs(g[1] - gs / b) <= 1e-12 * abs(gs / b) + 1e-15


def test_loo_gradient_rows_without_enough_points_are_flagged():
    X, Y, _ = synth.small(5, 1, 2, ell=1, seed=84)
    _, _, terms, st = oracle.loo_loss_grad(X, Y, np.array([0, 1]), 5, "matern", 1.5, 1.0, 0.1)
    assert st.tolist() == [2, 2] and np.all(np.isnan(terms))
