"""GPU parity of the leave-one-out loss Q(theta) of MuyGPs hyperparameter
training and of its gradient in (length scale, noise variance) (Algorithm 1;
Section 2.1), through the C ABI, against the FP64 oracle; and of the host-side
L-BFGS-B fit driven by it.  The gradient path computes in FP64 for every model
precision, on the FP32 values widened exactly, so the bar is FP64's."""
import numpy as np
import pytest
import torch
from scipy.optimize import minimize

import oracle
import synth

pytestmark = pytest.mark.gpu

DT = {"fp64": np.float64, "fp32": np.float32, "mixed": np.float32}
TOL = 1e-9  # FP64 arithmetic on identical inputs: only the summation order differs


def fmg():
    import paper_2205_10879_amd as f
    return f


def build(prec, X, Y, k, kernel, nu, rho, noise, flags=0):
    X = np.ascontiguousarray(X, dtype=DT[prec])
    Y = np.ascontiguousarray(Y, dtype=DT[prec])
    model = fmg().fastmuygps_build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), k,
                                   kernel, nu, rho, noise, precision=prec, flags=flags)
    return model, X.astype(np.float64), Y.astype(np.float64)


def check(got_q, got_g, ref_q, ref_g, rho, noise):
    assert abs(got_q - ref_q) <= TOL * ref_q
    assert abs(got_g[0] - ref_g[0]) <= TOL * (abs(ref_g[0]) + ref_q / rho)
    assert abs(got_g[1] - ref_g[1]) <= TOL * (abs(ref_g[1]) + ref_q / max(noise, 1e-12))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
@pytest.mark.parametrize("n,d,k,ell,kernel,nu,rho,noise", [
    (3000, 3, 24, 2, "matern", 1.5, 0.7, 1e-2),   # KMAX 32, ELLMAX 4
    (2000, 5, 50, 10, "rbf", 0.0, 1.2, 3e-2),     # KMAX 64, ELLMAX 16
    (1500, 8, 64, 1, "matern", 2.5, 1.0, 1e-3),   # k at its maximum
    (900, 2, 33, 5, "matern", 0.5, 0.3, 0.1)])    # ragged: one past the small tile
def test_loss_and_gradient_match_the_oracle(prec, n, d, k, ell, kernel, nu, rho, noise):
    X, Y, _ = synth.small(n, 1, d, ell=ell, seed=91 + k)
    model, X64, Y64 = build(prec, X, Y, k, kernel, nu, 1.0, 1e-2)
    rows = np.random.default_rng(k).choice(n, 300, replace=False).astype(np.int32)
    rows[:2] = [0, n - 1]
    q, g = model.loo_loss_grad(torch.from_numpy(rows).cuda(), kernel, nu, rho, noise)
    model.free()
    ref_q, ref_g, _, st = oracle.loo_loss_grad(X64, Y64, rows, k, kernel, nu, rho, noise)
    assert np.all(st == 0)
    check(q, g, ref_q, ref_g, rho, noise)


def test_fp64_loss_equals_the_loss_entry_point():
    X, Y, _ = synth.small(2500, 1, 4, ell=3, seed=95)
    model, _, _ = build("fp64", X, Y, 30, "matern", 1.5, 1.0, 1e-2)
    rows = torch.arange(0, 2500, 7, dtype=torch.int32, device="cuda")
    for rho in (0.4, 1.3):
        q, _ = model.loo_loss_grad(rows, "matern", 1.5, rho, 2e-2)
        assert abs(q - model.loo_loss(rows, "matern", 1.5, rho, 2e-2)) <= 1e-12 * q
    model.free()


def test_single_row_and_duplicate_rows():
    X, Y, _ = synth.small(700, 1, 3, ell=2, seed=96)
    model, X64, Y64 = build("fp32", X, Y, 16, "matern", 2.5, 1.0, 1e-2)
    for rows in (np.array([5], dtype=np.int32), np.array([3, 3, 3, 699], dtype=np.int32)):
        q, g = model.loo_loss_grad(torch.from_numpy(rows).cuda(), "matern", 2.5, 0.8, 1e-2)
        ref_q, ref_g, _, _ = oracle.loo_loss_grad(X64, Y64, rows, 16, "matern", 2.5, 0.8, 1e-2)
        check(q, g, ref_q, ref_g, 0.8, 1e-2)
    model.free()


def test_cfg2_shaped_model_sampled_rows():
    # the FP32 Fourier workload's shape (n = 100k, d = 8, k = 50), 2048 sampled rows
    w = synth.cfg2(n=100_000, m=1)
    model, X64, Y64 = build("fp32", w.X, w.Y, w.k, w.kernel, w.nu, w.rho, w.noise)
    rows = np.random.default_rng(7).choice(w.X.shape[0], 2048, replace=False).astype(np.int32)
    q, g = model.loo_loss_grad(torch.from_numpy(rows).cuda(), w.kernel, w.nu, w.rho, w.noise)
    model.free()
    ref_q, ref_g, _, _ = oracle.loo_loss_grad(X64, Y64, rows, w.k, w.kernel, w.nu, w.rho,
                                              w.noise)
    check(q, g, ref_q, ref_g, w.rho, w.noise)


def test_fit_reaches_the_oracle_optimum():
    n, k = 3000, 24
    X, Y, _ = synth.small(n, 1, 3, ell=2, seed=97)
    Y = np.sin(3.0 * X[:, :1]) * np.cos(2.0 * X[:, 1:2]) + 0.05 * Y  # smooth signal + noise
    model, X64, Y64 = build("mixed", X, Y, k, "matern", 1.5, 1.0, 1e-2)
    rows = np.random.default_rng(5).choice(n, 256, replace=False).astype(np.int32)
    fit = model.fit_hyper(torch.from_numpy(rows).cuda(), "matern", 1.5, length_scale=3.0,
                          noise_var=0.3)
    model.free()

    def obj(u):
        q, gr, _, _ = oracle.loo_loss_grad(X64, Y64, rows, k, "matern", 1.5, np.exp(u[0]),
                                           np.exp(u[1]))
        return q, np.array([gr[0] * np.exp(u[0]), gr[1] * np.exp(u[1])])

    ref = minimize(obj, np.log([3.0, 0.3]), jac=True, method="L-BFGS-B",
                   bounds=[tuple(np.log((1e-3, 1e3))), tuple(np.log((1e-8, 10.0)))])
    assert fit["success"] and ref.success
    assert fit["loss"] <= 1.0001 * ref.fun
    assert abs(np.log(fit["length_scale"]) - ref.x[0]) <= 1e-2
    assert abs(np.log(fit["noise_var"]) - ref.x[1]) <= 5e-2
    assert fit["loss"] < obj(np.log([3.0, 0.3]))[0]  # it moved downhill


def test_bad_rows_and_self_inclusive_models_are_rejected():
    f = fmg()
    X, Y, _ = synth.small(400, 1, 2, ell=1, seed=98)
    model, _, _ = build("fp32", X, Y, 10, "matern", 1.5, 1.0, 1e-2)
    with pytest.raises(f.FmgError) as e:
        model.loo_loss_grad(torch.tensor([0, 400], dtype=torch.int32, device="cuda"))
    assert e.value.status == f.FMG_E_INVALID_ARG
    with pytest.raises(f.FmgError):
        model.loo_loss_grad(torch.tensor([1], dtype=torch.int32, device="cuda"), "matern", 1.5,
                            -1.0, 1e-2)
    model.free()
    selfm, _, _ = build("fp32", X, Y, 10, "matern", 1.5, 1.0, 1e-2,
                        flags=f.FLAG_SELF_INCLUSIVE)
    with pytest.raises(f.FmgError):
        selfm.loo_loss_grad(torch.tensor([1], dtype=torch.int32, device="cuda"))
    selfm.free()
