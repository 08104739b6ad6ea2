"""GPU parity of the FP32 and mixed coefficient precompute over every
neighbourhood size class of its register-window Cholesky: k at, just below and
just above each 16-column window boundary and each multiple of four (the
factorisation runs four steps at a time, then single steps), with right-hand
side counts from every register-array width (ell = 1, 3, 5, 12, 16).  Each
case builds a model through the C ABI and compares neighbours, coefficients
(backward error) and means with the FP64 oracle."""
import numpy as np
import pytest

import synth
from tests.test_gpu_small import check_against_oracle, run

pytestmark = pytest.mark.gpu

CASES = [(3, 1), (4, 3), (5, 5), (7, 12), (8, 16), (9, 1), (15, 3), (16, 5), (19, 12),
         (31, 16), (32, 1), (33, 3), (36, 5), (47, 12), (48, 16), (49, 1), (52, 3), (61, 5),
         (63, 12), (64, 16)]


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("k,ell", CASES)
def test_precompute_window_classes(prec, k, ell):
    n = 260 + 3 * k
    X, Y, Z = synth.small(n, 40, 3, ell=ell, seed=1000 + 17 * k + ell, dist="normal")
    # rho keeps kappa moderate at every k (plain FP32 error ~ kappa * u_32)
    X, Y, Z, out = run(prec, X, Y, Z, k, "matern", 2.5, 0.6, 5e-2)
    assert out["info"]["nonpd_rows"] == 0
    check_against_oracle(prec, X, Y, Z, k, "matern", 2.5, 0.6, 5e-2, out)


@pytest.mark.parametrize("k", [4, 33, 50])
def test_precompute_rbf_mixed(k):
    # RBF takes no square roots in the assembly or the FP64 residual
    X, Y, Z = synth.small(400, 60, 5, ell=4, seed=77 + k, dist="normal")
    X, Y, Z, out = run("mixed", X, Y, Z, k, "rbf", 0.0, 1.5, 5e-2)
    check_against_oracle("mixed", X, Y, Z, k, "rbf", 0.0, 1.5, 5e-2, out)
