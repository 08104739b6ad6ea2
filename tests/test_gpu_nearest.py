"""GPU parity of the exact nearest-point search of FP64 models (the
prediction's lookup, split over candidate chunks and merged) against the
oracle: bit-exact indices for batch sizes around the wave size, on inputs
with many exactly tied distances (integer lattices, where ties must go to
the smaller index across chunks), and for the k = 1 leave-one-out build."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


@pytest.mark.parametrize("dist,n,d", [("grid", 5000, 2), ("normal", 20000, 8), ("grid", 3000, 3),
                                      ("normal", 777, 40)])
def test_nearest_indices_are_exact(dist, n, d):
    X, Y, Z = synth.small(n, 5000, d, ell=1, seed=n + d, dist=dist)
    model = fmg().fastmuygps_build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 4,
                                   "matern", 1.5, 1.0, 1e-2, precision="fp64")
    ref, _ = oracle.nearest(X, Z)
    for m in (1, 2, 63, 64, 65, 1000, 5000):
        nn = torch.empty(m, dtype=torch.int32, device="cuda")
        model.predict(torch.from_numpy(Z[:m]).cuda(), nn_out=nn)
        assert np.array_equal(nn.cpu().numpy(), ref[:m]), (dist, n, d, m)
    model.free()


def test_k1_leave_one_out_build_on_a_lattice():
    X, Y, _ = synth.small(4000, 1, 2, ell=1, seed=3, dist="grid")
    X = np.unique(X, axis=0)  # distinct points: the nearest other point is well defined
    Y = Y[:X.shape[0]]
    model = fmg().fastmuygps_build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 1,
                                   "matern", 0.5, 1.0, 1e-2, precision="fp64")
    N = model.neighbors().cpu().numpy()
    model.free()
    Nr, _, _ = oracle.build_model(X, Y, 1, "matern", 0.5, 1.0, 1e-2)
    assert np.array_equal(N, Nr)
