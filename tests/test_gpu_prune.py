"""GPU check of the build screen's tile pruning (mixed precision): building
with the training points ordered by nearest pivot and skipping the tiles no
query of a wavefront can take gives bit-identical neighbour lists and
coefficients to screening every tile (FMG_FLAG_NO_PRUNE), on clustered data
where most tiles are skipped, on unclustered data, with duplicates and with
a ragged last tile; and the lists equal the oracle's on sampled rows."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


def clustered(n, d, classes, seed, spread=2.0):
    rs = np.random.default_rng(seed)
    means = rs.normal(0.0, spread, size=(classes, d))
    lab = rs.integers(0, classes, size=n)
    X = (means[lab] + rs.normal(size=(n, d))).astype(np.float32)
    Y = np.full((n, 3), -0.5, dtype=np.float32)
    Y[np.arange(n), lab % 3] = 0.5
    return X, Y


def build_pair(X, Y, k, kernel="rbf", nu=0.0, rho=3.0, noise=1e-2):
    f = fmg()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = []
    for flags in (0, f.FLAG_NO_PRUNE):
        m = f.fastmuygps_build(Xd, Yd, k, kernel, nu, rho, noise, precision="mixed", flags=flags)
        out.append((m.neighbors().cpu().numpy(), m.coeffs().cpu().numpy(), m.info()))
        m.free()
    return out


@pytest.mark.parametrize("n,d,classes,k,seed", [(60_000, 40, 10, 50, 1), (33_333, 16, 6, 30, 2),
                                                (20_001, 8, 1, 20, 3)])
def test_pruned_build_equals_the_full_screen(n, d, classes, k, seed):
    X, Y = clustered(n, d, classes, seed)
    (Np, Cp, ip), (Nf, Cf, inf) = build_pair(X, Y, k)
    assert np.array_equal(Np, Nf)
    assert np.array_equal(Cp, Cf)
    rows = np.random.default_rng(seed).choice(n, 40, replace=False)
    Nr, _, _ = oracle.build_model(X.astype(np.float64), Y.astype(np.float64), k, "rbf", 0.0, 3.0,
                                  1e-2, rows=rows)
    assert np.array_equal(Np[rows], Nr)


def test_pruned_build_with_duplicates_and_self_inclusive_sets():
    f = fmg()
    X, Y = clustered(12_000, 12, 4, 7)
    X = np.concatenate([X, X[:3000]])  # 3,000 exact duplicates
    Y = np.concatenate([Y, Y[:3000]])
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    got = []
    for flags in (f.FLAG_SELF_INCLUSIVE, f.FLAG_SELF_INCLUSIVE | f.FLAG_NO_PRUNE):
        m = f.fastmuygps_build(Xd, Yd, 24, "matern", 1.5, 2.0, 1e-2, precision="mixed",
                               flags=flags)
        got.append(m.neighbors().cpu().numpy())
        m.free()
    assert np.array_equal(got[0], got[1])
    rows = np.array([0, 1, 2999, 3000, 12_000, 14_999])
    Nr, _, _ = oracle.build_model(X.astype(np.float64), Y.astype(np.float64), 24, "matern", 1.5,
                                  2.0, 1e-2, 1.0, oracle.MODE_SELF, rows=rows)
    assert np.array_equal(got[0][rows], Nr)
