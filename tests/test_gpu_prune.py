"""GPU check of the build screen's tile pruning (BF16 screen of mixed
precision, FP32 screen of the plain FP32 path): building
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


def build_pair(X, Y, k, kernel="rbf", nu=0.0, rho=3.0, noise=1e-2, prec="mixed"):
    f = fmg()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = []
    for flags in (0, f.FLAG_NO_PRUNE):
        m = f.fastmuygps_build(Xd, Yd, k, kernel, nu, rho, noise, precision=prec, flags=flags)
        out.append((m.neighbors().cpu().numpy(), m.coeffs().cpu().numpy(), m.info()))
        m.free()
    return out


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
@pytest.mark.parametrize("n,d,classes,k,seed", [(60_000, 40, 10, 50, 1), (33_333, 16, 6, 30, 2),
                                                (20_001, 8, 1, 20, 3)])
def test_pruned_build_equals_the_full_screen(n, d, classes, k, seed, prec):
    X, Y = clustered(n, d, classes, seed)
    (Np, Cp, ip), (Nf, Cf, inf) = build_pair(X, Y, k, prec=prec)
    assert np.array_equal(Np, Nf)
    assert np.array_equal(Cp, Cf)
    rows = np.random.default_rng(seed).choice(n, 40, replace=False)
    Nr, _, _ = oracle.build_model(X.astype(np.float64), Y.astype(np.float64), k, "rbf", 0.0, 3.0,
                                  1e-2, rows=rows)
    assert np.array_equal(Np[rows], Nr)


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_low_dimensional_uniform_build(prec):
    # d = 3 uniform points (the shape of the five-million-point model of the
    # multi-model serving workload): tiles in pivot order are compact and
    # most are skipped; a ragged last tile
    rs = np.random.default_rng(21)
    X = rs.random((50_003, 3)).astype(np.float32)
    Y = np.sin(6.0 * X[:, :1]).astype(np.float32)
    (Np, Cp, _), (Nf, Cf, _) = build_pair(X, Y, 30, kernel="matern", nu=0.5, rho=0.2,
                                           noise=4e-4, prec=prec)
    assert np.array_equal(Np, Nf)
    assert np.array_equal(Cp, Cf)
    rows = rs.choice(X.shape[0], 40, replace=False)
    Nr, _, _ = oracle.build_model(X.astype(np.float64), Y.astype(np.float64), 30, "matern", 0.5,
                                  0.2, 4e-4, rows=rows)
    assert np.array_equal(Np[rows], Nr)


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_pruned_build_with_duplicates_and_self_inclusive_sets(prec):
    f = fmg()
    X, Y = clustered(12_000, 12, 4, 7)
    X = np.concatenate([X, X[:3000]])  # 3,000 exact duplicates
    Y = np.concatenate([Y, Y[:3000]])
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    got = []
    for flags in (f.FLAG_SELF_INCLUSIVE, f.FLAG_SELF_INCLUSIVE | f.FLAG_NO_PRUNE):
        m = f.fastmuygps_build(Xd, Yd, 24, "matern", 1.5, 2.0, 1e-2, precision=prec,
                               flags=flags)
        got.append(m.neighbors().cpu().numpy())
        m.free()
    assert np.array_equal(got[0], got[1])
    rows = np.array([0, 1, 2999, 3000, 12_000, 14_999])
    Nr, _, _ = oracle.build_model(X.astype(np.float64), Y.astype(np.float64), 24, "matern", 1.5,
                                  2.0, 1e-2, 1.0, oracle.MODE_SELF, rows=rows)
    assert np.array_equal(got[0][rows], Nr)


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_pruned_prediction_equals_chunked_unpruned_prediction(prec):
    # 70,000 queries in one call take the pruned screen (queries sorted by
    # nearest pivot); chunks of 20,000 take the full screen
    f = fmg()
    X, Y = clustered(50_000, 24, 8, 11)
    Z, _ = clustered(70_000, 24, 8, 11)  # same cluster means (same seed), fresh points
    Z = Z + np.float32(0.01)
    m = f.fastmuygps_build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 30, "rbf",
                           0.0, 3.0, 1e-2, precision=prec)
    Zd = torch.from_numpy(Z).cuda()
    nn_all = torch.empty(70_000, dtype=torch.int32, device="cuda")
    mu_all = m.predict(Zd, nn_out=nn_all).cpu().numpy()
    parts_nn, parts_mu = [], []
    for lo in range(0, 70_000, 20_000):
        nn = torch.empty(min(20_000, 70_000 - lo), dtype=torch.int32, device="cuda")
        parts_mu.append(m.predict(Zd[lo:lo + 20_000], nn_out=nn).cpu().numpy())
        parts_nn.append(nn.cpu().numpy())
    m.free()
    assert np.array_equal(nn_all.cpu().numpy(), np.concatenate(parts_nn))
    assert np.array_equal(mu_all, np.concatenate(parts_mu))
    take = np.random.default_rng(4).choice(70_000, 300, replace=False)
    ref, _ = oracle.nearest(X.astype(np.float64), Z[take].astype(np.float64))
    assert np.array_equal(nn_all.cpu().numpy()[take], ref)
