"""Model checkpoints: a model written by fastmuygps_save and read back by
fastmuygps_load predicts bitwise identically to the model it was saved from,
with the same neighbour lists, coefficients and parameters, in every
precision and with the pruned screen's structures; damaged files are
rejected with FMG_E_IO and leave no model behind."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


def clustered(n, m, d, classes, seed):
    rs = np.random.default_rng(seed)
    means = rs.normal(0.0, 2.0, size=(classes, d))
    lab = rs.integers(0, classes, size=n + m)
    X = (means[lab] + rs.normal(size=(n + m, d))).astype(np.float32)
    Y = np.full((n + m, 3), -0.5, dtype=np.float32)
    Y[np.arange(n + m), lab % 3] = 0.5
    return X[:n], Y[:n], X[n:]


CASES = [
    # precision, kernel, nu, k, data
    ("mixed", "rbf", 0.0, 30, "clustered"),
    ("fp32", "matern", 2.5, 20, "clustered"),
    ("fp64", "matern", 1.5, 16, "small"),
]


@pytest.mark.parametrize("prec,kernel,nu,k,data", CASES)
def test_saved_model_predicts_bitwise_identically(prec, kernel, nu, k, data, tmp_path):
    f = fmg()
    if data == "clustered":
        X, Y, Z = clustered(30_000, 70_000, 16, 5, seed=41)
    else:
        X, Y, Z = synth.small(3000, 500, 3, ell=2, seed=42)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd, Yd, Zd = (torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda() for a in (X, Y, Z))
    m = f.fastmuygps_build(Xd, Yd, k, kernel, nu, 2.0, 1e-2, precision=prec)
    path = str(tmp_path / ("model_%s.fmg" % prec))
    m.save(path)
    loaded = f.fastmuygps_load(path)
    assert (loaded.n, loaded.d, loaded.k, loaded.ell, loaded.dtype) == (m.n, m.d, m.k, m.ell,
                                                                       m.dtype)
    a, b = m.info(), loaded.info()
    for key in ("n", "d", "ell", "k", "precision", "screen_cands", "query_cands", "nonpd_rows",
                "build_fallback_rows"):
        assert a[key] == b[key], key
    assert 0 < b["device_bytes"] <= a["device_bytes"]
    assert b["predict_fallback_rows"] == 0
    assert torch.equal(m.neighbors(), loaded.neighbors())
    assert torch.equal(m.coeffs(), loaded.coeffs())
    # a large batch (the pruned screen in query order where the model has one)
    # and a small one (the split screen)
    for Zq in (Zd, Zd[:700]):
        nn_a = torch.empty(Zq.shape[0], dtype=torch.int32, device="cuda")
        nn_b = torch.empty_like(nn_a)
        mu_a = m.predict(Zq, nn_out=nn_a)
        mu_b = loaded.predict(Zq, nn_out=nn_b)
        torch.cuda.synchronize()
        assert torch.equal(nn_a, nn_b)
        assert torch.equal(mu_a, mu_b)
    # the original is untouched by the save, the copy independent of it
    m.free()
    mu_c = loaded.predict(Zd[:700])
    torch.cuda.synchronize()
    assert torch.isfinite(mu_c).all()
    loaded.free()


def test_damaged_files_are_rejected(tmp_path):
    f = fmg()
    X, Y, Z = synth.small(2000, 100, 4, ell=1, seed=43)
    Xd, Yd = (torch.from_numpy(np.ascontiguousarray(a)).float().cuda() for a in (X, Y))
    m = f.fastmuygps_build(Xd, Yd, 12, "rbf", 0.0, 1.0, 1e-2, precision="mixed")
    path = tmp_path / "model.fmg"
    m.save(str(path))
    m.free()
    blob = path.read_bytes()
    h = ctypes.c_void_p()
    for name, data in (("truncated", blob[:-17]), ("header only", blob[:60]),
                       ("trailing", blob + b"\0"), ("bad tag", b"X" + blob[1:])):
        p = tmp_path / name.replace(" ", "_")
        p.write_bytes(data)
        st = f.lib().fastmuygps_load(str(p).encode(), ctypes.byref(h))
        assert st == f.FMG_E_IO, name
        assert not h.value, name
    good = f.fastmuygps_load(str(path))
    good.free()
