"""The allocation-free prediction (fastmuygps_predict_noalloc) against the
allocating one (fastmuygps_predict) through the C ABI: nearest points and
means bit-identical on two calls in a row, the second with a smaller batch
(the static scratch keeps the first call's contents), in every precision,
plus the batch limit and the oracle on the same queries."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity_util import TOL_MEAN, rel_err

pytestmark = pytest.mark.gpu

DT = {"fp64": (np.float64, torch.float64), "fp32": (np.float32, torch.float32),
      "mixed": (np.float32, torch.float32)}


def fmg():
    import paper_2205_10879_amd as f
    return f


def call_noalloc(f, model, Zd, out, nn):
    st = f.lib().fastmuygps_predict_noalloc(model.handle, ctypes.c_void_p(Zd.data_ptr()),
                                            Zd.shape[0], ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(nn.data_ptr()), None)
    return st


@pytest.mark.parametrize("prec", ["fp64", "fp32", "mixed"])
def test_noalloc_matches_predict_on_two_calls(prec):
    f = fmg()
    npdt, tdt = DT[prec]
    n, d, ell, k = 6000, 5, 3, 24
    X, Y, Z = synth.small(n, f.NOALLOC_MAX_M, d, ell=ell, seed=71, dist="normal")
    X, Y, Z = (np.ascontiguousarray(a, dtype=npdt) for a in (X, Y, Z))
    Xd, Yd, Zd = (torch.from_numpy(a).cuda() for a in (X, Y, Z))
    model = f.fastmuygps_build(Xd, Yd, k, "matern", 2.5, 0.8, 1e-2, precision=prec)
    sizes = (f.NOALLOC_MAX_M, 777)  # the full limit, then a smaller ragged batch
    refs = []
    for m in sizes:
        nn_r = torch.empty(m, dtype=torch.int32, device="cuda")
        mu_r = model.predict(Zd[:m], nn_out=nn_r)
        refs.append((mu_r, nn_r))
    outs = [(torch.full((m, ell), float("nan"), dtype=tdt, device="cuda"),
             torch.full((m,), -1, dtype=torch.int32, device="cuda")) for m in sizes]
    torch.cuda.synchronize()
    # The runtime places the static scratch array on the device when the
    # first call looks up its address; later calls take no device memory.
    free = []
    for m, (mu, nn) in zip(sizes, outs):
        assert call_noalloc(f, model, Zd[:m], mu, nn) == f.FMG_OK, f.lib().fastmuygps_last_error()
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
    assert free[1] >= free[0], "device memory was allocated by the second call"
    for m, (mu, nn), (mu_r, nn_r) in zip(sizes, outs, refs):
        assert torch.equal(nn, nn_r), "nearest points differ at m=%d" % m
        assert torch.equal(mu, mu_r), "means differ at m=%d" % m
    # the same queries against the oracle (the smaller batch)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    mu_o, nn_o, _ = oracle.predict(X64, Y64, Z[:sizes[1]].astype(np.float64), k, "matern", 2.5,
                                   0.8, 1e-2)
    assert np.array_equal(outs[1][1].cpu().numpy(), nn_o)
    assert rel_err(outs[1][0].cpu().numpy(), mu_o) <= TOL_MEAN[prec]
    model.free()


def test_noalloc_limits():
    f = fmg()
    X, Y, Z = synth.small(500, f.NOALLOC_MAX_M + 1, 3, seed=5, dist="uniform")
    X, Y, Z = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda() for a in (X, Y, Z))
    model = f.fastmuygps_build(X, Y, 10, "rbf", 0.0, 0.5, 1e-3, precision="mixed")
    out = torch.empty((Z.shape[0], 1), dtype=torch.float32, device="cuda")
    nn = torch.empty(Z.shape[0], dtype=torch.int32, device="cuda")
    assert call_noalloc(f, model, Z, out, nn) == f.FMG_E_INVALID_ARG
    assert b"allocation-free limit" in f.lib().fastmuygps_last_error()
    # m = 0 is a no-op; one query works and equals the allocating call
    assert call_noalloc(f, model, Z[:0], out, nn) == f.FMG_OK
    one = torch.empty((1, 1), dtype=torch.float32, device="cuda")
    nn1 = torch.empty(1, dtype=torch.int32, device="cuda")
    assert call_noalloc(f, model, Z[5:6], one, nn1) == f.FMG_OK
    ref_nn = torch.empty(1, dtype=torch.int32, device="cuda")
    ref = model.predict(Z[5:6], nn_out=ref_nn)
    torch.cuda.synchronize()
    assert torch.equal(one, ref) and torch.equal(nn1, ref_nn)
    assert 0 < f.noalloc_scratch_bytes() <= 128 << 20
    model.free()
