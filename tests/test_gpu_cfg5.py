"""GPU parity of the multi-model serving workload's models: model A (the
5,000,000-point, 3-D, Matern 1/2, FP32 model) at full size against the
sampled FP64 oracle (neighbour lists and nearest points bit for bit, means
within the FP32 tolerance), and its served results, in a server that swaps
it with a model of another kind (FP64, 2-D) under a budget for one of them,
bit-identical to direct prediction."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity_util import TOL_MEAN, TOL_RMSE, rel_err, rmse

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


def build(w):
    f = fmg()
    dt = torch.float64 if w.precision == "fp64" else torch.float32
    X = torch.from_numpy(w.X).to("cuda", dt)
    Y = torch.from_numpy(w.Y).to("cuda", dt)
    m = f.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision=w.precision)
    torch.cuda.synchronize()
    return m


@pytest.mark.timeout(600)
def test_model_a_full_size_sampled_oracle_and_served():
    f = fmg()
    wa = synth.cfg5a(m=4096)
    ma = build(wa)
    assert ma.info()["nonpd_rows"] == 0
    rs = synth.rng(5, 4)
    rows = np.sort(rs.choice(wa.X.shape[0], 128, replace=False))
    X64, Y64 = wa.X.astype(np.float64), wa.Y.astype(np.float64)
    N_o, _, st = oracle.build_model(X64, Y64, wa.k, wa.kernel, wa.nu, wa.rho, wa.noise, rows=rows)
    assert np.all(st == 0)
    assert np.array_equal(ma.neighbors().cpu().numpy()[rows], N_o)
    qs = np.sort(rs.choice(wa.Z.shape[0], 256, replace=False))
    Zd = torch.from_numpy(wa.Z).cuda()
    nn = torch.empty(len(qs), dtype=torch.int32, device="cuda")
    mu = ma.predict(Zd[torch.from_numpy(qs).cuda()], nn_out=nn).cpu().numpy()
    mu_o, nn_o, _ = oracle.predict(X64, Y64, wa.Z[qs].astype(np.float64), wa.k, wa.kernel, wa.nu,
                                   wa.rho, wa.noise)
    assert np.array_equal(nn.cpu().numpy(), nn_o)
    assert rel_err(mu, mu_o) <= TOL_MEAN["fp32"]
    assert abs(rmse(mu, wa.Yz[qs]) / rmse(mu_o, wa.Yz[qs]) - 1.0) <= TOL_RMSE

    # a 2-D FP64 model of the same workload (cfg-1 kind, its own seed stream)
    wb = synth.cfg1(n=24_231, m=2048, cfg=53)
    wb.k = 50
    mb = build(wb)
    ref_a = ma.predict(Zd).cpu().numpy()
    ref_b = mb.predict(torch.from_numpy(wb.Z).cuda()).cpu().numpy()
    fa, fb = ma.info()["device_bytes"], mb.info()["device_bytes"]
    with f.Server(slots=2, max_batch=8192) as probe:
        ws = probe.stats()["hbm_resident"]
    with f.Server(hbm_budget=ws + max(fa, fb) + min(fa, fb) // 2, slots=2, max_batch=8192,
                  swap_idle=True) as srv:
        ida, adm_a = srv.add_model(ma)
        idb, adm_b = srv.add_model(mb)
        assert adm_a and not adm_b
        sizes = np.floor(np.exp(np.random.default_rng(3).uniform(0, np.log(8193), 12))).astype(int)
        got = []
        for i, b in enumerate(sizes):
            if i % 2 == 0:
                o = int(b) % 97
                got.append(("a", o, int(b), srv.submit(ida, wa.Z[o:o + int(b)]).wait()[0]))
            else:
                o = int(b) % 89
                b = min(int(b), 2048 - o)
                got.append(("b", o, b, srv.submit(idb, wb.Z[o:o + b]).wait()[0]))
        st = srv.stats()
    for key, o, b, out in got:
        ref = ref_a if key == "a" else ref_b
        assert np.array_equal(out, ref[o:o + b]), (key, o, b)
    assert st["swaps"] >= 2
    ma.free()
    mb.free()
