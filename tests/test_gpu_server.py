"""GPU tests of the request server (continuous batching over resident models):
every request's result is the same alone and in a mix of concurrent requests
of uneven size (and equal to fastmuygps_predict of the same queries), with
and without graph replay; admission by HBM budget queues a model until
another is removed; the oracle agrees on a sample of served queries."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.parity_util import TOL_MEAN, rel_err

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


def build(prec, n, m, d, ell, k, seed, rho=1.0, noise=1e-2):
    f = fmg()
    npdt = np.float64 if prec == "fp64" else np.float32
    X, Y, Z = synth.small(n, m, d, ell=ell, seed=seed, dtype=npdt)
    model = f.fastmuygps_build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), k,
                               "matern", 1.5, rho, noise, precision=prec)
    return model, X, Y, Z


def direct(model, Z):
    out = model.predict(torch.from_numpy(Z).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def batch_sizes(total, seed, hi=700):
    rs = np.random.default_rng(seed)
    sizes = []
    while sum(sizes) < total:
        sizes.append(int(np.exp(rs.uniform(0.0, np.log(hi)))) + 1)
    return sizes


@pytest.mark.parametrize("use_graphs", [True, False])
def test_alone_and_in_the_mix(use_graphs):
    f = fmg()
    mixed, Xa, Ya, Za = build("mixed", 6000, 3000, 8, 3, 30, seed=11)
    plain, Xb, Yb, Zb = build("fp32", 4000, 2000, 5, 2, 20, seed=12)
    f64, Xc, Yc, Zc = build("fp64", 1500, 800, 3, 1, 16, seed=13)
    refs = {"a": direct(mixed, Za), "b": direct(plain, Zb), "c": direct(f64, Zc)}
    # These queries certify on the first screen: direct prediction needs no
    # exact rescan.  Served batches must not need one either (the padding of
    # a replayed bucket must not turn into invalid queries after batches of
    # another model, e.g. FP64 bytes left in the staging rows read as FP32).
    fb0 = {key: m.info()["predict_fallback_rows"] for key, m in
           (("a", mixed), ("b", plain), ("c", f64))}
    assert fb0 == {"a": 0, "b": 0, "c": 0}
    with f.Server(slots=3, max_batch=2048, use_graphs=use_graphs) as srv:
        ids = {"a": srv.add_model(mixed), "b": srv.add_model(plain), "c": srv.add_model(f64)}
        assert all(adm for _, adm in ids.values())
        Zs = {"a": Za, "b": Zb, "c": Zc}
        # requests: uneven slices of each model's queries
        reqs = []
        for key, seed in (("a", 1), ("b", 2), ("c", 3)):
            lo = 0
            for B in batch_sizes(len(Zs[key]), seed):
                hi = min(lo + B, len(Zs[key]))
                if hi > lo:
                    reqs.append((key, lo, hi))
                lo = hi
        # alone: one request at a time
        alone = {}
        for key, lo, hi in reqs:
            out, lat = srv.submit(ids[key][0], Zs[key][lo:hi]).wait()
            alone[(key, lo)] = out.copy()
            assert lat >= 0.0
        # in the mix: every request in flight at once, interleaved over models
        order = np.random.default_rng(5).permutation(len(reqs))
        tickets = [(reqs[i], srv.submit(ids[reqs[i][0]][0], Zs[reqs[i][0]][reqs[i][1]:reqs[i][2]]))
                   for i in order]
        mix = {}
        for (key, lo, hi), t in tickets:
            mix[(key, lo)] = t.wait()[0]
        st = srv.stats()
    for key, lo, hi in reqs:
        a, m = alone[(key, lo)], mix[(key, lo)]
        assert np.array_equal(a, m), (key, lo, hi)
        assert np.array_equal(a, refs[key][lo:hi]), (key, lo, hi)
    assert st["requests"] == 2 * len(reqs)
    assert st["queries"] == 2 * sum(hi - lo for _, lo, hi in reqs)
    assert st["batches"] < st["requests"]  # the mix was coalesced
    assert 0.0 <= st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    for key, m in (("a", mixed), ("b", plain), ("c", f64)):
        assert m.info()["predict_fallback_rows"] == 0, key
    for m in (mixed, plain, f64):
        m.free()


def test_served_means_match_the_oracle():
    f = fmg()
    k, rho, noise = 30, 1.0, 1e-2
    model, X, Y, Z = build("mixed", 5000, 400, 6, 2, k, seed=21, rho=rho, noise=noise)
    with f.Server(slots=2, max_batch=1024) as srv:
        mid, _ = srv.add_model(model)
        ts = [srv.submit(mid, Z[i:i + 37]) for i in range(0, len(Z), 37)]
        mu = np.concatenate([t.wait()[0] for t in ts])
    X64, Y64, Z64 = (a.astype(np.float64) for a in (X, Y, Z))
    ref, nn, _ = oracle.predict(X64, Y64, Z64, k, "matern", 1.5, rho, noise, 1.0,
                                oracle.MODE_LOO, model=None)
    assert rel_err(mu, ref) <= TOL_MEAN["mixed"]
    model.free()


def test_admission_by_budget_queues_then_admits():
    f = fmg()
    m1, X1, Y1, Z1 = build("fp32", 20000, 500, 8, 4, 40, seed=31)
    m2, X2, Y2, Z2 = build("fp32", 16000, 500, 8, 4, 40, seed=32)
    ref2 = direct(m2, Z2)
    fp1 = m1.info()["device_bytes"]
    fp2 = m2.info()["device_bytes"]
    with f.Server(slots=1, max_batch=1024) as probe:
        ws = probe.stats()["hbm_resident"]
    budget = ws + max(fp1, fp2) + min(fp1, fp2) // 2  # one model fits, not both
    with f.Server(hbm_budget=budget, slots=1, max_batch=1024) as srv:
        id1, adm1 = srv.add_model(m1)
        id2, adm2 = srv.add_model(m2)
        assert adm1 and not adm2
        st = srv.stats()
        assert st["models_resident"] == 1 and st["models_waiting"] == 1
        # an offloaded model cannot be used directly
        with pytest.raises(f.FmgError) as e:
            m2.predict(torch.from_numpy(Z2).cuda())
        assert e.value.status == f.FMG_E_BUSY
        t2 = srv.submit(id2, Z2)  # waits for admission
        out1, _ = srv.submit(id1, Z1).wait()
        assert np.array_equal(out1, direct(m1, Z1))
        srv.remove_model(id1)  # frees the budget: model 2 is admitted
        out2, _ = t2.wait()
        assert np.array_equal(out2, ref2)
        st = srv.stats()
        assert st["models_resident"] == 1 and st["models_waiting"] == 0
        assert st["hbm_peak"] <= budget
    # model 2 is back on the device for its owner
    assert np.array_equal(direct(m2, Z2), ref2)
    m1.free()
    m2.free()


def test_destroy_fails_requests_of_models_never_admitted():
    f = fmg()
    m1, _, _, Z1 = build("fp32", 12000, 100, 8, 2, 30, seed=41)
    m2, _, _, Z2 = build("fp32", 12000, 100, 8, 2, 30, seed=42)
    with f.Server(slots=1, max_batch=512) as probe:
        ws = probe.stats()["hbm_resident"]
    fp = max(m1.info()["device_bytes"], m2.info()["device_bytes"])
    srv = f.Server(hbm_budget=ws + fp + fp // 4, slots=1, max_batch=512)
    id1, _ = srv.add_model(m1)
    id2, adm2 = srv.add_model(m2)
    assert not adm2
    t = srv.submit(id2, Z2)
    srv.close()
    with pytest.raises(f.FmgError) as e:
        t.wait()
    assert e.value.status == f.FMG_E_BUSY
    ref = direct(m2, Z2)  # restored for its owner
    assert ref.shape == (len(Z2), 2)
    m1.free()
    m2.free()


@pytest.mark.parametrize("use_graphs", [True, False])
def test_swapping_idle_models_serves_every_stream(use_graphs):
    # Three models, a budget for two: with swap_idle, requests for the model
    # that waits in host memory bring it in for an idle one (least recently
    # used), and every result still equals direct prediction.
    f = fmg()
    ma, Xa, Ya, Za = build("mixed", 9000, 1500, 12, 3, 30, seed=51)
    mb, Xb, Yb, Zb = build("fp32", 8000, 1500, 8, 2, 25, seed=52)
    mc, Xc, Yc, Zc = build("fp64", 3000, 1200, 2, 1, 20, seed=53)
    models = {"a": ma, "b": mb, "c": mc}
    Zs = {"a": Za, "b": Zb, "c": Zc}
    refs = {key: direct(m, Zs[key]) for key, m in models.items()}
    fps = sorted(m.info()["device_bytes"] for m in models.values())
    with f.Server(slots=2, max_batch=1024) as probe:
        ws = probe.stats()["hbm_resident"]
    budget = ws + fps[2] + fps[1] + fps[0] // 2  # any two fit, not all three
    with f.Server(hbm_budget=budget, slots=2, max_batch=1024, use_graphs=use_graphs,
                  swap_idle=True) as srv:
        ids = {key: srv.add_model(m) for key, m in models.items()}
        assert sum(adm for _, adm in ids.values()) == 2
        results = {key: [] for key in models}
        # rounds of requests, each round to one model at a time, so that the
        # others turn idle and can be swapped out
        rs = np.random.default_rng(7)
        for rnd in range(6):
            for key in ("c", "a", "b") if rnd % 2 else ("a", "b", "c"):
                Z = Zs[key]
                lo = int(rs.integers(0, len(Z) - 300))
                hi = lo + int(rs.integers(1, 300))
                ts = [srv.submit(ids[key][0], Z[lo:hi]), srv.submit(ids[key][0], Z[:17])]
                outs = [t.wait()[0] for t in ts]
                results[key].append((lo, hi, outs))
        st = srv.stats()
    for key, lst in results.items():
        for lo, hi, (o1, o2) in lst:
            assert np.array_equal(o1, refs[key][lo:hi]), key
            assert np.array_equal(o2, refs[key][:17]), key
    assert st["swaps"] >= 2
    assert st["hbm_peak"] <= budget
    assert st["requests"] == 36
    # every model is back on the device for its owner
    for key, m in models.items():
        assert np.array_equal(direct(m, Zs[key]), refs[key])
        m.free()


def test_requests_larger_than_a_batch_are_split():
    # A request of more than max_batch queries is served as parts of at most
    # max_batch; the whole request completes once, with every query's mean
    # equal to direct prediction, and counts as one request.
    f = fmg()
    model, X, Y, Z = build("mixed", 6000, 5000, 8, 3, 30, seed=21)
    ref = direct(model, Z)
    with f.Server(slots=3, max_batch=1024, use_graphs=True) as srv:
        mid, adm = srv.add_model(model)
        assert adm
        big = srv.submit(mid, Z[:2600])           # three parts: 1024 + 1024 + 552
        small = srv.submit(mid, Z[2600:2700])     # queued behind it
        exact = srv.submit(mid, Z[2700:4748])     # exactly two full parts
        out_b, lat_b = big.wait()
        out_s, _ = small.wait()
        out_e, _ = exact.wait()
        st = srv.stats()
    assert np.array_equal(out_b, ref[:2600])
    assert np.array_equal(out_s, ref[2600:2700])
    assert np.array_equal(out_e, ref[2700:4748])
    assert lat_b > 0.0
    assert st["requests"] == 3
    assert st["queries"] == 2600 + 100 + 2048
    assert st["batches"] >= 5
    model.free()
