"""Calls on two streams.  A call's device scratch goes back to the library's
cache when the call returns, tagged with the call's stream and an event; a
later call on the same stream takes it at once, a call on another stream only
once the event has completed (else it allocates).  Builds and predictions
issued on two streams, with no synchronisation between the streams, several
times over and with back-to-back predictions on one stream, must give results
bit-identical to the same calls on the default stream."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def fmg():
    import paper_2205_10879_amd as f
    return f


def workload(n, m, d, classes, seed):
    rs = np.random.default_rng(seed)
    means = rs.normal(0.0, 2.0, size=(classes, d))
    lab = rs.integers(0, classes, size=n + m)
    X = (means[lab] + rs.normal(size=(n + m, d))).astype(np.float32)
    Y = np.full((n + m, 3), -0.5, dtype=np.float32)
    Y[np.arange(n + m), lab % 3] = 0.5
    return X[:n], Y[:n], X[n:]


@pytest.mark.parametrize("prec", ["mixed", "fp32"])
def test_two_streams_equal_the_default_stream(prec):
    f = fmg()
    X, Y, Z = workload(40_000, 6_000, 24, 6, seed=17)
    Xd, Yd, Zd = (torch.from_numpy(a).cuda() for a in (X, Y, Z))
    torch.cuda.synchronize()
    k = 30

    m = f.fastmuygps_build(Xd, Yd, k, "rbf", 0.0, 3.0, 1e-2, precision=prec)
    ref_mu = m.predict(Zd).cpu().numpy()
    ref_N = m.neighbors().cpu().numpy()
    ref_C = m.coeffs().cpu().numpy()
    torch.cuda.synchronize()
    m.free()

    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    for rnd in range(3):
        print("round", rnd, prec, flush=True)
        ma = f.fastmuygps_build(Xd, Yd, k, "rbf", 0.0, 3.0, 1e-2, precision=prec, stream=sa)
        mb = f.fastmuygps_build(Xd, Yd, k, "rbf", 0.0, 3.0, 1e-2, precision=prec, stream=sb)
        outs = [torch.empty((Z.shape[0], 3), dtype=torch.float32, device="cuda")
                for _ in range(4)]
        torch.cuda.synchronize()
        # back to back on each stream (the second call takes the first's
        # scratch at once), the two streams interleaved
        ma.predict(Zd, out=outs[0], stream=sa)
        mb.predict(Zd, out=outs[1], stream=sb)
        ma.predict(Zd[:4_000], out=outs[2][:4_000], stream=sa)
        mb.predict(Zd, out=outs[3], stream=sb)
        Na, Ca = ma.neighbors(stream=sa), ma.coeffs(stream=sa)
        Nb, Cb = mb.neighbors(stream=sb), mb.coeffs(stream=sb)
        torch.cuda.synchronize()
        for o in (outs[0], outs[1], outs[3]):
            assert np.array_equal(o.cpu().numpy(), ref_mu)
        assert np.array_equal(outs[2][:4_000].cpu().numpy(), ref_mu[:4_000])
        for N_, C_ in ((Na, Ca), (Nb, Cb)):
            assert np.array_equal(N_.cpu().numpy(), ref_N)
            assert np.array_equal(C_.cpu().numpy(), ref_C)
        ma.free()
        mb.free()
