"""The FP64 exponential of the mixed-precision refinement (exp of x <= 0 by
Cody-Waite range reduction and a degree-12 Taylor series) against the host's
exp over its whole domain [-745, 0]: a few units in the last place where the
result is normal, a few units of the smallest subnormal below that, exact at
0, and 0 past the underflow threshold.  Also the FP32 exponential of the
FP32 kernel values (two-part x log2(e), hardware 2^f, scaling by 2^n)
against the FP64 host exp: at most two units in the last place where the
float result is normal, within the smallest normal float below that."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def dev_exp(x):
    import paper_2205_10879_amd as f
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()
    yd = torch.empty_like(xd)
    st = f.lib().fastmuygps_debug_exp_nonpos(ctypes.c_void_p(xd.data_ptr()),
                                             ctypes.c_void_p(yd.data_ptr()), xd.numel(), None)
    assert st == f.FMG_OK
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def test_exp_nonpos64_accuracy():
    rs = np.random.default_rng(11)
    ln2 = np.log(2.0)
    x = np.concatenate([
        -np.linspace(0.0, 745.0, 400_001),
        -np.exp(rs.uniform(np.log(1e-300), np.log(745.0), 200_000)),  # every scale
        -(np.arange(0, 2150) * ln2 / 2.0),                            # reduction boundaries
        -(np.arange(0, 2150) * ln2 / 2.0) * (1 + 1e-15),
        np.array([0.0, -0.0, -5e-324, -1e-300, -1e-16, -0.5, -1.0, -708.39, -708.4,
                  -745.0, -745.13])])
    x = x[x >= -745.13]
    y = dev_exp(x)
    ref = np.exp(x)
    normal = ref >= np.finfo(np.float64).tiny
    ulp = np.abs(y[normal] - ref[normal]) / np.spacing(ref[normal])
    print("normal results: %d, max error %.2f ulp, mean %.3f ulp" % (
        normal.sum(), ulp.max(), ulp.mean()))
    assert ulp.max() <= 3.0
    sub = ~normal
    abs_err = np.abs(y[sub] - ref[sub])
    assert abs_err.max() <= 4 * 5e-324
    assert dev_exp(np.array([0.0, -0.0]))[0] == 1.0
    assert np.all(dev_exp(np.array([-746.0, -800.0, -1e4])) == 0.0)


def dev_exp32(x):
    import paper_2205_10879_amd as f
    xd = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    yd = torch.empty_like(xd)
    st = f.lib().fastmuygps_debug_exp_nonpos32(ctypes.c_void_p(xd.data_ptr()),
                                               ctypes.c_void_p(yd.data_ptr()), xd.numel(), None)
    assert st == f.FMG_OK
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def test_exp_nonpos32_accuracy():
    rs = np.random.default_rng(12)
    ln2 = np.log(2.0)
    x = np.concatenate([
        -np.linspace(0.0, 104.0, 400_001),
        -np.exp(rs.uniform(np.log(1e-38), np.log(104.0), 200_000)),   # every scale
        -(np.arange(0, 300) * ln2 / 2.0),                             # reduction boundaries
        -(np.arange(0, 300) * ln2 / 2.0) * (1 + 1e-7),
        np.array([0.0, -0.0, -1e-45, -1e-38, -1e-8, -0.5, -1.0, -87.3, -87.4, -103.0])])
    x = x.astype(np.float32)
    y = dev_exp32(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    normal = ref >= np.finfo(np.float32).tiny
    ulp = np.abs(y[normal] - ref[normal]) / np.spacing(ref[normal].astype(np.float32)).astype(np.float64)
    print("normal results: %d, max error %.2f ulp, mean %.3f ulp" % (
        normal.sum(), ulp.max(), ulp.mean()))
    assert ulp.max() <= 2.0
    sub = ~normal
    assert np.abs(y[sub] - ref[sub]).max() <= np.finfo(np.float32).tiny
    assert dev_exp32(np.array([0.0, -0.0]))[0] == 1.0
    assert np.all(dev_exp32(np.array([-120.0, -200.0, -1e4])) <= np.finfo(np.float32).tiny)
