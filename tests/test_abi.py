"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmuygps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastmuygps_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2205_10879_amd as fmg
    if not os.path.exists(fmg.LIB_PATH):
        pytest.fail("HIP library not built: run `python -m paper_2205_10879_amd.build`")
    return fmg.lib()


def test_header_declares_the_paper_calls():
    names = declared_functions()
    for required in ("fastmuygps_build", "fastmuygps_predict", "fastmuygps_free",
                     "fastmuygps_info", "fastmuygps_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    import paper_2205_10879_amd as fmg
    names = declared_functions()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(fmg.EXPORTS)


def test_version(lib):
    import paper_2205_10879_amd as fmg
    assert fmg.version().startswith("fastmuygps-gfx950")


def test_bad_arguments_fail_before_any_device_call(lib):
    import paper_2205_10879_amd as fmg
    h = ctypes.c_void_p()
    hyper = fmg.FmgHyper(fmg.KERNEL_MATERN, 1.5, 1.0, 0.1, 1.0)
    st = lib.fastmuygps_build(None, None, 10, 2, 1, 3, ctypes.byref(hyper), fmg.PREC_FP32, 0,
                              None, ctypes.byref(h))
    assert st == fmg.FMG_E_INVALID_ARG and not h.value
    assert b"null" in lib.fastmuygps_last_error()
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    for n, d, ell, k, prec, nu, rho, noise, flags in [
            (1, 2, 1, 1, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),      # n < 2
            (10, 0, 1, 3, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),     # d < 1
            (10, 2, 0, 3, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),     # ell < 1
            (10, 2, 17, 3, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),    # ell > 16
            (10, 2, 1, 10, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),    # LOO k > n-1
            (10, 2, 1, 11, fmg.PREC_FP32, 1.5, 1.0, 0.1, fmg.FLAG_SELF_INCLUSIVE),  # k > n
            (300, 2, 1, 257, fmg.PREC_FP32, 1.5, 1.0, 0.1, 0),  # k > 256
            (10, 2, 1, 3, fmg.PREC_FP32, 0.7, 1.0, 0.1, 0),     # nu
            (10, 2, 1, 3, fmg.PREC_FP32, 1.5, 0.0, 0.1, 0),     # rho
            (10, 2, 1, 3, fmg.PREC_FP32, 1.5, 1.0, -0.1, 0),    # noise
            (10, 2, 1, 3, 7, 1.5, 1.0, 0.1, 0)]:                # precision
        hy = fmg.FmgHyper(fmg.KERNEL_MATERN, nu, rho, noise, 1.0)
        st = lib.fastmuygps_build(fake, fake, n, d, ell, k, ctypes.byref(hy), prec, flags, None,
                                  ctypes.byref(h))
        assert st == fmg.FMG_E_INVALID_ARG, (n, d, ell, k, prec, nu, rho, noise)
    hy = fmg.FmgHyper(fmg.KERNEL_RBF, 0.0, 1.0, 0.1, 1.0)
    st = lib.fastmuygps_build(fake, fake, 100, 62, 1, 3, ctypes.byref(hy), fmg.PREC_MIXED, 0,
                              None, ctypes.byref(h))
    assert st == fmg.FMG_E_UNSUPPORTED
    st = lib.fastmuygps_predict(None, fake, 5, fake, None, None)
    assert st == fmg.FMG_E_INVALID_ARG
    lib.fastmuygps_free(None)


def test_package_has_no_cpu_fallback():
    """The product path never imports the oracle."""
    import paper_2205_10879_amd as fmg
    src = open(fmg.__file__).read()
    assert "oracle" not in src.replace("no fallback", "")


def test_server_calls_reject_bad_arguments_before_any_device_call(lib):
    import paper_2205_10879_amd as fmg
    h = ctypes.c_void_p()
    for slots, max_batch in ((9, 100), (-1, 100), (2, 70000), (2, -5)):
        opts = fmg.FmgServerOpts(slots, max_batch, 1)
        st = lib.fastmuygps_server_create(0, ctypes.byref(opts), ctypes.byref(h))
        assert st == fmg.FMG_E_INVALID_ARG and not h.value, (slots, max_batch)
    assert lib.fastmuygps_server_create(0, None, None) == fmg.FMG_E_INVALID_ARG
    t = ctypes.c_void_p()
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    assert lib.fastmuygps_server_submit(None, 0, fake, 1, fake, 0, ctypes.byref(t)) == \
        fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_server_wait(None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_server_add_model(None, None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_server_remove_model(None, 0) == fmg.FMG_E_INVALID_ARG
    st = fmg.FmgServerStats()
    assert lib.fastmuygps_server_stats(None, ctypes.byref(st)) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_server_reset_stats(None) == fmg.FMG_E_INVALID_ARG
    lib.fastmuygps_server_destroy(None)


def test_muygps_and_loo_calls_reject_bad_arguments(lib):
    import paper_2205_10879_amd as fmg
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    assert lib.fastmuygps_predict_muygps(None, fake, 5, fake, None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_predict_muygps(fake, None, 5, fake, None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_predict_muygps(fake, fake, -1, fake, None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_loo_predict(None, fake, 5, fake, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_loo_predict(fake, None, 5, fake, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_loo_predict(fake, fake, -2, fake, None) == fmg.FMG_E_INVALID_ARG


def test_loo_loss_rejects_bad_arguments(lib):
    import paper_2205_10879_amd as fmg
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    hy = fmg.FmgHyper(fmg.KERNEL_MATERN, 1.5, 1.0, 0.1, 1.0)
    out = ctypes.c_double()
    assert lib.fastmuygps_loo_loss(None, fake, 4, ctypes.byref(hy), ctypes.byref(out),
                                   None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_loo_loss(fake, fake, 0, ctypes.byref(hy), ctypes.byref(out),
                                   None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_loo_loss(fake, fake, 4, None, ctypes.byref(out),
                                   None) == fmg.FMG_E_INVALID_ARG


def test_loo_loss_grad_rejects_bad_arguments(lib):
    import paper_2205_10879_amd as fmg
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    hy = fmg.FmgHyper(fmg.KERNEL_MATERN, 1.5, 1.0, 0.1, 1.0)
    out = ctypes.c_double()
    grad = (ctypes.c_double * 2)()
    f = lib.fastmuygps_loo_loss_grad
    assert f(None, fake, 4, ctypes.byref(hy), ctypes.byref(out), grad, None) == fmg.FMG_E_INVALID_ARG
    assert f(fake, None, 4, ctypes.byref(hy), ctypes.byref(out), grad, None) == fmg.FMG_E_INVALID_ARG
    assert f(fake, fake, 0, ctypes.byref(hy), ctypes.byref(out), grad, None) == fmg.FMG_E_INVALID_ARG
    assert f(fake, fake, 4, None, ctypes.byref(out), grad, None) == fmg.FMG_E_INVALID_ARG
    assert f(fake, fake, 4, ctypes.byref(hy), None, grad, None) == fmg.FMG_E_INVALID_ARG
    assert f(fake, fake, 4, ctypes.byref(hy), ctypes.byref(out), None, None) == fmg.FMG_E_INVALID_ARG


def test_wide_neighbourhood_limits_are_checked_before_any_device_work(lib):
    import paper_2205_10879_amd as fmg
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    hy = fmg.FmgHyper(fmg.KERNEL_MATERN, 1.5, 1.0, 0.1, 1.0)
    out = ctypes.c_void_p()
    b = lib.fastmuygps_build
    # k above 256
    assert b(fake, fake, 1000, 4, 1, 257, ctypes.byref(hy), fmg.PREC_FP64, 0, None,
             ctypes.byref(out)) == fmg.FMG_E_INVALID_ARG
    # k > 64 is not offered in MIXED precision
    assert b(fake, fake, 1000, 4, 1, 100, ctypes.byref(hy), fmg.PREC_MIXED, 0, None,
             ctypes.byref(out)) == fmg.FMG_E_UNSUPPORTED
    # the packed FP64 factor of k = 256 does not fit 160 KB of LDS
    assert b(fake, fake, 1000, 4, 1, 256, ctypes.byref(hy), fmg.PREC_FP64, 0, None,
             ctypes.byref(out)) == fmg.FMG_E_UNSUPPORTED
    assert out.value is None


def test_noalloc_predict_rejects_bad_arguments_before_any_device_call(lib):
    import paper_2205_10879_amd as fmg
    fake = ctypes.c_void_p(16)  # never dereferenced: arguments are checked first
    assert lib.fastmuygps_predict_noalloc(None, fake, 5, fake, None, None) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_predict_noalloc(fake, fake, -1, fake, None, None) == fmg.FMG_E_INVALID_ARG
    st = lib.fastmuygps_predict_noalloc(fake, fake, fmg.NOALLOC_MAX_M + 1, fake, None, None)
    assert st == fmg.FMG_E_INVALID_ARG
    assert b"allocation-free limit" in lib.fastmuygps_last_error()
    assert lib.fastmuygps_predict_noalloc(fake, fake, 0, fake, None, None) == fmg.FMG_OK
    # a modest static array: the batch limit's workspace, well under 128 MiB
    assert 64 << 20 < lib.fastmuygps_noalloc_scratch_bytes() < 128 << 20


def test_noalloc_limit_matches_the_header():
    import re

    import paper_2205_10879_amd as fmg
    text = open(HEADER).read()
    assert int(re.search(r"#define FMG_NOALLOC_MAX_M (\d+)", text).group(1)) == fmg.NOALLOC_MAX_M


def test_model_files_are_checked_before_any_device_work(lib, tmp_path):
    import paper_2205_10879_amd as fmg
    h = ctypes.c_void_p()
    assert lib.fastmuygps_load(None, ctypes.byref(h)) == fmg.FMG_E_INVALID_ARG
    assert lib.fastmuygps_save(None, b"/dev/null") == fmg.FMG_E_INVALID_ARG
    missing = str(tmp_path / "no_such_model.fmg").encode()
    assert lib.fastmuygps_load(missing, ctypes.byref(h)) == fmg.FMG_E_IO
    assert not h.value
    other = tmp_path / "not_a_model.fmg"
    other.write_bytes(b"NOTMODEL" + bytes(64))
    assert lib.fastmuygps_load(str(other).encode(), ctypes.byref(h)) == fmg.FMG_E_IO
    assert b"not a model file" in lib.fastmuygps_last_error()
    newer = tmp_path / "newer_format.fmg"
    newer.write_bytes(b"FMGMODEL" + (2).to_bytes(4, "little") + bytes(64))
    assert lib.fastmuygps_load(str(newer).encode(), ctypes.byref(h)) == fmg.FMG_E_IO
    assert not h.value
