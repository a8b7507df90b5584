"""MI355X (gfx950) hot path of low-precision normalized IHT (QIHT).

Guerel et al., "Compressive Sensing Using Iterative Hard Thresholding with
Low Precision Data Representation: Theory and Applications", IEEE TSP 68
(2020), arXiv:1802.04907.

This module is a thin binding of the C ABI in ``include/qiht.h``
(``libqiht.so``, built from ``csrc/``): it only marshals arguments.  Every
step of the path runs in the HIP kernels; PyTorch supplies device memory
and the current stream.  If the library is missing, calls raise -- there is
no CPU fallback.

Functions keep the C names without the ``qiht_`` prefix:
``quantize_matrix``, ``quantize_vector``, ``niht_solve``,
``niht_solve_noalloc``, ``niht_solve_complex``, ``niht_solve_batched``, ``niht_solve_fresh``, ``gradient``,
``fourier_gradient``, ``fourier_niht_solve``, ``hard_threshold``,
``refit``, ``last_error``.
"""

import ctypes as C

from . import _lib

__all__ = ["QihtError", "QMatrix", "quantize_matrix", "quantize_vector",
           "niht_solve", "niht_solve_noalloc", "niht_solve_complex", "niht_solve_batched", "niht_solve_fresh", "gradient",
           "fourier_gradient", "fourier_niht_solve", "hard_threshold",
           "last_error", "tune_report", "version", "library_path"]

library_path = _lib.LIB_PATH


class QihtError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.status_name = _lib.STATUS_NAMES.get(status, str(status))
        super().__init__(f"qiht {self.status_name}: {message}")


def _torch():
    import torch
    return torch


def _check(status):
    if status != _lib.QIHT_OK:
        raise QihtError(status, last_error())


def tune_report():
    """The autotuner's choices so far in this process (dict)."""
    import json
    lib = _lib.load()
    need = lib.qiht_tune_report(None, 0)
    buf = C.create_string_buffer(max(1, int(need)))
    lib.qiht_tune_report(buf, len(buf))
    return json.loads(buf.value.decode() or "{}")


def last_error():
    return _lib.load().qiht_last_error().decode()


def version():
    return _lib.load().qiht_version().decode()


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dtype_code(t):
    torch = _torch()
    table = {torch.float64: "f64", torch.float32: "f32",
             torch.complex64: "c64", torch.complex128: "c128"}
    if t.dtype not in table:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _lib.DTYPE[table[t.dtype]]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


BF16 = _lib.QIHT_FMT_BF16  # dense storage formats for quantize_matrix(bits=...)
E4M3 = _lib.QIHT_FMT_E4M3
ODD_LEVELS = _lib.QIHT_ODD_LEVELS  # 2^(b-1) + 1 levels (odd=True below)


class QMatrix:
    """Handle on quantized measurement-matrix codes held in device memory."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)
        rows, n, cb = C.c_int64(), C.c_int64(), C.c_int64()
        bits, real = C.c_int(), C.c_int()
        scale = C.c_double()
        _check(_lib.load().qiht_qmatrix_info(self._h, C.byref(rows), C.byref(n),
                                             C.byref(bits), C.byref(real),
                                             C.byref(scale), C.byref(cb)))
        self.rows, self.n, self.bits = rows.value, n.value, bits.value
        self.realizations, self.scale, self.col_bytes = real.value, scale.value, cb.value

    @property
    def handle(self):
        return self._h

    def export_codes(self, realization=0):
        """Codes of one realization as a (rows, n) numpy array (host): uint8
        codes, or float32 values (bits 32 and BF16), or E4M3 bytes."""
        import numpy as np
        if self.bits in (32, _lib.QIHT_FMT_BF16):
            out = np.empty((self.n, self.rows), dtype=np.float32)
        else:
            out = np.empty((self.n, self.rows), dtype=np.uint8)
        _check(_lib.load().qiht_qmatrix_export_codes(
            self._h, int(realization), out.ctypes.data_as(C.c_void_p)))
        return out.T

    def row_exponents(self):
        """Row exponents e_i of a dense-format matrix (host int32 array)."""
        import numpy as np
        out = np.empty(self.rows, dtype=np.int32)
        _check(_lib.load().qiht_qmatrix_row_exponents(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def free(self):
        if self._h is not None and self._h.value:
            _lib.load().qiht_qmatrix_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def quantize_matrix(phi, bits, realizations=2, seed=0, stream=None, odd=False):
    """Q(Phi, b): ``phi`` is an (m, n) CUDA tensor, row-major (stride (ld, 1));
    ``odd`` selects the odd level set (2^(b-1) + 1 levels)."""
    bits = int(bits) | (ODD_LEVELS if odd else 0)
    if phi.dim() != 2 or phi.stride(1) != 1 or not phi.is_cuda:
        raise ValueError("phi must be a 2-D row-major CUDA tensor")
    m, n = phi.shape
    out = C.c_void_p()
    _check(_lib.load().qiht_quantize_matrix(
        _ptr(phi), m, n, phi.stride(0), _dtype_code(phi), int(bits),
        int(realizations), C.c_uint64(int(seed) & (2**64 - 1)), _stream(stream),
        C.byref(out)))
    return QMatrix(out.value)


def quantize_vector(y, bits, seed=0, stream=None, want_codes=False, odd=False):
    """Q(y, b) -> (y_hat FP64 CUDA tensor of the stacked rows, codes, scale);
    ``odd`` selects the odd level set (2^(b-1) + 1 levels)."""
    torch = _torch()
    bits = int(bits) | (ODD_LEVELS if odd else 0)
    if y.dim() != 1 or not y.is_contiguous() or not y.is_cuda:
        raise ValueError("y must be a contiguous 1-D CUDA tensor")
    rows = y.numel() * (2 if y.is_complex() else 1)
    yhat = torch.empty(rows, dtype=torch.float64, device=y.device)
    codes = torch.empty(rows, dtype=torch.uint8, device=y.device) if want_codes else None
    scale = C.c_double()
    _check(_lib.load().qiht_quantize_vector(
        _ptr(y), y.numel(), _dtype_code(y), int(bits),
        C.c_uint64(int(seed) & (2**64 - 1)), _stream(stream), _ptr(yhat),
        _ptr(codes), C.byref(scale)))
    return yhat, codes, scale.value


def _params(max_iters, tol, k, c, max_backtracks, mu_mode, x0=None, support0=None,
            profile=False, refit=False):
    p = _lib.QihtParams()
    _lib.load().qiht_default_params(C.byref(p))
    p.max_iters, p.tol, p.k, p.c = int(max_iters), float(tol), float(k), float(c)
    p.max_backtracks, p.mu_mode = int(max_backtracks), int(mu_mode)
    # profile: False/0 off, True/1 every pass launch timed, N every N-th
    p.profile = int(profile) if profile else 0
    p.refit = 1 if refit else 0
    p.x0 = None if x0 is None else x0.data_ptr()
    p.support0 = None if support0 is None else support0.data_ptr()
    return p


def _info_dict(inf):
    return dict(iterations=inf.iterations, reason=_lib.REASONS.get(inf.reason, inf.reason),
                backtracks=inf.backtracks, capped_iterations=inf.capped_iterations,
                mu_last=inf.mu_last, pass_ms=inf.pass_ms, pass_launches=inf.pass_launches,
                full_selects=inf.full_selects)


def niht_solve(q, yhat, s, max_iters=300, tol=1e-8, k=2.0, c=0.01, max_backtracks=32,
               mu_mode=0, x0=None, support0=None, stream=None, profile=False, refit=False):
    """QIHT solve -> (x FP32 CUDA tensor, support int32 CUDA tensor, info dict)."""
    torch = _torch()
    x = torch.empty(q.n, dtype=torch.float32, device=yhat.device)
    sup = torch.empty(int(s), dtype=torch.int32, device=yhat.device)
    if x0 is not None:
        x0 = x0.to(dtype=torch.float32).contiguous()
        support0 = support0.to(dtype=torch.int32).contiguous()
    p = _params(max_iters, tol, k, c, max_backtracks, mu_mode, x0, support0, profile, refit)
    inf = _lib.QihtInfo()
    _check(_lib.load().qiht_niht_solve(q.handle, _ptr(yhat), int(s), C.byref(p), _ptr(x),
                                       _ptr(sup), C.byref(inf), _stream(stream)))
    return x, sup, _info_dict(inf)


def niht_solve_complex(q, yhat, s, max_iters=300, tol=1e-8, k=2.0, c=0.01, max_backtracks=32,
                       mu_mode=0, stream=None, profile=False, refit=False):
    """QIHT with a complex unknown on a handle quantized from complex Phi
    -> (x complex64 CUDA tensor of n, support int32, info dict)."""
    torch = _torch()
    xr = torch.empty(2 * q.n, dtype=torch.float32, device=yhat.device)
    sup = torch.empty(int(s), dtype=torch.int32, device=yhat.device)
    p = _params(max_iters, tol, k, c, max_backtracks, mu_mode, profile=profile, refit=refit)
    inf = _lib.QihtInfo()
    _check(_lib.load().qiht_niht_solve_complex(q.handle, _ptr(yhat), int(s), C.byref(p), _ptr(xr),
                                               _ptr(sup), C.byref(inf), _stream(stream)))
    x = torch.complex(xr[:q.n], xr[q.n:])
    return x, sup, _info_dict(inf)


def niht_solve_noalloc(q, yhat, s, max_iters=300, tol=1e-8, k=2.0, c=0.01, max_backtracks=32,
                       mu_mode=0, x0=None, support0=None, stream=None):
    """The solve of ``niht_solve`` with its workspace in the library's fixed
    device array (no device allocation by the library; the outputs are the
    caller's tensors, allocated here by PyTorch) -> (x, support, info)."""
    torch = _torch()
    x = torch.empty(q.n, dtype=torch.float32, device=yhat.device)
    sup = torch.empty(int(s), dtype=torch.int32, device=yhat.device)
    if x0 is not None:
        x0 = x0.to(dtype=torch.float32).contiguous()
        support0 = support0.to(dtype=torch.int32).contiguous()
    p = _params(max_iters, tol, k, c, max_backtracks, mu_mode, x0, support0)
    inf = _lib.QihtInfo()
    _check(_lib.load().qiht_niht_solve_noalloc(q.handle, _ptr(yhat), int(s), C.byref(p), _ptr(x),
                                               _ptr(sup), C.byref(inf), _stream(stream)))
    return x, sup, _info_dict(inf)


def niht_solve_fresh(phi, y, s, bits, ybits=8, seed=0, max_iters=300, tol=1e-8, k=2.0,
                     c=0.01, max_backtracks=32, mu_mode=0, stream=None, odd=False, yodd=False,
                     profile=False):
    """Algorithm 2 with new realizations of Q(Phi) and Q(y) every iteration
    (``phi``: (m, n) row-major CUDA tensor, ``y``: its m observations; both are
    re-quantized on the device each iteration) -> (x, support, info)."""
    torch = _torch()
    if phi.dim() != 2 or phi.stride(1) != 1 or not phi.is_cuda:
        raise ValueError("phi must be a 2-D row-major CUDA tensor")
    if y.dim() != 1 or not y.is_contiguous() or not y.is_cuda:
        raise ValueError("y must be a contiguous 1-D CUDA tensor")
    m, n = phi.shape
    x = torch.empty(n, dtype=torch.float32, device=phi.device)
    sup = torch.empty(s, dtype=torch.int32, device=phi.device)
    p = _params(max_iters, tol, k, c, max_backtracks, mu_mode, profile=profile)
    inf = _lib.QihtInfo()
    _check(_lib.load().qiht_niht_solve_fresh(
        _ptr(phi), m, n, phi.stride(0), _dtype_code(phi), int(bits) | (ODD_LEVELS if odd else 0),
        _ptr(y), _dtype_code(y), int(ybits) | (ODD_LEVELS if yodd else 0),
        C.c_uint64(int(seed) & (2**64 - 1)), int(s), C.byref(p), _ptr(x), _ptr(sup),
        C.byref(inf), _stream(stream)))
    return x, sup, _info_dict(inf)


def niht_solve_batched(problems, max_iters=300, tol=1e-8, k=2.0, c=0.01,
                       max_backtracks=32, mu_mode=0, stream=None, profile=False, refit=False):
    """Batched solve; ``problems`` is a list of (QMatrix, yhat, s).

    Returns a list of (x, support, info)."""
    torch = _torch()
    cnt = len(problems)
    arr = (_lib.QihtProblem * cnt)()
    # one allocation each for all x and all supports; the outputs are views
    dev = problems[0][1].device
    nx = [q.n for q, _, _ in problems]
    ns = [int(s) for _, _, s in problems]
    xall = torch.empty(sum(nx), dtype=torch.float32, device=dev)
    sall = torch.empty(max(1, sum(ns)), dtype=torch.int32, device=dev)
    outs = []
    ox = osp = 0
    for i, (q, yhat, s) in enumerate(problems):
        x = xall[ox:ox + nx[i]]
        sup = sall[osp:osp + ns[i]]
        ox += nx[i]
        osp += ns[i]
        outs.append((x, sup))
        arr[i] = _lib.QihtProblem(q.handle.value, yhat.data_ptr(), ns[i],
                                  x.data_ptr(), sup.data_ptr())
    p = _params(max_iters, tol, k, c, max_backtracks, mu_mode, profile=profile, refit=refit)
    infos = (_lib.QihtInfo * cnt)()
    _check(_lib.load().qiht_niht_solve_batched(cnt, arr, C.byref(p), infos, _stream(stream)))
    return [(x, sup, _info_dict(infos[i])) for i, (x, sup) in enumerate(outs)]


_DTYPES = {"float64": 0, "float32": 1, "complex64": 2, "complex128": 3}


def refit(support, y, q=None, phi=None, n=None, stream=None):
    """FP64 least-squares refit on a support (not part of the paper's method).

    A is ``phi`` (a CUDA tensor, m x n row-major, real or complex) when given,
    else the dequantized first realization of ``q``.  ``y`` holds the
    rows measurements in FP64.  Returns (x FP32 n, z FP64 on the support)."""
    torch = _torch()
    sup = support.to(torch.int32).contiguous()
    s = sup.numel()
    yv = y.to(torch.float64).contiguous()
    if phi is not None:
        phi = phi.contiguous()
        m, nn = phi.shape
        ld = nn
        dt = _DTYPES[str(phi.dtype).replace("torch.", "")]
        handle = None
    else:
        nn, m, ld, dt, handle = q.n, 0, 0, 0, q.handle
    x = torch.empty(nn, dtype=torch.float32, device=yv.device)
    z = torch.empty(s, dtype=torch.float64, device=yv.device)
    _check(_lib.load().qiht_refit(handle, _ptr(phi), int(m), int(nn), int(ld), int(dt),
                                  _ptr(yv), _ptr(sup), int(s), _ptr(x), _ptr(z),
                                  _stream(stream)))
    return x, z


def gradient(q, yhat, x, support, stream=None):
    """(g, r): r = y_hat - Q2_G x_G and g = Q1^T r at a sparse x."""
    torch = _torch()
    g = torch.empty(q.n, dtype=torch.float32, device=yhat.device)
    r = torch.empty(q.rows, dtype=torch.float32, device=yhat.device)
    s = 0 if support is None else support.numel()
    xs = None if x is None else x.to(torch.float32).contiguous()
    ss = None if support is None else support.to(torch.int32).contiguous()
    _check(_lib.load().qiht_gradient(q.handle, _ptr(yhat), _ptr(xs), _ptr(ss), s, _ptr(g),
                                     _ptr(r), _stream(stream)))
    return g, r


def fourier_gradient(uv, side, r, stream=None):
    """g = [Re Phi; Im Phi]^T r of the Fourier-sampled matrix
    Phi_jk = exp(-2 pi i (u_j l_k + v_j m_k)) computed on the fly (no matrix
    in memory).  uv: (n_vis, 2) CUDA tensor of (u, v); r: 2 n_vis stacked
    [Re; Im]; returns g, side * side float32."""
    torch = _torch()
    uv = uv.to(torch.float64).contiguous()
    r = r.to(torch.float32).contiguous()
    g = torch.empty(int(side) * int(side), dtype=torch.float32, device=r.device)
    _check(_lib.load().qiht_fourier_gradient(_ptr(uv), uv.shape[0], int(side), _ptr(r), _ptr(g),
                                             _stream(stream)))
    return g


def fourier_niht_solve(uv, side, y, s, max_iters=300, tol=1e-8, k=2.0, c=0.01, max_backtracks=32,
                       stream=None):
    """Normalized IHT on the Fourier-sampled Phi computed on the fly.  uv:
    (n_vis, 2) CUDA tensor; y: 2 n_vis stacked [Re; Im] -> (x, support, info)."""
    torch = _torch()
    uv = uv.to(torch.float64).contiguous()
    y = y.to(torch.float64).contiguous()
    n = int(side) * int(side)
    x = torch.empty(n, dtype=torch.float32, device=y.device)
    sup = torch.empty(int(s), dtype=torch.int32, device=y.device)
    p = _params(max_iters, tol, k, c, max_backtracks, 0)
    inf = _lib.QihtInfo()
    _check(_lib.load().qiht_fourier_niht_solve(_ptr(uv), uv.shape[0], int(side), _ptr(y), int(s),
                                               C.byref(p), _ptr(x), _ptr(sup), C.byref(inf),
                                               _stream(stream)))
    return x, sup, _info_dict(inf)


def hard_threshold(a, s, stream=None):
    """H_s support (ascending int32 CUDA tensor) of a float32 CUDA vector."""
    torch = _torch()
    a = a.to(torch.float32).contiguous()
    out = torch.empty(int(s), dtype=torch.int32, device=a.device)
    _check(_lib.load().qiht_hard_threshold(_ptr(a), a.numel(), int(s), _ptr(out),
                                           _stream(stream)))
    return out
