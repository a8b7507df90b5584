"""The no-allocation solve (qiht_niht_solve_noalloc) against qiht_niht_solve,
both called through the C ABI: the same kernels run on the library's fixed
device array instead of pool memory, so x, the support and the solve's
counters must be bitwise equal.  Two calls in a row, the second on a smaller
problem (the array then still holds the first call's contents), then a warm
start, and the host-side rejections (profiling, refit) with the outputs left
untouched.
"""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
from paper_1802_04907_amd import _lib  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problem(m, n, s, bits, seed):
    p = workloads.gaussian(m, n, s, 1e-3, seed=seed, dtype=np.float32)
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), bits, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), 8, p.seed)
    return q, yhat, s


def _params(max_iters, x0=None, sup0=None, profile=0, refit=0):
    prm = _lib.QihtParams()
    lib = _lib.load()
    lib.qiht_default_params(C.byref(prm))
    prm.max_iters, prm.tol = max_iters, 1e-7
    prm.x0 = None if x0 is None else x0.data_ptr()
    prm.support0 = None if sup0 is None else sup0.data_ptr()
    prm.profile, prm.refit = profile, refit
    return prm


def _call(fn, q, yhat, s, prm):
    x = torch.full((q.n,), -7.0, dtype=torch.float32, device=DEV)
    sup = torch.full((s,), -7, dtype=torch.int32, device=DEV)
    inf = _lib.QihtInfo()
    st = fn(q.handle, C.c_void_p(yhat.data_ptr()), s, C.byref(prm), C.c_void_p(x.data_ptr()),
            C.c_void_p(sup.data_ptr()), C.byref(inf),
            C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, x, sup, inf


def _same(q, yhat, s, max_iters, x0=None, sup0=None, label=""):
    lib = _lib.load()
    st_a, xa, sa, ia = _call(lib.qiht_niht_solve, q, yhat, s, _params(max_iters, x0, sup0))
    assert st_a == 0, qiht.last_error()
    st_b, xb, sb, ib = _call(lib.qiht_niht_solve_noalloc, q, yhat, s, _params(max_iters, x0, sup0))
    assert st_b == 0, qiht.last_error()
    print(f"{label}: {ia.iterations} iterations, {ia.backtracks} shrinks", flush=True)
    assert torch.equal(xa.view(torch.int32), xb.view(torch.int32)), label
    assert torch.equal(sa, sb), label
    for f in ("iterations", "reason", "backtracks", "capped_iterations", "mu_last", "full_selects"):
        assert getattr(ia, f) == getattr(ib, f), (label, f)
    return xb, sb


def test_noalloc_solve_matches_pool_solve_twice_then_smaller():
    q1, y1, s1 = _problem(1500, 6000, 60, 4, seed=11)
    _same(q1, y1, s1, 80, label="1500 x 6000, 4-bit")
    q2, y2, s2 = _problem(300, 1000, 12, 8, seed=12)
    _same(q2, y2, s2, 60, label="300 x 1000, 8-bit (after the larger call)")
    # warm start from a partial solve of the first problem
    x0, sup0, _ = qiht.niht_solve(q1, y1, s1, max_iters=5, tol=-1.0)
    _same(q1, y1, s1, 20, x0=x0, sup0=sup0, label="warm start")
    q1.free()
    q2.free()


def test_noalloc_rejects_profile_and_refit_untouched():
    q, yhat, s = _problem(200, 800, 8, 4, seed=13)
    lib = _lib.load()
    for kw in (dict(profile=1), dict(refit=1)):
        st, x, sup, _ = _call(lib.qiht_niht_solve_noalloc, q, yhat, s, _params(10, **kw))
        assert st == 2, kw  # UNSUPPORTED
        assert bool((x == -7.0).all()) and bool((sup == -7).all()), "outputs touched on error"
    q.free()
