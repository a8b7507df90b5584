"""Resume and failure paths on the GPU.

* Resume: the solver's state after an iteration is x (FP32) and its support,
  so 50 iterations, then 50 more warm-started from that state, must give the
  same bits as 100 in one call (fixed realizations Q1, Q2, no stop test).
* Allocation failure: with QIHT_FAIL_ALLOC_AFTER=N the library's (N+1)-th
  device allocation fails; every call must then return OUT_OF_MEMORY (or
  succeed, when it needed no more than N), and once the injection ends the
  library must give the same bits as before.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("bits", [4, 8])
def test_resume_50_plus_50_equals_100(bits):
    p = workloads.gaussian(1200, 4000, 24, 1e-3, seed=31 + bits, dtype=np.float32)
    q = qiht.quantize_matrix(_t(p.phi), bits, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(_t(p.y), 8, p.seed)
    x100, s100, i100 = qiht.niht_solve(q, yhat, p.s, max_iters=100, tol=-1.0)
    x50, s50, i50 = qiht.niht_solve(q, yhat, p.s, max_iters=50, tol=-1.0)
    xr, sr, ir = qiht.niht_solve(q, yhat, p.s, max_iters=50, tol=-1.0, x0=x50, support0=s50)
    say(f"  {bits}-bit: shrinks {i100['backtracks']} = {i50['backtracks']} + {ir['backtracks']}")
    assert i100["iterations"] == 100 and i50["iterations"] == 50 and ir["iterations"] == 50
    assert torch.equal(sr, s100)
    assert torch.equal(xr, x100)
    assert i100["backtracks"] == i50["backtracks"] + ir["backtracks"]
    q.free()


def _run_all(p):
    """Quantize, solve with refit, gradient and a hard threshold; the results
    as host arrays (handles freed on the way out, also on errors)."""
    q = None
    try:
        q = qiht.quantize_matrix(_t(p.phi), 4, 2, p.seed)
        yhat, _, _ = qiht.quantize_vector(_t(p.y), 8, p.seed)
        x, sup, info = qiht.niht_solve(q, yhat, p.s, max_iters=30, tol=-1.0, refit=True)
        g, r = qiht.gradient(q, yhat, x, sup)
        ht = qiht.hard_threshold(g, p.s)
        return [t.cpu().numpy() for t in (yhat, x, sup, g, r, ht)] + [info["iterations"]]
    finally:
        if q is not None:
            q.free()


def test_allocation_failure_injection(monkeypatch):
    p = workloads.gaussian(400, 1500, 12, 1e-3, seed=5, dtype=np.float32)
    monkeypatch.delenv("QIHT_FAIL_ALLOC_AFTER", raising=False)
    ref = _run_all(p)
    failed, passed = [], []
    for n in range(0, 16):
        monkeypatch.setenv("QIHT_FAIL_ALLOC_AFTER", str(n))
        try:
            got = _run_all(p)
        except qiht.QihtError as e:
            assert e.status_name == "OUT_OF_MEMORY", (n, e.status_name, str(e))
            failed.append(n)
            continue
        passed.append(n)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    say(f"  injected failures at N = {failed}; whole sequence succeeded at N = {passed}")
    assert failed and failed[0] == 0 and passed, (failed, passed)
    monkeypatch.delenv("QIHT_FAIL_ALLOC_AFTER")
    again = _run_all(p)
    for a, b in zip(again, ref):
        np.testing.assert_array_equal(a, b)
