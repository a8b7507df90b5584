"""QIHT with a complex unknown on the GPU (qiht_niht_solve_complex) against
the complex oracle (oracle/complex_niht.py), which runs Algorithm 2 in
complex arithmetic on the oracle's own realizations of Q(Phi) = Q(Re Phi) +
i Q(Im Phi) and of y_hat.  Bars: identical supports and iteration counts,
x within 1e-4 relative (the GPU holds x in FP32; the oracle rounds its
iterate to FP32 between iterations as the GPU does), and the shrink counts
where the support settles (8 and 32 bits)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
from paper_1802_04907_amd import QihtError  # noqa: E402
import workloads  # noqa: E402
from oracle import complex_niht as cn  # noqa: E402
from oracle import quantizer as qz  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def _gpu(p, bits, ybits):
    q = qiht.quantize_matrix(torch.from_numpy(np.ascontiguousarray(p.phi)).to(DEV), bits, 2, p.seed)
    y = torch.from_numpy(np.ascontiguousarray(p.y.astype(np.complex128))).to(DEV)
    yhat, _, _ = qiht.quantize_vector(y, ybits, p.seed)
    return q, yhat


def _oracle(p, bits, ybits):
    y = p.y.astype(np.complex128)
    if bits == 32:
        st = qz.stack_real(p.phi).astype(np.float32).astype(np.float64)
        q1 = q2 = cn.complex_from_stacked(st)
    else:
        q1 = cn.complex_from_stacked(qz.dequantized_matrix(p.phi, bits, p.seed, 0))
        q2 = cn.complex_from_stacked(qz.dequantized_matrix(p.phi, bits, p.seed, 1))
    if ybits == 32:
        yh = cn.complex_from_stacked(qz.stack_real(y).astype(np.float32).astype(np.float64))
    else:
        yh = cn.complex_from_stacked(qz.dequantized_vector(y, ybits, p.seed))
    return q1, q2, yh


def _compare(p, bits, ybits, iters, tol, label, shrinks=True):
    q, yhat = _gpu(p, bits, ybits)
    x, sup, info = qiht.niht_solve_complex(q, yhat, p.s, max_iters=iters, tol=tol)
    q1, q2, yh = _oracle(p, bits, ybits)
    ref = cn.qiht_solve(q1, q2, yh, p.s, max_iters=iters, tol=tol, x_fp32=True)
    xg = x.cpu().numpy().astype(np.complex128)
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    say(f"  {label}: {info['iterations']}/{ref.iterations} iterations, shrinks "
        f"{info['backtracks']}/{ref.backtracks}, |x - x_oracle|/|x_oracle| = {err:.2e}, "
        f"recovery {np.linalg.norm(ref.x - p.x_true) / np.linalg.norm(p.x_true):.3g}")
    np.testing.assert_array_equal(sup.cpu().numpy(), ref.support)
    assert info["iterations"] == ref.iterations
    if shrinks:
        assert info["backtracks"] == ref.backtracks
    assert err <= 1e-4, err
    # x is zero off the support
    off = np.setdiff1d(np.arange(q.n), ref.support)
    assert np.all(xg[off] == 0)
    q.free()


@pytest.mark.parametrize("bits,ybits", [(32, 32), (8, 8), (5, 8), (4, 8), (3, 8)])
def test_complex_gaussian_matches_oracle(bits, ybits):
    p = workloads.complex_gaussian(192, 640, 8, 1e-3, seed=7)
    # At 3 bits the iterate settles with |x - x_prev| / |x| near 1e-7, the
    # size of the FP32 rounding differences between the two x: a stop test at
    # 1e-7 would be decided by that noise, so it is taken at 1e-5.
    tol = 1e-5 if bits == 3 else 1e-7
    _compare(p, bits, ybits, 150, tol, f"complex Gaussian {bits}/{ybits}", shrinks=bits >= 5)


def test_complex_gaussian_ragged():
    p = workloads.complex_gaussian(77, 301, 5, 1e-3, seed=8)
    _compare(p, 8, 8, 120, 1e-7, "ragged 77 x 301, 8-bit")


def test_complex_sky_on_the_interferometry_matrix():
    p = workloads.interferometry(n_vis=1200, side=32, s=12, snr_db=30.0, seed=3, complex_sky=True)
    assert np.iscomplexobj(p.x_true) and np.all(np.abs(p.x_true[p.support]) > 0)
    _compare(p, 8, 8, 120, 1e-7, "interferometry 1200 x 1024, complex sky, 8-bit")


def test_real_data_with_odd_levels_keeps_x_real():
    """Phi and y with zero imaginary parts on the odd level set (0 is a level,
    so Q(0) = 0 and the quantized imaginary parts vanish): the gradient's
    imaginary part is exactly 0 and x stays real, on the oracle's support.
    (With 2^b levels 0 is not a level: Q(0) = +-c/(2^b - 1) at random.)"""
    p = workloads.gaussian(150, 500, 6, 1e-3, seed=4, dtype=np.float32)
    phic = p.phi.astype(np.complex64)
    yc = p.y.astype(np.complex128)
    q = qiht.quantize_matrix(torch.from_numpy(phic).to(DEV), 8, 2, 1, odd=True)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(yc).to(DEV), 8, 1, odd=True)
    x, sup, info = qiht.niht_solve_complex(q, yhat, p.s, max_iters=100, tol=1e-7)
    q1 = cn.complex_from_stacked(qz.dequantized_matrix(phic, 8, 1, 0, odd=True))
    q2 = cn.complex_from_stacked(qz.dequantized_matrix(phic, 8, 1, 1, odd=True))
    yh = cn.complex_from_stacked(qz.dequantized_vector(yc, 8, 1, odd=True))
    assert np.max(np.abs(q1.imag)) == 0.0 and np.max(np.abs(yh.imag)) == 0.0
    ref = cn.qiht_solve(q1, q2, yh, p.s, max_iters=100, tol=1e-7, x_fp32=True)
    np.testing.assert_array_equal(sup.cpu().numpy(), ref.support)
    assert info["iterations"] == ref.iterations
    assert float(x.imag.abs().max()) == 0.0
    xg = x.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(xg - ref.x) <= 1e-4 * np.linalg.norm(ref.x)
    q.free()


def test_complex_refit_is_complex_least_squares():
    p = workloads.complex_gaussian(160, 400, 6, 1e-3, seed=9)
    q, yhat = _gpu(p, 8, 8)
    x, sup, _ = qiht.niht_solve_complex(q, yhat, p.s, max_iters=150, tol=1e-7, refit=True)
    q1, _, yh = _oracle(p, 8, 8)
    sp = sup.cpu().numpy()
    z, *_ = np.linalg.lstsq(q1[:, sp], yh, rcond=None)
    xg = x.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(xg[sp] - z) <= 1e-6 * np.linalg.norm(z)
    q.free()


def test_complex_solve_rejections():
    p = workloads.gaussian(64, 128, 4, 1e-3, seed=2, dtype=np.float32)
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), 8, 2, 0)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), 8, 0)
    with pytest.raises(QihtError) as e:
        qiht.niht_solve_complex(q, yhat, 4)
    assert e.value.status_name == "INVALID_ARG"
    q.free()
