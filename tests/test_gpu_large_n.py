"""Selections above 65536 entries (up to 262144, a 512 x 512 image): the
full-rank path of H_s on its large instance, a solve on 262144 columns (the
candidate path), and a complex unknown of 40000 entries (80000 real columns,
every proposal on the large full-rank path), each against the oracle."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
import workloads  # noqa: E402
from oracle import complex_niht as cn  # noqa: E402
from oracle import niht  # noqa: E402
from oracle import quantizer as qz  # noqa: E402

from parity_util import oracle_matrix  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("s", [1, 1000, 100000, 262144])
def test_hard_threshold_262144_tie_heavy(s):
    rng = np.random.default_rng(s)
    n = 262144
    a = rng.integers(-50, 51, size=n).astype(np.float32)  # many equal magnitudes
    a[rng.choice(n, 30, replace=False)] = np.float32(-0.0)
    got = qiht.hard_threshold(torch.from_numpy(a).to(DEV), s).cpu().numpy()
    np.testing.assert_array_equal(got, niht.hard_threshold_support(a.astype(np.float64), s))


def test_solve_on_262144_columns_matches_oracle():
    p = workloads.gaussian(1024, 262144, 16, 1e-3, seed=12, dtype=np.float32)
    bits = 8
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), bits, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), 8, p.seed)
    x, sup, info = qiht.niht_solve(q, yhat, p.s, max_iters=60, tol=1e-7)
    say(f"  1024 x 262144: {info['iterations']} iterations ({info['reason']}), "
        f"{info['full_selects']} full selections")
    q1 = oracle_matrix(p.phi, bits, p.seed, 0)
    q2 = oracle_matrix(p.phi, bits, p.seed, 1)
    yh = qz.dequantized_vector(p.y, 8, p.seed)
    ref = niht.qiht_solve(q1, q2, yh, p.s, max_iters=60, tol=1e-7)
    np.testing.assert_array_equal(sup.cpu().numpy(), ref.support)
    assert info["iterations"] == ref.iterations
    err = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-4, err
    q.free()


def test_complex_unknown_above_65536_columns():
    p = workloads.complex_gaussian(200, 40000, 6, 1e-3, seed=13)
    q = qiht.quantize_matrix(torch.from_numpy(p.phi).to(DEV), 8, 2, p.seed)
    yhat, _, _ = qiht.quantize_vector(torch.from_numpy(p.y).to(DEV), 8, p.seed)
    x, sup, info = qiht.niht_solve_complex(q, yhat, p.s, max_iters=60, tol=1e-7)
    q1 = cn.complex_from_stacked(qz.dequantized_matrix(p.phi, 8, p.seed, 0))
    q2 = cn.complex_from_stacked(qz.dequantized_matrix(p.phi, 8, p.seed, 1))
    yh = cn.complex_from_stacked(qz.dequantized_vector(p.y, 8, p.seed))
    ref = cn.qiht_solve(q1, q2, yh, p.s, max_iters=60, tol=1e-7, x_fp32=True)
    say(f"  complex 200 x 40000: {info['iterations']}/{ref.iterations} iterations")
    np.testing.assert_array_equal(sup.cpu().numpy(), ref.support)
    assert info["iterations"] == ref.iterations
    xg = x.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(xg - ref.x) <= 1e-4 * np.linalg.norm(ref.x)
    q.free()
