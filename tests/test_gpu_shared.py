"""GPU parity of the shared-matrix path: one measurement matrix held in a
dense format (FP32, BF16, FP8 E4M3 with power-of-two row scales) and many
right-hand sides solved together, the per-iteration products of all of them
one GEMM on the matrix cores.

Bars (stated per test):
* stored values and row exponents: bit-exact against oracle.lowprec;
* gradient g: |g_gpu - g_orc| <= 1e-5 max(|g_orc|, 1e-3 |g0|) with the
  oracle in FP64 on the effective matrix A = diag(2^e) Phi~ at the GPU's x,
  and entry by entry |g_gpu_j - g_orc_j| <= 1e-5 sum_i |a_ij r_i|;
  r: the FP64 residual rounded once to FP32;
* solves: against the oracle's NIHT on A (the stored operand, exact in
  FP64) with y_hat = y: identical supports, |x_gpu - x_orc| / |x_orc| <= 1e-4;
* refit on a dense handle: as the other refits, 1e-9 relative.
The effect of the format itself (A against the unrounded Phi) is reported
as the recovery error against the true signal, not as a parity bar.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1802_04907_amd as qiht  # noqa: E402
import workloads  # noqa: E402
from oracle import lowprec as lp  # noqa: E402
from oracle import niht  # noqa: E402
from oracle import quantizer as qz  # noqa: E402

from parity_util import assert_g_elementwise, g_bound  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
FMTS = {"f32": 32, "bf16": qiht.BF16, "e4m3": qiht.E4M3}


def say(*a):
    print(*a, flush=True)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _stored(q, fmt):
    """Stored values of a handle as FP64 (rows, n)."""
    c = q.export_codes(0)
    if fmt == "e4m3":
        return lp.e4m3_decode(c)
    return c.astype(np.float64)


def _scaled_rows(rng, m, n, dtype):
    """Gaussian rows spread over 2^-30 .. 2^30, one all-zero row, one row
    whose maximum sits exactly on a format boundary."""
    phi = rng.standard_normal((m, n)) * np.ldexp(1.0, rng.integers(-30, 30, (m, 1)))
    phi[m // 3] = 0.0
    phi[m // 2, 1] = 448.0 * 2.0 ** 3
    return phi.astype(dtype)


# ---------------------------------------------------------------- storage
@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
@pytest.mark.parametrize("m,n,dt", [(37, 50, np.float32), (300, 129, np.float64),
                                    (1000, 700, np.float32), (5000, 260, np.float64)])
def test_storage_bit_exact(fmt, m, n, dt):
    say(f"storage {fmt} m={m} n={n} {np.dtype(dt).name}")
    rng = np.random.default_rng(m * n)
    phi = _scaled_rows(rng, m, n, dt)
    q = qiht.quantize_matrix(_t(phi), FMTS[fmt], 1, 0)
    assert q.rows == m and q.n == n and q.realizations == 1
    st, e, _ = lp.store_matrix(phi, fmt)
    np.testing.assert_array_equal(q.row_exponents(), e)
    np.testing.assert_array_equal(_stored(q, fmt), st)
    if fmt == "e4m3":
        assert np.all(np.isin(st, lp.e4m3_values()))
    q.free()


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_storage_complex_is_stacked_real(fmt):
    rng = np.random.default_rng(9)
    m, n = 90, 130
    phi = (rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))).astype(np.complex64)
    q = qiht.quantize_matrix(_t(phi), FMTS[fmt], 1, 0)
    assert q.rows == 2 * m
    st, e, _ = lp.store_matrix(qz.stack_real(phi), fmt)
    np.testing.assert_array_equal(q.row_exponents(), e)
    np.testing.assert_array_equal(_stored(q, fmt), st)


def test_storage_zero_matrix():
    q = qiht.quantize_matrix(_t(np.zeros((40, 30), np.float32)), qiht.E4M3, 1, 0)
    assert np.all(q.row_exponents() == 0) and np.all(q.export_codes(0) == 0)


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("fmt", list(FMTS))
# (1100, 2000): BF16 rows padded to 1152, four row splits of 9 steps each
# (an odd step count through the GEMM's two-stage ring)
@pytest.mark.parametrize("m,n,s,cplx", [(300, 1200, 12, False), (1000, 3000, 40, False),
                                        (1100, 2000, 30, False), (140, 300, 9, True)])
def test_gradient_teacher_forced(fmt, m, n, s, cplx):
    say(f"shared gradient {fmt} m={m} n={n} s={s} cplx={cplx}")
    if cplx:
        p = workloads.interferometry(n_vis=m, side=int(np.sqrt(n)) + 1, s=s, seed=1)
    else:
        p = workloads.gaussian(m, n, s, 1e-3, seed=m + n, dtype=np.float32)
    q = qiht.quantize_matrix(_t(p.phi), FMTS[fmt], 1, 0)
    _, _, A = lp.store_matrix(qz.stack_real(p.phi), fmt)
    y = qz.stack_real(p.y.reshape(-1, 1)).reshape(-1)
    yt = _t(y)
    g0_gpu, r0 = qiht.gradient(q, yt, None, None)
    g0 = A.T @ y
    tol = lambda ref: 1e-5 * max(np.linalg.norm(ref), 1e-3 * np.linalg.norm(g0))  # noqa: E731
    assert np.linalg.norm(g0_gpu.cpu().numpy() - g0) <= tol(g0)
    assert_g_elementwise(g0_gpu.cpu().numpy(), g0, g_bound(A, y), what="g0")
    np.testing.assert_array_equal(r0.cpu().numpy(), y.astype(np.float32))
    rng = np.random.default_rng(0)
    for trial in range(3):
        nn = q.n
        sup = np.sort(rng.choice(nn, s, replace=False)).astype(np.int32)
        x = np.zeros(nn, dtype=np.float32)
        x[sup] = rng.standard_normal(s).astype(np.float32)
        g, r = qiht.gradient(q, yt, _t(x), _t(sup))
        r_or = y - A @ x.astype(np.float64)
        g_or = A.T @ r_or
        rg = r.cpu().numpy()
        assert np.all(np.abs(rg - r_or) <= 2.0 ** -23 * np.abs(r_or) + 1e-30), trial
        err = np.linalg.norm(g.cpu().numpy() - g_or)
        worst = assert_g_elementwise(g.cpu().numpy(), g_or, g_bound(A, r_or), what=f"trial {trial}")
        say(f"  trial {trial}: |dg|/|g| {err / np.linalg.norm(g_or):.2e}, "
            f"worst |dg_j| / sum_i |a_ij r_i| {worst:.2e}")
        assert err <= tol(g_or), trial
    q.free()


# ---------------------------------------------------------------- solves
# Solves run a fixed number of iterations (tol disabled: a stop test at
# 1e-7 relative sits at FP32 resolution and may end the two sides one
# iteration apart) on equal-magnitude signals whose sparsity is the solve's s
# (noise-level entries would leave the support to near-ties: on these
# workloads the oracle's s-th and (s+1)-th |x + mu g| differ by more than
# 0.4% at every iteration).
ITERS = 60


def _shared_batch(fmt, m, n, nrhs, s_of, seed):
    phi, Y, X, _ = workloads.shared_phi(m, n, nrhs, [s_of(j) for j in range(nrhs)], 1e-3, seed,
                                        equal=True)
    q = qiht.quantize_matrix(_t(phi), FMTS[fmt], 1, 0)
    ys = [_t(Y[:, j]) for j in range(nrhs)]
    res = qiht.niht_solve_batched([(q, ys[j], s_of(j)) for j in range(nrhs)],
                                  max_iters=ITERS, tol=-1.0)
    _, _, A = lp.store_matrix(phi, fmt)
    return q, A, Y, X, res


def _check_against_oracle(A, Y, X, res, s_of, js, rel=1e-4):
    worst = 0.0
    for j in js:
        x, sup, info = res[j]
        ref = niht.qiht_solve(A, A, Y[:, j], s_of(j), max_iters=ITERS, tol=-1.0)
        gs = sup.cpu().numpy()
        np.testing.assert_array_equal(gs, ref.support, err_msg=f"rhs {j}")
        assert info["iterations"] == ref.iterations
        xg = x.cpu().numpy().astype(np.float64)
        assert np.count_nonzero(np.delete(xg, gs)) == 0
        err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
        worst = max(worst, err)
        assert err <= rel, (j, err, info, ref.iterations)
    return worst


@pytest.mark.parametrize("fmt", list(FMTS))
def test_shared_batch_matches_oracle(fmt):
    # ragged: rows 300 (padded to 320 / 384 / 512), 1200 columns (9 1/3
    # tiles of 128), 40 right-hand sides of sparsity 8 .. 12
    s_of = lambda j: 8 + j % 5  # noqa: E731
    say(f"shared batch {fmt}")
    q, A, Y, X, res = _shared_batch(fmt, 300, 1200, 40, s_of, seed=11)
    worst = _check_against_oracle(A, Y, X, res, s_of, range(40))
    rec = max(np.linalg.norm(res[j][0].cpu().numpy() - X[:, j]) / np.linalg.norm(X[:, j])
              for j in range(40))
    say(f"  worst rel err vs oracle {worst:.2e}; recovery error vs x_true {rec:.2e}")
    q.free()


@pytest.mark.parametrize("fmt", ["bf16", "e4m3"])
def test_shared_batch_above_one_tile_of_rhs(fmt):
    # 300 right-hand sides: two workgroup rows of 256, the second ragged
    s_of = lambda j: 5  # noqa: E731
    say(f"shared batch 300 rhs {fmt}")
    q, A, Y, X, res = _shared_batch(fmt, 200, 520, 300, s_of, seed=12)
    worst = _check_against_oracle(A, Y, X, res, s_of, range(300))
    say(f"  worst rel err {worst:.2e}")
    q.free()


def test_shared_single_problem_dense():
    s_of = lambda j: 10  # noqa: E731
    q, A, Y, X, res = _shared_batch("bf16", 256, 1024, 1, s_of, seed=13)
    _check_against_oracle(A, Y, X, res, s_of, [0])
    # the single-problem entry point on the same handle
    x, sup, info = qiht.niht_solve(q, _t(Y[:, 0]), 10, max_iters=ITERS, tol=-1.0)
    assert torch.equal(x, res[0][0]) and torch.equal(sup, res[0][1])
    q.free()


def test_dense_handles_must_be_shared():
    rng = np.random.default_rng(3)
    a = qiht.quantize_matrix(_t(rng.standard_normal((64, 100)).astype(np.float32)), qiht.BF16, 1, 0)
    b = qiht.quantize_matrix(_t(rng.standard_normal((64, 100)).astype(np.float32)), qiht.BF16, 1, 0)
    y = _t(rng.standard_normal(64))
    with pytest.raises(qiht.QihtError) as e:
        qiht.niht_solve_batched([(a, y, 4), (b, y, 4)])
    assert e.value.status_name == "UNSUPPORTED"


@pytest.mark.parametrize("fmt", list(FMTS))
def test_refit_on_dense_handle(fmt):
    rng = np.random.default_rng(21)
    m, n, s = 300, 700, 40
    phi = (rng.standard_normal((m, n)) / np.sqrt(m)).astype(np.float32)
    y = rng.standard_normal(m)
    sup = np.sort(rng.choice(n, s, replace=False)).astype(np.int32)
    q = qiht.quantize_matrix(_t(phi), FMTS[fmt], 1, 0)
    _, _, A = lp.store_matrix(phi, fmt)
    want = niht.refit(A, y, sup)
    x, z = qiht.refit(_t(sup), _t(y), q=q)
    z = z.cpu().numpy()
    assert np.linalg.norm(z - want[sup]) <= 1e-9 * np.linalg.norm(want[sup])
    np.testing.assert_array_equal(x.cpu().numpy()[sup], z.astype(np.float32))
    q.free()
