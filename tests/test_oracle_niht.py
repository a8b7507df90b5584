"""Pins for the oracle's NIHT / QIHT (``oracle.niht``).

Each test checks the oracle against a fact fixed by the paper or by
mathematics, not against a retyped copy of its own formulas:

* H_s against its defining property (brute force over index pairs) on
  tie-heavy integer vectors;
* the step size against closed forms (orthonormal columns give mu = 1) and
  the Rayleigh bounds 1/sigma_max^2 <= mu <= 1/sigma_min^2 of the appendix;
* the backtracking rule against three hand-derived 2x2 cases;
* the whole solve against lstsq (s = n), the closed-form optimum for
  orthonormal columns, exact noiseless recovery, brute force over all
  supports (n <= 20), the monotone cost of the convergence theorem, and the
  unbiased double-sampled gradient of Sec. III-A.
"""

import itertools

import numpy as np
import pytest

from oracle import niht
from oracle import quantizer as qz


def _defining_property(a, sup, s):
    a = np.abs(np.asarray(a, dtype=np.float64))
    sup = list(sup)
    assert len(sup) == s and len(set(sup)) == s
    assert sup == sorted(sup)
    inside = set(sup)
    for i in sup:
        for j in range(a.size):
            if j in inside:
                continue
            assert a[i] > a[j] or (a[i] == a[j] and i < j)


@pytest.mark.parametrize("seed", range(20))
def test_hard_threshold_brute_force_ties(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    a = rng.integers(-3, 4, size=n).astype(np.float64)  # many ties, zeros
    for s in range(0, n + 1):
        sup = niht.hard_threshold_support(a, s)
        _defining_property(a, sup, s)
        x, sup2 = niht.hard_threshold(a, s)
        np.testing.assert_array_equal(sup, sup2)
        np.testing.assert_array_equal(x[sup], a[sup])
        assert np.count_nonzero(np.delete(x, sup)) == 0


def test_hard_threshold_matches_python_sort():
    rng = np.random.default_rng(7)
    a = np.round(rng.standard_normal(500), 1)
    for s in (1, 10, 100, 499):
        want = sorted(sorted(range(a.size), key=lambda j: (-abs(a[j]), j))[:s])
        assert list(niht.hard_threshold_support(a, s)) == want


def _orthonormal(m, n, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    return q


def test_step_size_orthonormal_is_one():
    q = _orthonormal(50, 20, 0)
    g = np.random.default_rng(1).standard_normal(20)
    sup = np.array([1, 4, 7, 9])
    mu, num, den = niht.step_size(g, sup, q, q)
    assert abs(mu - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_step_size_rayleigh_bounds(seed):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((30, 60))
    g = rng.standard_normal(60)
    sup = np.sort(rng.choice(60, 8, replace=False))
    mu, _, _ = niht.step_size(g, sup, phi, phi)
    sv = np.linalg.svd(phi[:, sup], compute_uv=False)
    assert 1 / sv[0] ** 2 * (1 - 1e-12) <= mu <= 1 / sv[-1] ** 2 * (1 + 1e-12)


def test_step_size_denominator_fallback():
    # Phi2 = -Phi1 makes the cross denominator negative: fall back to
    # |Phi1_G g_G|^2, i.e. the single-realization step.
    rng = np.random.default_rng(3)
    p1 = rng.standard_normal((10, 6))
    g = rng.standard_normal(6)
    sup = np.array([0, 2])
    mu_neg, _, _ = niht.step_size(g, sup, p1, -p1)
    mu_same, _, _ = niht.step_size(g, sup, p1, p1, mu_mode="same")
    assert mu_neg == mu_same > 0


def test_omega_closed_form():
    phi = np.diag([1.0, 2.0])
    dx = np.array([-0.5, 2.0])
    assert abs(niht.omega(dx, phi) - 4.25 / 16.25) < 1e-15
    assert niht.omega(np.zeros(2), np.zeros((2, 2))) == np.inf


# Hand-derived backtracking cases, n = m = 2, s = 1, state x = (0.5, 0),
# support {0}, k = 2, c = 0.01 (shrink factor k(1-c) = 1.98).
def test_backtracking_identity_one_shrink_keeps_new_support():
    # Phi = I, y = (1, 2): g = (0.5, 2), mu0 = 1, proposal (0, 2) changes
    # support, omega = 1 > ... so mu0 = 1 > 0.99 -> shrink to 1/1.98;
    # a = (0.5 + 0.5/1.98, 2/1.98) still picks index 1, omega = 1 and
    # 1/1.98 <= 0.99: accept with one shrink.
    phi = np.eye(2)
    res = niht.qiht_iteration(phi, phi, np.array([1.0, 2.0]),
                              np.array([0.5, 0.0]), np.array([0]), 1)
    assert res.mu0 == 1.0 and res.backtracks == 1 and res.changed
    assert abs(res.mu - 1 / 1.98) < 1e-15
    np.testing.assert_allclose(res.x, [0.0, 2 / 1.98], rtol=1e-15)
    assert list(res.support) == [1]


def test_backtracking_identity_returns_to_old_support():
    # Phi = I, y = (1, 1.2): mu0 = 1 proposes index 1; after one shrink
    # a = (0.5 + 0.5/1.98, 1.2/1.98) = (0.7525, 0.6061) keeps index 0.
    phi = np.eye(2)
    res = niht.qiht_iteration(phi, phi, np.array([1.0, 1.2]),
                              np.array([0.5, 0.0]), np.array([0]), 1)
    assert res.backtracks == 1 and list(res.support) == [0]
    np.testing.assert_allclose(res.x, [0.5 + 0.5 / 1.98, 0.0], rtol=1e-15)


def test_backtracking_two_shrinks():
    # Phi = diag(1, 2), y = (1, 1): g = (0.5, 2), mu0 = 1.
    # mu = 1:      a = (1, 2), dx = (-0.5, 2), omega = 4.25/16.25 = 0.2615
    # mu = 1/1.98: a = (0.7525, 1.0101), omega = 1.2703/4.3312 = 0.2933
    #              and 0.505 > 0.99 * 0.2933 -> shrink again
    # mu = 1/1.98^2: a = (0.6275, 0.5102) keeps index 0: accept.
    phi = np.diag([1.0, 2.0])
    res = niht.qiht_iteration(phi, phi, np.array([1.0, 1.0]),
                              np.array([0.5, 0.0]), np.array([0]), 1)
    assert res.backtracks == 2 and list(res.support) == [0]
    assert abs(res.mu - 1 / 1.98 ** 2) < 1e-15
    np.testing.assert_allclose(res.x, [0.5 + 0.5 / 1.98 ** 2, 0.0], rtol=1e-14)


def test_backtracking_cap():
    phi = np.diag([1.0, 2.0])
    res = niht.qiht_iteration(phi, phi, np.array([1.0, 1.0]),
                              np.array([0.5, 0.0]), np.array([0]), 1,
                              max_backtracks=1)
    assert res.backtracks == 1 and res.capped
    assert list(res.support) == [1]


def test_full_support_converges_to_lstsq():
    # s = n: H_s is the identity, the support never changes and NIHT is
    # steepest descent with exact line search -> the least-squares solution.
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((40, 10))
    y = rng.standard_normal(40)
    res = niht.qiht_solve(phi, phi, y, 10, max_iters=5000, tol=1e-15)
    want = np.linalg.lstsq(phi, y, rcond=None)[0]
    np.testing.assert_allclose(res.x, want, rtol=1e-9, atol=1e-12)
    assert res.backtracks == 0


def test_orthonormal_columns_one_step_optimum():
    # Orthonormal columns: mu = 1 and x1 = H_s(Phi^T y), which is the exact
    # minimizer of |y - Phi x| over s-sparse x; the next gradient vanishes
    # on the support, so the solve stops as stationary after one iteration.
    q = _orthonormal(64, 24, 5)
    y = np.random.default_rng(6).standard_normal(64)
    res = niht.qiht_solve(q, q, y, 5, max_iters=50)
    want, sup = niht.hard_threshold(q.T @ y, 5)
    np.testing.assert_allclose(res.x, want, rtol=1e-12, atol=1e-14)
    # the second gradient is zero on the support up to rounding
    assert res.iterations <= 2 and res.reason in (niht.REASON_STATIONARY,
                                                  niht.REASON_CONVERGED)
    assert abs(res.mu_last - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_noiseless_exact_recovery(seed):
    rng = np.random.default_rng(seed)
    m, n, s = 64, 256, 4
    phi = rng.standard_normal((m, n)) / np.sqrt(m)
    x = np.zeros(n)
    sup = np.sort(rng.choice(n, s, replace=False))
    x[sup] = rng.standard_normal(s)
    res = niht.qiht_solve(phi, phi, phi @ x, s, max_iters=2000, tol=1e-14)
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)
    assert list(res.support) == list(sup)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_support_small_n(seed):
    # n <= 20: the l0-constrained least squares (Eq. cost_function) solved by
    # enumerating all C(n, s) supports equals the NIHT support.
    rng = np.random.default_rng(100 + seed)
    m, n, s = 14, 18, 3
    phi = rng.standard_normal((m, n)) / np.sqrt(m)
    x = np.zeros(n)
    sup = rng.choice(n, s, replace=False)
    x[sup] = rng.choice([-1, 1], s) * (1 + rng.random(s))
    y = phi @ x + 1e-3 * rng.standard_normal(m)
    best, best_sup = np.inf, None
    for cand in itertools.combinations(range(n), s):
        cand = list(cand)
        z = np.linalg.lstsq(phi[:, cand], y, rcond=None)[0]
        cost = np.sum((y - phi[:, cand] @ z) ** 2)
        if cost < best:
            best, best_sup = cost, cand
    res = niht.qiht_solve(phi, phi, y, s, max_iters=3000, tol=1e-13)
    assert list(res.support) == best_sup
    cost = np.sum((y - phi @ res.x) ** 2)
    assert cost <= best * (1 + 1e-6) + 1e-18


@pytest.mark.parametrize("seed", range(4))
def test_monotone_cost_single_realization(seed):
    rng = np.random.default_rng(seed)
    m, n, s = 48, 200, 8
    phi = rng.standard_normal((m, n)) / np.sqrt(m)
    x = np.zeros(n)
    x[rng.choice(n, s, replace=False)] = rng.standard_normal(s)
    y = phi @ x + 0.05 * rng.standard_normal(m)
    xs = np.zeros(n)
    sup = niht.initial_support(phi, y, s)
    prev = np.sum(y ** 2)
    for _ in range(60):
        it = niht.qiht_iteration(phi, phi, y, xs, sup, s)
        xs, sup = it.x, it.support
        assert np.count_nonzero(xs) <= s
        cost = np.sum((y - phi @ xs) ** 2)
        assert cost <= prev * (1 + 1e-12)
        prev = cost


def test_double_sampled_gradient_unbiased():
    # Sec. III-A: with independent Q1(Phi), Q2(Phi) and Q(y),
    # E[Q1^T (Q(y) - Q2 x)] = Phi^T (y - Phi x).
    rng = np.random.default_rng(11)
    m, n = 24, 12
    phi = rng.standard_normal((m, n))
    y = rng.standard_normal(m)
    x = rng.standard_normal(n)
    want = phi.T @ (y - phi @ x)
    R = 3000
    samples = np.empty((R, n))
    for r in range(R):
        c1, s1 = qz.quantize(phi.reshape(-1, order="F"), 2, r, 0, 0)
        c2, s2 = qz.quantize(phi.reshape(-1, order="F"), 2, r, 0, 1)
        cy, sy = qz.quantize(y, 2, r, 1, 0)
        q1 = qz.dequantize(c1, s1, 2).reshape((m, n), order="F")
        q2 = qz.dequantize(c2, s2, 2).reshape((m, n), order="F")
        yh = qz.dequantize(cy, sy, 2)
        samples[r] = q1.T @ (yh - q2 @ x)
    mean = samples.mean(axis=0)
    sd = samples.std(axis=0, ddof=1) / np.sqrt(R)
    assert np.all(np.abs(mean - want) <= 5 * sd)
    # a single realization (no double sampling) is biased: E[Q^T Q] has the
    # quantization variance on its diagonal
    biased = np.empty((R, n))
    for r in range(R):
        c1, s1 = qz.quantize(phi.reshape(-1, order="F"), 2, r, 0, 0)
        cy, sy = qz.quantize(y, 2, r, 1, 0)
        q1 = qz.dequantize(c1, s1, 2).reshape((m, n), order="F")
        biased[r] = q1.T @ (qz.dequantize(cy, sy, 2) - q1 @ x)
    assert np.any(np.abs(biased.mean(axis=0) - want)
                  > 6 * biased.std(axis=0, ddof=1) / np.sqrt(R))


def test_refit_noiseless_exact():
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((30, 80))
    x = np.zeros(80)
    sup = np.array([3, 17, 50])
    x[sup] = [1.0, -2.0, 0.5]
    z = niht.refit(phi, phi @ x, sup)
    np.testing.assert_allclose(z, x, atol=1e-12)


def test_qiht_256x1024_quality():
    # Config-1 recipe: the quantized solve recovers the true support; the
    # 8-bit error floor is small (Sec. IV-A: >= 5 bits is close to NIHT).
    import workloads
    p = workloads.gaussian_256x1024(0)
    q1 = qz.dequantized_matrix(p.phi, 8, p.seed, 0)
    q2 = qz.dequantized_matrix(p.phi, 8, p.seed, 1)
    yh = qz.dequantized_vector(p.y, 8, p.seed)
    res = niht.qiht_solve(q1, q2, yh, p.s, max_iters=300, tol=1e-8)
    assert list(res.support) == list(p.support)
    err = np.linalg.norm(res.x - p.x_true) / np.linalg.norm(p.x_true)
    assert err < 0.05


def test_argument_checks():
    phi = np.eye(3)
    with pytest.raises(ValueError):
        niht.qiht_solve(phi, phi, np.ones(3), 0)
    with pytest.raises(ValueError):
        niht.qiht_solve(phi, phi, np.ones(3), 4)
    with pytest.raises(ValueError):
        niht.qiht_solve(phi, phi[:2], np.ones(3), 1)


def test_synthetic_recipe():
    # the synthetic experiment's draws: shapes, unit-variance entries,
    # reproducible per (s, trial), and the stated SNR (|Phi x|^2 / m sigma^2)
    import workloads
    p = workloads.synthetic(16, 3)
    q = workloads.synthetic(16, 3)
    assert p.phi.shape == (128, 1024) and p.s == 16 and p.seed == 3
    np.testing.assert_array_equal(p.phi, q.phi)
    np.testing.assert_allclose(p.y, p.phi @ p.x_true, rtol=1e-12, atol=1e-12)
    assert abs(p.phi.std() - 1.0) < 0.01
    assert set(np.nonzero(p.x_true)[0]) == set(p.support)
    e = workloads.synthetic(16, 3, equal=True)
    assert np.all(e.x_true[e.support] == 1.0)
    snrs = []
    for t in range(40):
        d = workloads.synthetic(16, t, snr_db=10.0)
        clean = d.phi @ d.x_true
        snrs.append(10 * np.log10(np.sum(clean ** 2) / np.sum((d.y - clean) ** 2)))
    assert abs(np.mean(snrs) - 10.0) < 0.5


def test_fresh_realizations_solver():
    # Algorithm 2 with realizations drawn per iteration: at 32 bits (no
    # randomness) it is the fixed-realization solve; at 4 bits consecutive
    # iterations see different draws, and iteration 1 is the fixed solve's
    # first iteration on realizations 0 and 1 with y_hat realization 0
    import workloads
    from oracle import quantizer as qzz
    p = workloads.gaussian(60, 150, 5, 1e-3, seed=3)
    f32 = niht.qiht_solve_fresh(p.phi, p.y, p.s, 32, 32, 7, max_iters=25, tol=-1.0)
    a = qzz.dequantized_matrix(p.phi, 32, 7, 0)
    ref = niht.qiht_solve(a, a, qzz.dequantized_vector(p.y, 32, 7), p.s, max_iters=25, tol=-1.0)
    np.testing.assert_array_equal(f32.support, ref.support)
    np.testing.assert_array_equal(f32.x, ref.x)
    assert f32.backtracks == ref.backtracks
    one = niht.qiht_solve_fresh(p.phi, p.y, p.s, 4, 8, 7, max_iters=1, tol=-1.0)
    q1 = qzz.dequantized_matrix(p.phi, 4, 7, 0)
    q2 = qzz.dequantized_matrix(p.phi, 4, 7, 1)
    yh = qzz.dequantized_vector(p.y, 8, 7)
    fixed = niht.qiht_solve(q1, q2, yh, p.s, max_iters=1, tol=-1.0)
    np.testing.assert_array_equal(one.x, fixed.x)
    assert not np.array_equal(qzz.dequantized_vector(p.y, 8, 7, realization=1), yh)
    assert not np.array_equal(qzz.dequantized_matrix(p.phi, 4, 7, 2), q1)


def test_step_size_zero_fallback_is_stationary():
    # The second fallback of the step size (reading N3): the cross
    # denominator is not positive and |Phi1_G g_G|^2 is 0 as well, with
    # g_G != 0.  Two identical support columns and g_G = (1, -1) give
    # Phi1_G g_G = 0 exactly, so no step exists: stationary (mu = None).
    phi = np.zeros((4, 3))
    phi[:, 0] = phi[:, 1] = [1.0, -2.0, 0.5, 3.0]
    phi[:, 2] = [0.0, 1.0, 0.0, 0.0]
    g = np.array([1.0, -1.0, 5.0])
    mu, num, den = niht.step_size(g, np.array([0, 1]), phi, phi)
    assert mu is None and num == 2.0 and den == 0.0
    mu, num, den = niht.step_size(g, np.array([0, 1]), phi, -phi)
    assert mu is None and num == 2.0 and den == 0.0
    # the third column alone (a unit column with g = 5) has the step 1
    mu, _, _ = niht.step_size(g, np.array([2]), phi, phi)
    assert mu == 1.0


def test_stationary_when_gradient_vanishes_on_support():
    # With g = Phi1^T r the second fallback coincides with g_G = 0: if
    # Phi1_G g_G = 0 then |g_G|^2 = g_G^T Phi1_G^T r = (Phi1_G g_G)^T r = 0,
    # so in exact arithmetic an iteration reaches it only as g_G = 0.  A state
    # whose residual is orthogonal to the support columns (unit columns and
    # zero observations there) stops at once, with the warm-start iterate.
    phi = np.zeros((5, 4))
    phi[0, 0] = phi[1, 1] = 1.0
    phi[2:, 2] = [1.0, 2.0, 0.0]
    phi[2:, 3] = [0.0, 1.0, 1.0]
    y = np.array([0.0, 0.0, 1.0, 2.0, 3.0])
    res = niht.qiht_solve(phi, phi, y, 2, max_iters=10, tol=-1.0,
                          x0=np.zeros(4), support0=np.array([0, 1]))
    assert res.reason == niht.REASON_STATIONARY and res.iterations == 0
    np.testing.assert_array_equal(res.x, np.zeros(4))
    # the same data from x0 = 0 without the warm start moves off at once
    res = niht.qiht_solve(phi, phi, y, 2, max_iters=10, tol=-1.0)
    assert res.reason != niht.REASON_STATIONARY and res.iterations >= 1


def test_fresh_draw_indices_per_iteration():
    # Algorithm 2's inputs: iteration n uses Phi_hat_{2n-1} for Phi^T,
    # Phi_hat_{2n} for Phi and y_hat_n, i.e. matrix realizations 2n-2 and
    # 2n-1 and vector realization n-1 (0-based).  Chain three iterations by
    # hand from those realizations and compare with the solver, for every
    # prefix; a shifted index map (realizations n-1 and n) gives another x.
    import workloads
    p = workloads.gaussian(80, 200, 5, 1e-3, seed=11)
    seed = 5

    def dm(r):
        return qz.dequantized_matrix(p.phi, 4, seed, r)

    def dv(r):
        return qz.dequantized_vector(p.y, 8, seed, realization=r)

    x = np.zeros(p.n)
    sup = niht.initial_support(dm(0), dv(0), p.s)
    shifted_x = x.copy()
    shifted_sup = sup.copy()
    for it in range(1, 4):
        ref = niht.qiht_iteration(dm(2 * it - 2), dm(2 * it - 1), dv(it - 1), x, sup, p.s)
        x, sup = ref.x, ref.support
        got = niht.qiht_solve_fresh(p.phi, p.y, p.s, 4, 8, seed, max_iters=it, tol=-1.0)
        assert got.iterations == it
        np.testing.assert_array_equal(got.support, sup)
        np.testing.assert_array_equal(got.x, x)
        wrong = niht.qiht_iteration(dm(it - 1), dm(it), dv(it - 1), shifted_x, shifted_sup, p.s)
        shifted_x, shifted_sup = wrong.x, wrong.support
        if it >= 2:
            assert not np.array_equal(shifted_x, x)


def test_two_bit_divergence_and_its_cause():
    # Fixed realizations at 2 bits on a Gaussian Phi (max-abs scale: the
    # quantization noise is about three times the signal): Q1_G^T Q2_G loses
    # positive definiteness on the support, the cross step-size denominator
    # turns non-positive (the fallback of reading N3 is taken) and the
    # iterate grows without bound.  The same instance at 8 bits converges
    # and Q1_G^T Q2_G stays positive definite on every support.
    import workloads
    m, n, s = 1024, 4096, 64
    p = workloads.gaussian(m, n, s, 1e-3, seed=0, dtype=np.float32)
    yh = qz.dequantized_vector(p.y, 8, p.seed)
    out = {}
    for bits in (2, 8):
        q1 = qz.dequantized_matrix(p.phi, bits, p.seed, 0)
        q2 = qz.dequantized_matrix(p.phi, bits, p.seed, 1)
        x = np.zeros(n)
        sup = niht.initial_support(q1, yh, s)
        min_eig, fallbacks = np.inf, 0
        for _ in range(100):
            a = q1[:, sup].T @ q2[:, sup]
            min_eig = min(min_eig, np.linalg.eigvalsh(0.5 * (a + a.T)).min())
            g = q1.T @ (yh - q2 @ x)
            fallbacks += float((q1[:, sup] @ g[sup]) @ (q2[:, sup] @ g[sup])) <= 0.0
            res = niht.qiht_iteration(q1, q2, yh, x, sup, s)
            assert not res.stationary
            x, sup = res.x, res.support
        err = np.linalg.norm(x - p.x_true) / np.linalg.norm(p.x_true)
        out[bits] = (err, min_eig, fallbacks)
    err2, eig2, fb2 = out[2]
    err8, eig8, fb8 = out[8]
    assert err2 > 100.0 and eig2 < 0.0 and fb2 >= 1
    assert err8 < 0.02 and eig8 > 0.3 and fb8 == 0
