"""Pins of the complex-x oracle (oracle/complex_niht.py) against things other
than itself: the real oracle on real data, the invariances the problem has
under phases (which a missing conjugation breaks), brute force over all
supports on tiny noiseless problems, the orthonormal-column closed form, and
hand-built ties of the modulus threshold."""

import itertools

import numpy as np
import pytest

from oracle import complex_niht as cn
from oracle import niht


def _cgauss(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def _problem(m, n, s, seed, noise=1e-3):
    rng = np.random.default_rng(seed)
    phi = _cgauss(rng, (m, n)) / np.sqrt(m)
    x = np.zeros(n, dtype=np.complex128)
    sup = np.sort(rng.choice(n, s, replace=False))
    x[sup] = _cgauss(rng, s)
    y = phi @ x + noise * _cgauss(rng, m)
    return phi, x, sup, y


def test_modulus_threshold_ties_and_order():
    a = np.array([3.0, 4j, -5.0, 3 + 4j, 1.0, -0.5j])
    assert list(cn.hard_threshold_support(a, 2)) == [2, 3]      # |.| = 5, 5
    assert list(cn.hard_threshold_support(a, 1)) == [2]         # tie -> lower index
    assert list(cn.hard_threshold_support(a, 3)) == [1, 2, 3]   # then 4i
    # ranking by modulus, not by real part
    b = np.array([2.0, 0.1 + 3j, -1.0])
    assert list(cn.hard_threshold_support(b, 1)) == [1]
    x, sup = cn.hard_threshold(a, 2)
    assert np.array_equal(x, [0, 0, -5.0, 3 + 4j, 0, 0])


def test_real_data_reduces_to_the_real_oracle():
    rng = np.random.default_rng(5)
    m, n, s = 60, 200, 6
    q1 = rng.standard_normal((m, n)) / np.sqrt(m)
    q2 = q1 + 0.05 * rng.standard_normal((m, n)) / np.sqrt(m)
    xt = np.zeros(n)
    xt[rng.choice(n, s, replace=False)] = rng.standard_normal(s)
    y = q1 @ xt + 1e-3 * rng.standard_normal(m)
    rr = niht.qiht_solve(q1, q2, y, s, max_iters=80, tol=1e-10)
    rc = cn.qiht_solve(q1.astype(complex), q2.astype(complex), y.astype(complex), s,
                       max_iters=80, tol=1e-10)
    assert np.array_equal(rc.support, rr.support)
    assert rc.iterations == rr.iterations and rc.backtracks == rr.backtracks
    assert np.max(np.abs(rc.x.imag)) == 0.0
    assert np.allclose(rc.x.real, rr.x, rtol=0, atol=1e-12 * np.abs(rr.x).max())


@pytest.mark.parametrize("theta", [0.7, 2.9])
def test_phase_invariances(theta):
    """Phi -> e^{i t} Phi with y -> e^{i t} y leaves the iterates unchanged;
    y -> e^{i t} y alone rotates them by e^{i t} (moduli, supports, steps and
    backtracking unchanged)."""
    phi, _, _, y = _problem(50, 160, 5, seed=11, noise=1e-2)
    rot = np.exp(1j * theta)
    base = cn.qiht_solve(phi, phi, y, 5, max_iters=40, tol=-1.0)
    both = cn.qiht_solve(rot * phi, rot * phi, rot * y, 5, max_iters=40, tol=-1.0)
    assert np.array_equal(both.support, base.support) and both.backtracks == base.backtracks
    assert np.allclose(both.x, base.x, rtol=0, atol=1e-12)
    yrot = cn.qiht_solve(phi, phi, rot * y, 5, max_iters=40, tol=-1.0)
    assert np.array_equal(yrot.support, base.support) and yrot.backtracks == base.backtracks
    assert np.allclose(yrot.x, rot * base.x, rtol=0, atol=1e-12)


def test_planted_missing_conjugate_breaks_the_phase_pin(monkeypatch):
    """A gradient Q1^T r (no conjugation) instead of Q1^H r fails the joint
    phase invariance above (e^{i t} Phi and e^{i t} y): the pin can see that
    mistake.  (A rotation of y alone rotates such a gradient as well, so that
    invariance cannot.)"""
    phi, _, _, y = _problem(50, 160, 5, seed=11, noise=1e-2)
    rot = np.exp(0.7j)
    orig = cn.qiht_iteration

    def wrong(q1, q2, yhat, x, support, s, k=2.0, c=0.01, max_backtracks=32, mu_mode="cross"):
        return orig(q1.conj(), q2, yhat, x, support, s, k, c, max_backtracks, mu_mode)

    monkeypatch.setattr(cn, "qiht_iteration", wrong)
    base = cn.qiht_solve(phi, phi, y, 5, max_iters=40, tol=-1.0)
    both = cn.qiht_solve(rot * phi, rot * phi, rot * y, 5, max_iters=40, tol=-1.0)
    assert not np.allclose(both.x, base.x, rtol=0, atol=1e-6)


def _brute_force_support(phi, y, s):
    best, arg = np.inf, None
    for sup in itertools.combinations(range(phi.shape[1]), s):
        sup = list(sup)
        z, *_ = np.linalg.lstsq(phi[:, sup], y, rcond=None)
        res = float(np.linalg.norm(y - phi[:, sup] @ z))
        if res < best:
            best, arg = res, sup
    return np.array(arg)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_support_on_tiny_noiseless_problems(seed):
    phi, x, sup, y = _problem(14, 10, 2, seed=seed, noise=0.0)
    res = cn.qiht_solve(phi, phi, y, 2, max_iters=500, tol=1e-14)
    assert np.array_equal(res.support, _brute_force_support(phi, y, 2))
    assert np.array_equal(res.support, sup)
    assert np.linalg.norm(res.x - x) <= 1e-8 * np.linalg.norm(x)


def test_orthonormal_columns_give_unit_step_and_a_closed_form_first_iterate():
    rng = np.random.default_rng(9)
    m, n, s = 40, 24, 4
    u, _ = np.linalg.qr(_cgauss(rng, (m, m)))
    phi = u[:, :n]
    x = np.zeros(n, dtype=complex)
    x[[2, 7, 11, 20]] = [1 + 1j, -2.0, 0.5j, 1.5 - 0.5j]
    y = phi @ x + 0.01 * _cgauss(rng, m)
    g0 = phi.conj().T @ y
    sup0 = cn.initial_support(phi, y, s)
    res = cn.qiht_iteration(phi, phi, y, np.zeros(n, dtype=complex), sup0, s)
    assert abs(res.mu0 - 1.0) < 1e-12
    want, _ = cn.hard_threshold(g0, s)
    assert np.allclose(res.x, want, rtol=0, atol=1e-12)


def test_step_fallback_and_stationary():
    """A non-positive cross denominator falls back to |Q1_G g_G|^2, and a
    vanishing g_G stops the solve (the real solver's readings)."""
    q1 = np.array([[1.0 + 0j, 0.0], [0.0, 1.0]])
    q2 = -q1
    g = np.array([1.0 + 1j, 0.0])
    mu, num, den = cn.step_size(g, np.array([0]), q1, q2)
    assert num == 2.0 and den == 2.0 and mu == 1.0
    mu, _, _ = cn.step_size(np.zeros(2, dtype=complex), np.array([0]), q1, q1)
    assert mu is None
    res = cn.qiht_iteration(q1, q1, np.zeros(2, dtype=complex), np.zeros(2, dtype=complex),
                            np.array([0]), 1)
    assert res.stationary
