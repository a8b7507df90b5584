"""QIHT with a complex unknown x, in plain complex FP64 (complex128).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The problem of Sec. I-A with Phi in C^{M x N} and x in C^N (the general case
the paper states; the MRI images of Sec. IV are complex): minimize
|y - Phi x|^2 subject to |x|_0 <= s, solved by Algorithm 2 on two
quantizations Q1, Q2 of Phi and one of y.  Written directly in complex
arithmetic (this module never forms a real embedding of the problem):

* g = Q1^H (y_hat - Q2 x), with ^H the conjugate transpose (Sec. I-A notation);
* H_s keeps the s entries of largest modulus |a_j| (ties to the lower index);
* mu = |g_G|^2 / Re((Q1_G g_G)^H (Q2_G g_G)) -- the real part of the Hermitian
  form, which is real when Q1 = Q2; the same fallback as the real solver
  (reading N3): a denominator <= 0 or not finite is replaced by |Q1_G g_G|^2,
  and |g_G| = 0 stops the solve;
* the support-change test mu <= (1 - c)|x+ - x|^2 / |Q1 (x+ - x)|^2 and the
  shrinking by k(1 - c) of Sec. II-A, with the real solver's readings N5-N9.

The quantized complex matrix is Q(Re Phi) + i Q(Im Phi): the codes of the
stacked real matrix [Re Phi; Im Phi] (Q9), one scale for both parts.
"""

import numpy as np

from .niht import (REASON_CONVERGED, REASON_MAX_ITERS, REASON_STATIONARY,
                   IterationResult, SolveResult)


def complex_from_stacked(a):
    """[Re A; Im A] (2m x n real) -> A (m x n complex)."""
    a = np.asarray(a)
    m = a.shape[0] // 2
    return a[:m] + 1j * a[m:]


def hard_threshold_support(a, s):
    """Indices of the s entries of a largest in modulus, ascending (larger
    |a_j| first, equal moduli by lower index)."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    n = a.size
    if not 0 <= s <= n:
        raise ValueError("need 0 <= s <= n")
    order = np.lexsort((np.arange(n), -np.abs(a)))
    return np.sort(order[:s]).astype(np.int64)


def hard_threshold(a, s):
    """H_s(a) for complex a -> (x, support)."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    sup = hard_threshold_support(a, s)
    x = np.zeros_like(a)
    x[sup] = a[sup]
    return x, sup


def step_size(g, support, q1, q2, mu_mode="cross"):
    """mu = |g_G|^2 / Re((Q1_G g_G)^H (Q2_G g_G)) -> (mu or None, num, den)."""
    gG = g[support]
    num = float(np.vdot(gG, gG).real)
    if num == 0.0:
        return None, num, 0.0
    u = q1[:, support] @ gG
    uu = float(np.vdot(u, u).real)
    den = float(np.vdot(u, q2[:, support] @ gG).real) if mu_mode == "cross" else uu
    if not (np.isfinite(den) and den > 0.0):
        den = uu
    if not den > 0.0:
        return None, num, den
    return num / den, num, den


def omega(dx, q1):
    """|dx|^2 / |Q1 dx|^2 (+inf when Q1 dx = 0)."""
    num = float(np.vdot(dx, dx).real)
    w = q1 @ dx
    den = float(np.vdot(w, w).real)
    return np.inf if den == 0.0 else num / den


def qiht_iteration(q1, q2, yhat, x, support, s, k=2.0, c=0.01, max_backtracks=32,
                   mu_mode="cross"):
    """One iteration of Algorithm 2 from (x^[n-1], G^[n-1]), complex x."""
    x = np.asarray(x, dtype=np.complex128)
    support = np.asarray(support, dtype=np.int64)
    g = q1.conj().T @ (yhat - q2 @ x)
    mu, _, _ = step_size(g, support, q1, q2, mu_mode)
    if mu is None:
        return IterationResult(g, None, None, x.copy(), support.copy(), 0, False, False, True)
    mu0 = mu
    xn, sn = hard_threshold(x + mu * g, s)
    changed = not np.array_equal(sn, support)
    nb, capped = 0, False
    if changed:
        w = omega(xn - x, q1)
        while mu > (1.0 - c) * w:
            if nb >= max_backtracks:
                capped = True
                break
            mu = mu / (k * (1.0 - c))
            nb += 1
            xn, sn = hard_threshold(x + mu * g, s)
            if np.array_equal(sn, support):
                break
            w = omega(xn - x, q1)
    return IterationResult(g, mu0, mu, xn, sn, nb, capped, changed, False)


def initial_support(q1, yhat, s):
    """G0 = supp H_s(Q1^H y_hat)."""
    return hard_threshold_support(q1.conj().T @ yhat, s)


def qiht_solve(q1, q2, yhat, s, max_iters=300, tol=1e-8, k=2.0, c=0.01, max_backtracks=32,
               mu_mode="cross", x_fp32=False):
    """Algorithm 2 with a complex unknown on fixed realizations Q1, Q2
    (complex m x n) and y_hat (complex m).  ``x_fp32`` rounds the real and
    imaginary parts of x to FP32 between iterations (the state a GPU solver
    holds)."""
    q1 = np.asarray(q1, dtype=np.complex128)
    q2 = np.asarray(q2, dtype=np.complex128)
    yhat = np.asarray(yhat, dtype=np.complex128).reshape(-1)
    m, n = q1.shape
    if q2.shape != (m, n) or yhat.size != m:
        raise ValueError("shape mismatch")
    if not 1 <= s <= min(m, n):
        raise ValueError("need 1 <= s <= min(m, n)")
    x = np.zeros(n, dtype=np.complex128)
    sup = initial_support(q1, yhat, s)
    reason, it, total_bt, capped_its, mu_last = REASON_MAX_ITERS, 0, 0, 0, 0.0
    for it in range(1, max_iters + 1):
        xs = x
        if x_fp32:
            xs = x.real.astype(np.float32).astype(np.float64) + \
                1j * x.imag.astype(np.float32).astype(np.float64)
        res = qiht_iteration(q1, q2, yhat, xs, sup, s, k, c, max_backtracks, mu_mode)
        if res.stationary:
            it -= 1
            reason = REASON_STATIONARY
            break
        dx = float(np.linalg.norm(res.x - xs))
        x, sup = res.x, res.support
        mu_last = res.mu
        total_bt += res.backtracks
        capped_its += int(res.capped)
        if dx <= tol * float(np.linalg.norm(x)):
            reason = REASON_CONVERGED
            break
    return SolveResult(x, sup, it, reason, total_bt, capped_its, mu_last, [])
