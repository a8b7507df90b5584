"""Normalized IHT (Algorithm 1) and QIHT (Algorithm 2) in plain FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The solver works on the dequantized FP64 matrices Phi1_hat (used for Phi^T),
Phi2_hat (used for Phi) and the observation y_hat.  With Phi1 = Phi2 = Phi and
y_hat = y it is plain normalized IHT (Algorithm 1).

What the paper fixes
--------------------
* Update x+ = H_s(x + mu g) with g = Phi1^T (y - Phi2 x), x0 = 0
  (Eq. NIHT, Eq. modified_update_rule).
* H_s keeps the s entries largest in magnitude and zeroes the rest
  (Sec. I-A, Normalized IHT paragraph).
* Step size mu = |g_G|^2 / (Phi1_G g_G)^T (Phi2_G g_G) on the current
  support G (Eq. step_size; Algorithm 2 uses the two realizations).
* If the support changes, the step must satisfy
  mu <= (1 - c) |x+ - x|^2 / |Phi (x+ - x)|^2; otherwise mu <- mu / (k(1-c))
  and a new proposal is made, with k > 1/(1-c) (Sec. II-A, step size
  determination; Algorithms 1 and 2).
* Initial support G0 = supp(H_s(Phi1^T y)) (Algorithms 1 and 2).

Readings where the paper is silent, ambiguous or garbled (listed in the design doc)
-----------------------------------------------------------------------------
* N2: iteration n evaluates g at x^[n-1] (Algorithm 2 prints x^[n] inside
  the gradient, which does not exist yet).
* N3: if the step-size denominator is <= 0 or not finite, use
  |Phi1_G g_G|^2; if |g_G| = 0, or that fallback is 0 as well, stop
  (reason STATIONARY).
* N4: H_s ties go to the lower index; the new support is the selected index
  set (always s indices, even if some selected values are zero).
* N5/N6: the "x^[n] = x^[n-1]" lines of the accept branches are read as
  "accept x^[n]" (read literally the solver never leaves x = 0).
* N7: the backtracking loop re-proposes x^[n] = H_s(x^[n-1] + mu g) with the
  shrunk mu, stops as soon as the proposal keeps the old support or satisfies
  the step test, recomputes omega with Phi1, treats |Phi1 dx| = 0 as
  omega = +inf, and is capped at ``max_backtracks`` shrinks (the last
  proposal is then accepted and the iteration counted as capped).
* N8: defaults k = 2, c = 0.01 (the paper gives neither value).
* N9: stop after iteration n when |x^[n] - x^[n-1]| <= tol |x^[n]|, or at
  ``max_iters`` (the paper only gives the iteration count n*).
* N10: optional least-squares refit of x on the final support (not in the
  paper; ``refit``).
"""

from dataclasses import dataclass, field

import numpy as np

from . import quantizer

REASON_CONVERGED = 1
REASON_MAX_ITERS = 2
REASON_STATIONARY = 3


def hard_threshold_support(a, s):
    """Indices of the s entries of a largest in magnitude, ascending.

    Order: larger |a_j| first, equal magnitudes by lower index first.
    """
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    n = a.size
    s = int(s)
    if s < 0 or s > n:
        raise ValueError("need 0 <= s <= n")
    order = np.lexsort((np.arange(n), -np.abs(a)))
    return np.sort(order[:s]).astype(np.int64)


def hard_threshold(a, s):
    """H_s(a): keep the selected entries, zero the rest.

    Returns (x, support)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    sup = hard_threshold_support(a, s)
    x = np.zeros_like(a)
    x[sup] = a[sup]
    return x, sup


def step_size(g, support, phi1, phi2, mu_mode="cross"):
    """Normalized step on support G (Eq. step_size, Algorithm 2).

    mu = |g_G|^2 / ((Phi1_G g_G) . (Phi2_G g_G)); ``mu_mode='same'`` uses
    Phi1 for both factors.  Returns (mu, num, den) with mu = None when
    |g_G| = 0.
    """
    gG = g[support]
    num = float(gG @ gG)
    if num == 0.0:
        return None, num, 0.0
    u = phi1[:, support] @ gG
    if mu_mode == "cross":
        v = phi2[:, support] @ gG
        den = float(u @ v)
    else:
        den = float(u @ u)
    if not (np.isfinite(den) and den > 0.0):
        den = float(u @ u)
    if not den > 0.0:
        return None, num, den
    return num / den, num, den


def omega(dx, phi1):
    """|dx|^2 / |Phi1 dx|^2 (the step bound of the support-change test)."""
    num = float(dx @ dx)
    w = phi1 @ dx
    den = float(w @ w)
    if den == 0.0:
        return np.inf
    return num / den


@dataclass
class IterationResult:
    """One QIHT iteration from a given state (used for teacher forcing)."""
    g: np.ndarray
    mu0: float            # step before backtracking (None if stationary)
    mu: float             # accepted step
    x: np.ndarray         # accepted x^[n]
    support: np.ndarray   # accepted support G^[n]
    backtracks: int
    capped: bool
    changed: bool         # proposal support differed from G^[n-1]
    stationary: bool


def qiht_iteration(phi1, phi2, yhat, x, support, s, k=2.0, c=0.01,
                   max_backtracks=32, mu_mode="cross"):
    """One iteration of Algorithm 2 from state (x^[n-1], G^[n-1])."""
    x = np.asarray(x, dtype=np.float64)
    support = np.asarray(support, dtype=np.int64)
    r = yhat - phi2 @ x
    g = phi1.T @ r
    mu, _, _ = step_size(g, support, phi1, phi2, mu_mode)
    if mu is None:
        return IterationResult(g, None, None, x.copy(), support.copy(),
                               0, False, False, True)
    mu0 = mu
    xn, sn = hard_threshold(x + mu * g, s)
    changed = not np.array_equal(sn, support)
    nb = 0
    capped = False
    if changed:
        w = omega(xn - x, phi1)
        while mu > (1.0 - c) * w:
            if nb >= max_backtracks:
                capped = True
                break
            mu = mu / (k * (1.0 - c))
            nb += 1
            xn, sn = hard_threshold(x + mu * g, s)
            if np.array_equal(sn, support):
                break
            w = omega(xn - x, phi1)
    return IterationResult(g, mu0, mu, xn, sn, nb, capped, changed, False)


@dataclass
class SolveResult:
    x: np.ndarray
    support: np.ndarray
    iterations: int
    reason: int
    backtracks: int
    capped_iterations: int
    mu_last: float
    trace: list = field(default_factory=list)


def initial_support(phi1, yhat, s):
    """G0 = supp(H_s(Phi1^T y_hat)) (Algorithms 1 and 2)."""
    return hard_threshold_support(phi1.T @ yhat, s)


def qiht_solve(phi1, phi2, yhat, s, max_iters=300, tol=1e-8, k=2.0, c=0.01,
               max_backtracks=32, mu_mode="cross", x0=None, support0=None,
               record=False):
    """Algorithm 2 (QIHT) on fixed realizations; Algorithm 1 when
    phi1 is phi2 and yhat is the unquantized y."""
    phi1 = np.asarray(phi1, dtype=np.float64)
    phi2 = np.asarray(phi2, dtype=np.float64)
    yhat = np.asarray(yhat, dtype=np.float64).reshape(-1)
    m, n = phi1.shape
    if phi2.shape != (m, n) or yhat.size != m:
        raise ValueError("shape mismatch")
    if not (1 <= s <= min(m, n)):
        raise ValueError("need 1 <= s <= min(m, n)")
    if x0 is None:
        x = np.zeros(n)
        sup = initial_support(phi1, yhat, s)
    else:
        x = np.asarray(x0, dtype=np.float64).copy()
        sup = np.sort(np.asarray(support0, dtype=np.int64))
    reason = REASON_MAX_ITERS
    it = 0
    total_bt = 0
    capped_its = 0
    mu_last = 0.0
    trace = []
    for it in range(1, max_iters + 1):
        res = qiht_iteration(phi1, phi2, yhat, x, sup, s, k, c,
                             max_backtracks, mu_mode)
        if res.stationary:
            it -= 1
            reason = REASON_STATIONARY
            break
        dx = float(np.linalg.norm(res.x - x))
        x, sup = res.x, res.support
        mu_last = res.mu
        total_bt += res.backtracks
        capped_its += int(res.capped)
        if record:
            trace.append(dict(mu0=res.mu0, mu=res.mu, backtracks=res.backtracks,
                              changed=res.changed, dx=dx,
                              xnorm=float(np.linalg.norm(x)),
                              support=sup.copy()))
        if dx <= tol * float(np.linalg.norm(x)):
            reason = REASON_CONVERGED
            break
    return SolveResult(x, sup, it, reason, total_bt, capped_its, mu_last, trace)


def qiht_solve_fresh(phi, y, s, bits, ybits, seed, max_iters=300, tol=1e-8, k=2.0,
                     c=0.01, max_backtracks=32, mu_mode="cross", x_fp32=False):
    """Algorithm 2 as its input states: 2n* realizations of Q(Phi) and n* of
    Q(y).  Iteration n uses Phi_hat_{2n-1} for Phi^T and Phi_hat_{2n} for
    Phi (matrix realizations 2n-2 and 2n-1) and y_hat_n (vector realization
    n-1); the initial support uses Phi_hat_1 and y_hat_1.  Realizations are
    drawn per iteration, not per trial of the step size: backtracking within
    an iteration reuses them.  ``x_fp32`` rounds x to FP32 between iterations
    (the state the GPU solver holds)."""
    def draws(it):
        q1 = quantizer.dequantized_matrix(phi, bits, seed, 2 * (it - 1))
        q2 = quantizer.dequantized_matrix(phi, bits, seed, 2 * (it - 1) + 1)
        yh = quantizer.dequantized_vector(y, ybits, seed, realization=it - 1)
        return q1, q2, yh
    q1, q2, yh = draws(1)
    n = q1.shape[1]
    if not (1 <= s <= min(q1.shape)):
        raise ValueError("need 1 <= s <= min(m, n)")
    x = np.zeros(n)
    sup = initial_support(q1, yh, s)
    reason = REASON_MAX_ITERS
    it = 0
    total_bt = capped_its = 0
    mu_last = 0.0
    for it in range(1, max_iters + 1):
        if it > 1:
            q1, q2, yh = draws(it)
        xs = x.astype(np.float32).astype(np.float64) if x_fp32 else x
        res = qiht_iteration(q1, q2, yh, xs, sup, s, k, c, max_backtracks, mu_mode)
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


def refit(phi, yhat, support):
    """Least-squares refit of x on a fixed support: argmin |y - Phi_G z|."""
    support = np.asarray(support, dtype=np.int64)
    z, *_ = np.linalg.lstsq(phi[:, support], yhat, rcond=None)
    x = np.zeros(phi.shape[1])
    x[support] = z
    return x
