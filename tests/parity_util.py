"""Helpers of the GPU parity tests (test infrastructure; calls only the
oracle and the workload generators, never the HIP path).

* ``oracle_matrix``: the oracle's dequantized realization of Q(Phi) in FP64,
  quantized column block by column block on host threads (the element
  order, Philox counters and scale are those of
  ``oracle.quantizer.quantize_matrix``; only the work is split).
* ``g_bound`` / ``assert_g_elementwise``: the element-wise gradient bar
  |g_gpu_j - g_j| <= rel * sum_i |q_ij r_i| (each entry of g is a sum of
  products; this bounds the error of each entry by the size of its own
  terms, so a few wrong entries cannot hide in a norm).
* ``check_step``: one warm-started GPU iteration against the oracle's
  iteration from the same state.  Identical supports, equal shrink counts,
  the accepted step within 2e-5 (floored as the gradient bar) and x within
  1e-5 relative.  Where a decision of the iteration is a near-tie (the s-th
  and (s+1)-th |x + mu g| of a proposal, or mu against (1 - c) omega, within
  ``tie`` relative), either outcome is correct: the GPU's outcome is then
  checked to be one the iteration may take, and the comparison continues
  from the GPU's state.
"""

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import niht
from oracle import quantizer as qz


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def _stacked_block(phi, j0, j1):
    blk = phi[:, j0:j1]
    if np.iscomplexobj(blk):
        return np.concatenate([blk.real, blk.imag], axis=0).astype(np.float64)
    return blk.astype(np.float64)


def stacked_absmax(phi, block=1024):
    """max |Phi_ij| over the stacked real matrix (the quantizer's scale)."""
    def part(j0):
        return float(np.max(np.abs(_stacked_block(phi, j0, min(phi.shape[1], j0 + block)))))
    with ThreadPoolExecutor(workers()) as ex:
        return max(ex.map(part, range(0, phi.shape[1], block)))


def oracle_matrix(phi, bits, seed, realization, odd=False, scale=None, block=512):
    """FP64 dequantized realization of Q(Phi, b) (stacked rows), Fortran order.

    bits == 32: the FP32-rounded stacked matrix."""
    n = phi.shape[1]
    rows = phi.shape[0] * (2 if np.iscomplexobj(phi) else 1)
    out = np.empty((rows, n), dtype=np.float64, order="F")
    c = None
    if int(bits) != 32:
        c = stacked_absmax(phi) if scale is None else float(scale)

    def fill(j0):
        j1 = min(n, j0 + block)
        a = _stacked_block(phi, j0, j1)
        if int(bits) == 32:
            out[:, j0:j1] = a.astype(np.float32).astype(np.float64)
            return
        codes, _ = qz.quantize(a.reshape(-1, order="F"), bits, seed, qz.STREAM_MATRIX,
                               realization, odd=odd, e_offset=j0 * rows, scale=c)
        out[:, j0:j1] = qz.dequantize(codes, c, bits, odd).reshape((rows, j1 - j0), order="F")

    with ThreadPoolExecutor(workers()) as ex:
        list(ex.map(fill, range(0, n, block)))
    return out


def g_bound(q1, r, block=2048):
    """sum_i |q_ij| |r_i| for every column j."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    n = q1.shape[1]
    out = np.empty(n)

    def part(j0):
        j1 = min(n, j0 + block)
        out[j0:j1] = np.abs(q1[:, j0:j1]).T @ r

    with ThreadPoolExecutor(workers()) as ex:
        list(ex.map(part, range(0, n, block)))
    return out


def assert_g_elementwise(g_gpu, g_ref, bound, rel=1e-5, what="g"):
    """|g_gpu - g_ref| <= rel * bound entry by entry (bound = g_bound or a
    sample of it); returns the largest ratio |dg| / bound."""
    g_gpu = np.asarray(g_gpu, dtype=np.float64)
    d = np.abs(g_gpu - g_ref)
    lim = rel * np.asarray(bound) + 1e-300
    bad = np.flatnonzero(d > lim)
    assert bad.size == 0, (f"{what}: {bad.size} entries outside the bar, e.g. j={bad[:5]} "
                           f"|dg|={d[bad[:5]]} bar={lim[bad[:5]]}")
    return float(np.max(d / lim) * rel)


class TieLog:
    """Counts the near-tie decisions a comparison accepted."""

    def __init__(self):
        self.count = 0
        self.notes = []

    def add(self, note):
        self.count += 1
        self.notes.append(note)


def _margin_topk(a, s):
    """Relative gap between the s-th and (s+1)-th largest |a| (inf if s = n)."""
    v = np.sort(np.abs(a))[::-1]
    if s >= v.size:
        return np.inf
    return (v[s - 1] - v[s]) / max(v[s - 1], 1e-300)


def _support_near(a, s, sup_a, sup_b, tie):
    """Two supports differ only by entries whose |a| lie within `tie` of the
    s-th largest |a|."""
    if np.array_equal(sup_a, sup_b):
        return True
    va = np.abs(a)
    t = np.sort(va)[::-1][s - 1]
    diff = np.setxor1d(sup_a, sup_b)
    return bool(np.all(np.abs(va[diff] - t) <= tie * max(t, 1e-300)))


def _trials(phi1, x, sup, g, mu0, s, k, c, cap):
    """The oracle iteration's trials: per shrink count t the step, the
    proposal's support, whether it keeps the old support, omega and the
    decision margins."""
    out = []
    mu = mu0
    for t in range(cap + 1):
        if t > 0:
            mu = mu / (k * (1.0 - c))
        a = x + mu * g
        sn = niht.hard_threshold_support(a, s)
        xn = np.zeros_like(x)
        xn[sn] = a[sn]
        changed = not np.array_equal(sn, sup)
        om = niht.omega(xn - x, phi1) if changed else np.inf
        out.append(dict(mu=mu, a=a, sup=sn, x=xn, changed=changed, omega=om,
                        margin_sel=_margin_topk(a, s),
                        margin_test=(abs(mu - (1.0 - c) * om) / mu) if changed else np.inf))
    return out


def check_step(phi1, phi2, yhat, x_prev, sup_prev, s, gpu_x, gpu_sup, gpu_info, g0norm,
               ties, label, k=2.0, c=0.01, cap=32, mu_mode="cross", tie=2e-5):
    """Compare one GPU iteration from (x_prev, sup_prev) with the oracle's.

    x_prev is the FP32 state the GPU started from (as FP64).  Returns the
    oracle's IterationResult."""
    ref = niht.qiht_iteration(phi1, phi2, yhat, x_prev, sup_prev, s, k=k, c=c,
                              max_backtracks=cap, mu_mode=mu_mode)
    assert not ref.stationary, label
    gs = np.asarray(gpu_sup)
    xg = np.asarray(gpu_x, dtype=np.float64)
    assert np.count_nonzero(np.delete(xg, gs)) == 0, label
    # the accepted step: a ratio of quadratic forms in g_G, so twice the
    # gradient's relative bar, floored like it
    gG = np.linalg.norm(ref.g[sup_prev])
    mu_tol = 2e-5 * max(1.0, 1e-3 * g0norm / max(gG, 1e-300))
    same = (np.array_equal(gs, ref.support) and gpu_info["backtracks"] == ref.backtracks)
    if same:
        assert abs(gpu_info["mu_last"] - ref.mu) <= mu_tol * ref.mu, \
            (label, gpu_info["mu_last"], ref.mu)
        err = np.linalg.norm(xg - ref.x) / max(np.linalg.norm(ref.x), 1e-300)
        assert err <= 1e-5, (label, err)
        return ref
    # A different outcome is correct only through near-ties: every trial
    # before the GPU's shrink count either continues in the oracle too or
    # sits on a tie, and at the GPU's shrink count the proposal (up to
    # near-tied swaps) may be accepted.
    b = gpu_info["backtracks"]
    assert 0 <= b <= cap, label
    tr = _trials(phi1, x_prev, sup_prev, ref.g, ref.mu0, s, k, c, max(b, ref.backtracks))
    for t in range(b):
        stops = (not tr[t]["changed"]) or tr[t]["mu"] <= (1.0 - c) * tr[t]["omega"]
        near = tr[t]["margin_sel"] <= tie or tr[t]["margin_test"] <= tie
        assert (not stops) or near, (label, "GPU shrank past a clear stop", t)
    last = tr[b]
    stops = (not last["changed"]) or last["mu"] <= (1.0 - c) * last["omega"] or b == cap
    near = last["margin_sel"] <= tie or last["margin_test"] <= tie
    assert stops or near, (label, "GPU stopped where the test clearly fails", b)
    assert _support_near(last["a"], s, gs, last["sup"], tie), (label, "support beyond a tie")
    assert abs(gpu_info["mu_last"] - last["mu"]) <= mu_tol * last["mu"], label
    ties.add(f"{label}: GPU {b} shrinks / oracle {ref.backtracks}, "
             f"support {'same' if np.array_equal(gs, ref.support) else 'near-tied'}")
    return ref


def chain_oracle(phi1, phi2, yhat, s, iters, k=2.0, c=0.01, cap=32, mu_mode="cross"):
    """The oracle's iterations from x = 0 with x rounded to FP32 between
    iterations (the state a GPU solver holds); returns (x, support,
    iterations, shrinks)."""
    x = np.zeros(phi1.shape[1])
    sup = niht.initial_support(phi1, yhat, s)
    its = bts = 0
    for _ in range(iters):
        r = niht.qiht_iteration(phi1, phi2, yhat, x.astype(np.float32).astype(np.float64), sup, s,
                                k=k, c=c, max_backtracks=cap, mu_mode=mu_mode)
        if r.stationary:
            break
        its += 1
        bts += r.backtracks
        x, sup = r.x, r.support
    return x, sup, its, bts
