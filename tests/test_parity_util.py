"""CPU checks of the parity helpers (``tests/parity_util.py``): the threaded
oracle matrices equal the oracle's whole-matrix quantizer, and the
comparison functions reject planted mistakes that the bars are meant to
catch."""

import numpy as np
import pytest

import workloads
from oracle import niht
from oracle import quantizer as qz
from parity_util import TieLog, assert_g_elementwise, check_step, g_bound, oracle_matrix


@pytest.mark.parametrize("bits", [2, 4, 8, 32])
def test_oracle_matrix_equals_whole_matrix_quantizer(bits):
    p = workloads.gaussian(70, 1300, 5, 1e-3, seed=4, dtype=np.float32)
    for r in (0, 1):
        a = oracle_matrix(p.phi, bits, p.seed, r, block=128)
        np.testing.assert_array_equal(a, qz.dequantized_matrix(p.phi, bits, p.seed, r))


def test_oracle_matrix_complex_and_odd():
    p = workloads.interferometry(n_vis=90, side=20, s=4, seed=3)
    a = oracle_matrix(p.phi, 4, p.seed, 1, block=64)
    np.testing.assert_array_equal(a, qz.dequantized_matrix(p.phi, 4, p.seed, 1))
    a = oracle_matrix(p.phi, 4, p.seed, 0, odd=True, block=100)
    np.testing.assert_array_equal(a, qz.dequantized_matrix(p.phi, 4, p.seed, 0, odd=True))


def test_elementwise_bar_catches_one_wrong_entry():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((400, 3000))
    r = rng.standard_normal(400)
    g = q.T @ r
    bound = g_bound(q, r)
    np.testing.assert_allclose(bound, np.abs(q).T @ np.abs(r), rtol=1e-14)
    assert_g_elementwise(g * (1 + 1e-7), g, bound)
    bad = g.copy()
    bad[17] += 2e-5 * bound[17]
    # a norm-wise bar of 1e-5 |g| would accept this entry
    assert np.linalg.norm(bad - g) <= 1e-5 * np.linalg.norm(g)
    with pytest.raises(AssertionError):
        assert_g_elementwise(bad, g, bound)


def _state():
    p = workloads.gaussian(120, 400, 6, 1e-3, seed=9)
    q1 = qz.dequantized_matrix(p.phi, 8, p.seed, 0)
    q2 = qz.dequantized_matrix(p.phi, 8, p.seed, 1)
    yh = qz.dequantized_vector(p.y, 8, p.seed)
    x = np.zeros(p.n)
    sup = niht.initial_support(q1, yh, p.s)
    for _ in range(3):
        r = niht.qiht_iteration(q1, q2, yh, x, sup, p.s)
        x, sup = r.x.astype(np.float32).astype(np.float64), r.support
    return p, q1, q2, yh, x, sup


def test_check_step_accepts_the_oracle_and_rejects_mistakes():
    p, q1, q2, yh, x, sup = _state()
    ref = niht.qiht_iteration(q1, q2, yh, x, sup, p.s)
    g0n = float(np.linalg.norm(q1.T @ yh))
    info = dict(backtracks=ref.backtracks, mu_last=ref.mu)
    ties = TieLog()
    check_step(q1, q2, yh, x, sup, p.s, ref.x.astype(np.float32), ref.support, info, g0n, ties, "ok")
    assert ties.count == 0
    # a wrong support entry (a clear loser swapped in)
    a = np.abs(x + ref.mu * ref.g)
    loser = int(np.argsort(a)[0])
    wrong = np.sort(np.concatenate([ref.support[1:], [loser]]))
    xw = np.zeros_like(ref.x)
    xw[wrong] = 1.0
    with pytest.raises(AssertionError):
        check_step(q1, q2, yh, x, sup, p.s, xw, wrong, info, g0n, ties, "support")
    # a wrong step
    with pytest.raises(AssertionError):
        check_step(q1, q2, yh, x, sup, p.s, ref.x, ref.support,
                   dict(backtracks=ref.backtracks, mu_last=ref.mu * 1.01), g0n, ties, "mu")
    # a wrong shrink count
    with pytest.raises(AssertionError):
        check_step(q1, q2, yh, x, sup, p.s, ref.x, ref.support,
                   dict(backtracks=ref.backtracks + 3, mu_last=ref.mu), g0n, ties, "shrinks")
