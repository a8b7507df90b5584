"""Pins for the oracle's stochastic quantizer (``oracle.quantizer``).

Sec. III-A defines Q(v, b): 2^b equispaced levels in [-1, 1], randomized
rounding to one of the two neighbours with the probability that makes
E[Q(v)] = v.  The appendix lemma on the quantized vector bounds
E|Q(v) - v| by c sqrt(M) / 2^(b-1) and its proof uses the per-element
variance (q_{j+1} - v)(v - q_j).  These tests check those facts directly,
plus the level search done a second way (by scanning the level list).
"""

import numpy as np
import pytest

from oracle import quantizer as qz


def _vec(n, seed=0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v[0] = np.abs(v).max() * 1.5      # the max-abs element, positive
    v[1] = -v[0]                      # and its negative
    v[2] = 0.0
    return v


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5, 6, 7, 8, 12])
def test_codes_are_a_neighbouring_level(bits):
    v = _vec(5000, bits)
    codes, c = qz.quantize(v, bits, 11, 0, 0)
    L = qz.num_levels(bits)
    assert codes.min() >= 0 and codes.max() <= L - 1
    assert c == np.abs(v).max()
    # independent level search: scan the level list scaled by c
    lev = qz.level_values(bits) * c
    lo = np.searchsorted(lev, v, side="right") - 1
    lo = np.clip(lo, 0, L - 2)
    assert np.all((codes == lo) | (codes == lo + 1))
    # a value lying strictly inside (q_i, q_i+1) never lands elsewhere
    deq = qz.dequantize(codes, c, bits)
    assert np.all(deq >= lev[lo] - 1e-12 * c)
    assert np.all(deq <= lev[lo + 1] + 1e-12 * c)


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5, 7, 8])
def test_endpoints_are_deterministic(bits):
    v = _vec(64, 1)
    L = qz.num_levels(bits)
    for real in range(50):
        codes, c = qz.quantize(v, bits, real, 0, real)
        assert codes[0] == L - 1
        assert codes[1] == 0


def test_one_bit_levels_are_plus_minus_c():
    v = _vec(1000, 2)
    codes, c = qz.quantize(v, 1, 3, 0, 1)
    deq = qz.dequantize(codes, c, 1)
    assert set(np.unique(deq)) <= {-c, c}


def test_level_values_equispaced():
    for bits in (1, 2, 3, 4, 5, 6, 7, 8):
        lev = qz.level_values(bits)
        assert lev[0] == -1.0 and lev[-1] == 1.0
        assert lev.size == 2 ** bits
        np.testing.assert_allclose(np.diff(lev), 2.0 / (2 ** bits - 1),
                                   rtol=1e-12)
    odd = qz.level_values(4, odd=True)
    assert odd.size == 9
    np.testing.assert_allclose(np.diff(odd), 1.0 / 2 ** (4 - 2))


def test_zero_vector():
    codes, c = qz.quantize(np.zeros(10), 4, 0, 0, 0)
    assert c == 0.0 and np.all(codes == 0)
    assert np.all(qz.dequantize(codes, c, 4) == 0.0)


def _realizations(v, bits, R, seed=21):
    out = np.empty((R, v.size))
    for r in range(R):
        codes, c = qz.quantize(v, bits, seed, 0, r)
        out[r] = qz.dequantize(codes, c, bits)
    return out, c


@pytest.mark.parametrize("bits", [2, 3, 4, 5])
def test_unbiased_with_exact_variance(bits):
    """E[Q(v)] = v (Sec. III-A) and Var = (q_{j+1} - v)(v - q_j)."""
    v = _vec(256, 3)
    R = 4096
    samp, c = _realizations(v, bits, R)
    lev = qz.level_values(bits) * c
    L = lev.size
    lo = np.clip(np.searchsorted(lev, v, side="right") - 1, 0, L - 2)
    var = (lev[lo + 1] - v) * (v - lev[lo])
    var = np.maximum(var, 0.0)
    mean = samp.mean(axis=0)
    tol = 5.0 * np.sqrt(var / R) + 1e-12 * c
    assert np.all(np.abs(mean - v) <= tol)
    # the variance itself: sample variance within ~6 sd of its estimator
    sv = samp.var(axis=0, ddof=1)
    inner = var > 1e-6 * c * c
    # Bernoulli-scaled variance: sd of sample variance <= var*sqrt(2/R)*~3
    assert np.all(np.abs(sv[inner] - var[inner])
                  <= 6 * np.sqrt(2.0 / R) * np.maximum(var[inner],
                                                       (lev[1] - lev[0]) ** 2 / 4))


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 5, 6, 7, 8])
def test_lemma_error_bound(bits):
    """E|Q(v) - v| <= c sqrt(M) / 2^(b-1) (appendix lemma)."""
    v = _vec(512, 4)
    samp, c = _realizations(v, bits, 256)
    err = np.linalg.norm(samp - v[None, :], axis=1).mean()
    assert err <= c * np.sqrt(v.size) / 2 ** (bits - 1)


def test_round_up_frequency_matches_fraction():
    """A single value a fraction f above a level rounds up with prob. f."""
    bits, c = 3, 1.0
    L = 8
    lev = qz.level_values(bits)
    f = 0.3
    val = lev[2] + f * (lev[3] - lev[2])
    v = np.full(200000, val)
    v[0] = c  # fixes the scale at exactly 1
    codes, _ = qz.quantize(v, bits, 5, 0, 0)
    k = codes[1:]
    assert set(np.unique(k)) <= {2, 3}
    p = np.mean(k == 3)
    assert abs(p - f) < 6 * np.sqrt(f * (1 - f) / k.size)


def test_matrix_order_is_column_major_and_stacks_complex():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((7, 5)) + 1j * rng.standard_normal((7, 5))
    codes, c = qz.quantize_matrix(a, 4, 9, 1)
    assert codes.shape == (14, 5)
    st = np.concatenate([a.real, a.imag], axis=0)
    ref, c2 = qz.quantize(st.reshape(-1, order="F"), 4, 9, qz.STREAM_MATRIX, 1)
    assert c == c2 == np.abs(st).max()
    np.testing.assert_array_equal(codes, ref.reshape((14, 5), order="F"))
    # realizations are independent draws
    codes2, _ = qz.quantize_matrix(a, 4, 9, 0)
    assert np.any(codes2 != codes)


def test_fp32_path_is_rounding_only():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((6, 4))
    q, c = qz.quantize_matrix(a, 32, 0, 0)
    assert c is None
    np.testing.assert_array_equal(q, a.astype(np.float32).astype(np.float64))


def test_nonfinite_rejected():
    with pytest.raises(ValueError):
        qz.quantize(np.array([1.0, np.nan]), 4, 0, 0, 0)
