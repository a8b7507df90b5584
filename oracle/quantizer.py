"""Stochastic quantizer Q(v, b) of Sec. III-A ("The Algorithm"), FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What the paper fixes
--------------------
* Q maps a value in [-1, 1] to one of l = 2^b equispaced levels
  q_1 = -1 < q_2 < ... < q_l = 1 (Sec. III-A).
* A value v in [q_i, q_{i+1}] goes to q_i with probability
  (q_{i+1} - v) / (q_{i+1} - q_i) and to q_{i+1} otherwise, so E[Q(v)] = v.
* Before quantizing, a vector is divided by c_v = max_i |v_i| (appendix,
  Lemma on the quantized vector and its proof), so the values lie in [-1, 1].
* Matrices and vectors are quantized element-wise; Phi^T and Phi use two
  independent quantizations ("double sampling", Sec. III-A).

Readings where the paper is silent (listed in the design doc)
--------------------------------------------------------
* The position of v between levels is computed in FP64 as
  p = (v + c) * K with K = (l - 1) / (2c), no fused multiply-add;
  i = floor(p) clamped to [0, l - 2]; f = p - i.
* The coin is one 32-bit Philox word u (``oracle.philox``):
  code = i + [u < f * 2^32].  Both sides of the comparison are exact in
  FP64, so the probability of rounding up is f rounded down to a multiple
  of 2^-32.
* Element order is column-major over the matrix (stacked [Re; Im] rows for
  complex input); stream 0 is the matrix, stream 1 the observation vector;
  the realization index (0 = the copy used for Phi^T, 1 = the copy used for
  Phi) is the last counter word.
* c = 0 gives all codes 0 and dequantized value 0.
* b = 32 means plain single precision: Q(v) = fp32(v) (no randomness).
* ``odd=True`` selects the Remark's level set for fixed-point hardware:
  2^(b-1) + 1 levels with spacing 1 / 2^(b-2).
"""

import numpy as np

from . import philox

STREAM_MATRIX = 0
STREAM_VECTOR = 1
TWO32 = 4294967296.0


def num_levels(bits, odd=False):
    """Number of quantization levels l for a bit width."""
    bits = int(bits)
    if odd:
        if bits < 2:
            raise ValueError("odd level set needs b >= 2")
        return (1 << (bits - 1)) + 1
    return 1 << bits


def level_values(bits, odd=False):
    """The l levels q_k = -1 + 2k/(l-1), k = 0..l-1 (equispaced in [-1, 1])."""
    L = num_levels(bits, odd)
    k = np.arange(L, dtype=np.float64)
    return 2.0 * k / (L - 1) - 1.0


def quantize(v, bits, seed, stream, realization, odd=False, e_offset=0,
             scale=None):
    """Quantize a 1-D array of values given in element order.

    Returns (codes, c): integer codes in [0, l-1] and the max-abs scale c.
    The dequantized value of code k is c * (2k/(l-1) - 1).
    ``e_offset`` is the element index of v[0]; ``scale`` supplies c when v
    is only a slice of the quantized matrix (default: max |v|).
    """
    v = np.asarray(v, dtype=np.float64).reshape(-1)
    L = num_levels(bits, odd)
    codes = np.zeros(v.size, dtype=np.int64)
    if v.size == 0:
        return codes, 0.0
    if not np.all(np.isfinite(v)):
        raise ValueError("non-finite input to the quantizer")
    c = float(np.max(np.abs(v))) if scale is None else float(scale)
    if c == 0.0:
        return codes, 0.0
    K = (L - 1) / (2.0 * c)
    t = v + c
    p = t * K
    i = np.floor(p)
    i = np.minimum(np.maximum(i, 0.0), float(L - 2))
    f = p - i
    u = philox.words(seed, stream, realization, e_offset, v.size)
    up = u.astype(np.float64) < f * TWO32
    codes = i.astype(np.int64) + up.astype(np.int64)
    return codes, c


def dequantize(codes, c, bits, odd=False):
    """Level value times scale: c * (2k/(l-1) - 1), in FP64."""
    L = num_levels(bits, odd)
    k = np.asarray(codes, dtype=np.float64)
    return c * (2.0 * k / (L - 1) - 1.0)


def stack_real(a):
    """Complex rows become [Re; Im] (real problem with real unknowns)."""
    a = np.asarray(a)
    if np.iscomplexobj(a):
        return np.concatenate([a.real, a.imag], axis=0).astype(np.float64)
    return a.astype(np.float64)


def quantize_matrix(phi, bits, seed, realization, odd=False):
    """Q(Phi, b) for one realization.

    phi : (m, n) real or complex array.  Complex input is stacked [Re; Im].
    returns (codes (rows, n) int64, c) for bits < 32, or
            (fp32 values as float64 (rows, n), None) for bits == 32.
    """
    a = stack_real(phi)
    if int(bits) == 32:
        return a.astype(np.float32).astype(np.float64), None
    rows, n = a.shape
    flat = a.reshape(-1, order="F")
    codes, c = quantize(flat, bits, seed, STREAM_MATRIX, realization, odd)
    return codes.reshape((rows, n), order="F"), c


def quantize_vector(y, bits, seed, odd=False, realization=0):
    """Q(y, b): one realization on the vector stream (realization 0 unless
    the realizations of Algorithm 2 are drawn one per iteration).

    returns (codes int64, c) for bits < 32, or (fp32 values, None).
    """
    a = stack_real(np.asarray(y).reshape(-1, 1)).reshape(-1)
    if int(bits) == 32:
        return a.astype(np.float32).astype(np.float64), None
    return quantize(a, bits, seed, STREAM_VECTOR, realization, odd)


def dequantized_matrix(phi, bits, seed, realization, odd=False):
    """Convenience: the FP64 matrix Phi_hat of one realization."""
    codes, c = quantize_matrix(phi, bits, seed, realization, odd)
    if c is None:
        return codes
    return dequantize(codes, c, bits, odd)


def dequantized_vector(y, bits, seed, odd=False, realization=0):
    """Convenience: the FP64 vector y_hat."""
    codes, c = quantize_vector(y, bits, seed, odd, realization)
    if c is None:
        return codes
    return dequantize(codes, c, bits, odd)
