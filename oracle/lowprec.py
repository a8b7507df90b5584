"""Deterministic low-precision storage of Phi for the shared-Phi solve, FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper quantizes at random (``oracle.quantizer``); the shared-Phi variant
holds one Phi for many right-hand sides in a dense floating-point format
instead, and runs plain NIHT (Algorithm 1) on the stored matrix.  Readings
(listed in the design doc; the paper has no such format):

* Formats: FP32 (the plain single-precision copy), BF16 (1 sign, 8 exponent,
  7 stored significand bits) and FP8 E4M3 in the OCP form (1 sign, 4 exponent
  bits with bias 7, 3 stored significand bits, no infinities, largest finite
  value 448, subnormals down to 2^-9).
* Row scale: row i is stored as Phi_ij / 2^e_i, with e_i the smallest integer
  for which max_j |Phi_ij| / 2^e_i <= F (F = 448 for E4M3, 1 for BF16; FP32
  has no scale, e_i = 0).  A power of two makes the scaling exact, so the
  only rounding is the conversion itself.
* Conversion: round to nearest, ties to even significand, from the exact
  FP64 value; an all-zero row has e_i = 0.  Scaled values never exceed F, so
  E4M3 saturation never triggers.
* The effective matrix is A = diag(2^e) Phi~, exactly representable in FP64.
"""

import math

import numpy as np

FORMATS = ("f32", "bf16", "e4m3")

# (significand bits incl. the implicit one, smallest normal exponent, largest finite)
_SPEC = {
    "bf16": (8, -126, (2.0 - 2.0 ** -7) * 2.0 ** 127),
    "e4m3": (4, -6, 448.0),
}
_ROW_MAX = {"bf16": 1.0, "e4m3": 448.0}


def round_to(v, fmt):
    """Round FP64 values to the nearest value of `fmt` ('bf16' or 'e4m3'),
    ties to the even significand, saturating at the largest finite value.
    Returns FP64 values that the format represents exactly."""
    p, emin, vmax = _SPEC[fmt]
    v = np.asarray(v, dtype=np.float64)
    out = v.copy()
    nz = np.isfinite(v) & (v != 0.0)
    x = v[nz]
    _, e2 = np.frexp(np.abs(x))           # |x| = f 2^e2, f in [0.5, 1)
    e = np.maximum(e2 - 1, emin)          # exponent of the leading bit (clamped: subnormals)
    quantum = np.ldexp(1.0, e - (p - 1))  # spacing of representable values there
    # x / quantum is exact (a power of two); np.round rounds halves to even
    out[nz] = np.clip(np.round(x / quantum) * quantum, -vmax, vmax)
    return out


def row_exponents(phi, fmt):
    """e_i of the row scale 2^e_i (all zero for 'f32')."""
    phi = np.asarray(phi)
    if fmt == "f32":
        return np.zeros(phi.shape[0], dtype=np.int64)
    top = _ROW_MAX[fmt]
    e = np.zeros(phi.shape[0], dtype=np.int64)
    for i in range(phi.shape[0]):
        mx = float(np.max(np.abs(phi[i]))) if phi.shape[1] else 0.0
        if mx == 0.0:
            continue
        k = math.ceil(math.log2(mx / top))
        # correct the floating log at exact powers of two and just beyond
        while mx / 2.0 ** k > top:
            k += 1
        while mx / 2.0 ** (k - 1) <= top:
            k -= 1
        e[i] = k
    return e


def store_matrix(phi, fmt):
    """(stored values Phi~ as FP64, row exponents e, effective A = diag(2^e) Phi~)."""
    phi = np.asarray(phi)
    if fmt == "f32":
        st = phi.astype(np.float32).astype(np.float64)
        return st, np.zeros(phi.shape[0], dtype=np.int64), st
    e = row_exponents(phi, fmt)
    st = np.empty(phi.shape, dtype=np.float64)
    for r0 in range(0, phi.shape[0], 1024):  # row blocks bound the temporaries
        blk = phi[r0:r0 + 1024].astype(np.float64)
        # division by a power of two is exact
        st[r0:r0 + 1024] = round_to(blk / np.ldexp(1.0, e[r0:r0 + 1024])[:, None], fmt)
    return st, e, st * np.ldexp(1.0, e)[:, None]


def e4m3_byte_value(b):
    """Value of one E4M3 bit pattern (sign, 4-bit exponent with bias 7, 3-bit
    significand; exponent 0 is subnormal; S.1111.111 is NaN)."""
    s, ex, m = (b >> 7) & 1, (b >> 3) & 15, b & 7
    if ex == 15 and m == 7:
        return math.nan
    mag = (m / 8.0) * 2.0 ** -6 if ex == 0 else (1.0 + m / 8.0) * 2.0 ** (ex - 7)
    return -mag if s else mag


def e4m3_decode(codes):
    """FP64 values of an array of E4M3 bytes."""
    table = np.array([e4m3_byte_value(b) for b in range(256)])
    return table[np.asarray(codes, dtype=np.uint8)]


def e4m3_values():
    """All finite E4M3 values, ascending."""
    vals = [e4m3_byte_value(b) for b in range(256)]
    return np.array(sorted(set(v for v in vals if not math.isnan(v))))
