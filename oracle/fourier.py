"""Fourier-sampled measurement matrix from its definition, and its transpose
product -- test infrastructure (CPU oracle), never on the product path.

Radio-interferometric imaging (Sec. IV-B): the measurement matrix is a
function of the inner products between baseline and pixel positions.
Visibility j at baseline (u_j, v_j) samples pixel k of a side x side sky at
integer coordinates

    l_k = (k mod side) - side / 2,   m_k = (k div side) - side / 2

(side / 2 rounded down), with

    Phi_jk = exp(-2 pi i (u_j l_k + v_j m_k)).

The real form used throughout stacks [Re Phi; Im Phi] (2 n_vis rows), so for
a stacked residual r = [r_re; r_im] the gradient is

    g_k = sum_j cos(2 pi th_jk) r_re_j - sin(2 pi th_jk) r_im_j,
    th_jk = u_j l_k + v_j m_k.

Sec. IV-C notes that such a Phi can be computed on the fly instead of being
read from memory; this module is the plain FP64 definition the on-the-fly
kernel is checked against.  Everything is FP64 (numpy cos/sin of the phase).
"""

import numpy as np


def pixel_coords(side):
    """(l, m) integer coordinates of the side * side pixels, row-major."""
    k = np.arange(side * side)
    return (k % side) - side // 2, (k // side) - side // 2


def phase(uv, side, cols=None):
    """th_jk = u_j l_k + v_j m_k (FP64), n_vis x len(cols)."""
    uv = np.asarray(uv, dtype=np.float64)
    lk, mk = pixel_coords(side)
    if cols is not None:
        lk, mk = lk[cols], mk[cols]
    return np.outer(uv[:, 0], lk) + np.outer(uv[:, 1], mk)


def stacked_matrix(uv, side, cols=None):
    """The real form [Re Phi; Im Phi] (2 n_vis x len(cols)) in FP64."""
    th = 2.0 * np.pi * phase(uv, side, cols)
    return np.concatenate([np.cos(th), -np.sin(th)], axis=0)


def gradient(uv, side, r, cols=None, block=512):
    """g = [Re Phi; Im Phi]^T r over the pixels `cols` (all by default),
    FP64, the matrix built block by block from its definition."""
    uv = np.asarray(uv, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    nv = uv.shape[0]
    assert r.shape == (2 * nv,)
    cols = np.arange(side * side) if cols is None else np.asarray(cols)
    g = np.empty(len(cols))
    for c0 in range(0, len(cols), block):
        cc = cols[c0:c0 + block]
        th = 2.0 * np.pi * phase(uv, side, cc)
        g[c0:c0 + block] = np.cos(th).T @ r[:nv] - np.sin(th).T @ r[nv:]
    return g
