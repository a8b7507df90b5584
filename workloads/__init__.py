"""Seeded synthetic inputs for the QIHT hot path.

This module only draws problem instances y = Phi x + e (Eq. CS_model); it
holds none of the method's arithmetic (no quantization, no thresholding, no
step sizes).  Both the CPU oracle and the GPU path are fed the very same
arrays from here.

Recipes (numpy PCG64 ``default_rng``; draw order per instance is
Phi -> support -> nonzero values -> noise):

* ``gaussian``: Phi (m x n) i.i.d. N(0, 1/m) in FP64 or FP32; x s-sparse,
  support uniform without replacement, nonzeros N(0, 1) (or all ones for the
  equal-magnitude variant of the synthetic experiments); e ~ N(0, sigma^2).
* ``complex_gaussian``: complex Phi (m x n) with i.i.d. circular complex
  Gaussian entries of variance 1/m, an s-sparse complex x with circular
  complex N(0, 1) nonzeros, circular complex noise (a complex unknown).
* ``interferometry``: complex Phi_jk = exp(-2 pi i (u_j l_k + v_j m_k)) with
  (u_j, v_j) uniform in a disk of radius 0.5 and integer pixel coordinates
  l, m in [-side/2, side/2); real sky x with s point sources of log-uniform
  flux in [0.1, 10]; complex noise at a given SNR
  10 log10(|Phi x|^2 / |e|^2) (the definition used for the radio-astronomy
  experiment).  Stands in for the telescope data of the paper, which are not
  available.  ``complex_sky`` gives each source a uniform phase as well (a
  complex unknown on the same matrix).
* ``interferometry_visibilities``: the same draws without the matrix (uv,
  the sky and the stacked visibilities), for Phi computed on the fly.
* ``batch_uneven``: independent Gaussian problems with m drawn uniformly in
  [m_lo, m_hi], n = 4m, s = m // 16, per-instance generator seeds [seed, i].
* ``shared_phi``: one Gaussian Phi and many sparse right-hand sides.
* ``synthetic``: the synthetic experiment of Sec. IV-A: Phi 128 x 1024 with
  i.i.d. N(0, 1) entries (unit variance, as stated there), s-sparse x with
  N(0, 1) or all-one nonzeros, y = Phi x, or with noise at a given SNR
  (|Phi x|^2 / |e|^2, in dB); generator seeds [seed, s, trial].
"""

from dataclasses import dataclass
import math

import numpy as np


@dataclass
class Problem:
    phi: np.ndarray        # (m, n) real or complex, row-major
    y: np.ndarray          # (m,)
    x_true: np.ndarray     # (n,) real (complex for a complex unknown)
    support: np.ndarray    # (s,) sorted true support
    s: int
    seed: int              # the quantizer seed for this instance

    @property
    def m(self):
        return self.phi.shape[0]

    @property
    def n(self):
        return self.phi.shape[1]


def gaussian(m, n, s, sigma_e=1e-3, seed=0, dtype=np.float64, equal=False,
             qseed=None):
    """Real Gaussian instance: Phi m x n N(0, 1/m), an s-sparse signal, noise sigma_e."""
    rng = np.random.default_rng(seed)
    if np.dtype(dtype) == np.float32:
        phi = rng.standard_normal((m, n), dtype=np.float32)
        phi *= np.float32(1.0 / math.sqrt(m))
    else:
        phi = rng.standard_normal((m, n)) * (1.0 / math.sqrt(m))
    sup = np.sort(rng.choice(n, s, replace=False))
    x = np.zeros(n)
    x[sup] = 1.0 if equal else rng.standard_normal(s)
    e = sigma_e * rng.standard_normal(m) if sigma_e > 0 else np.zeros(m)
    y = _matvec(phi, x) + e
    return Problem(phi, y, x, sup, s, seed if qseed is None else qseed)


def _matvec(phi, x):
    """Phi x in FP64, in row blocks (Phi may be FP32 and large)."""
    nz = np.flatnonzero(x)
    out = np.zeros(phi.shape[0], dtype=np.result_type(phi.dtype, np.float64)
                   if not np.iscomplexobj(phi) else np.complex128)
    step = 4096
    for r0 in range(0, phi.shape[0], step):
        blk = phi[r0:r0 + step][:, nz]
        blk = blk.astype(np.complex128 if np.iscomplexobj(blk) else np.float64)
        out[r0:r0 + step] = blk @ x[nz]
    return out


def synthetic(s, trial, equal=False, snr_db=None, seed=0, m=128, n=1024):
    """One draw of the synthetic experiment (Sec. IV-A): Phi m x n N(0, 1),
    x s-sparse (N(0, 1) or, with ``equal``, all-one nonzeros), y = Phi x,
    plus N(0, sigma^2) noise with |Phi x|^2 / (m sigma^2) = 10^(snr_db/10)
    when ``snr_db`` is given.  The quantizer seed is the trial index."""
    rng = np.random.default_rng([seed, s, trial])
    phi = rng.standard_normal((m, n))
    sup = np.sort(rng.choice(n, s, replace=False))
    x = np.zeros(n)
    x[sup] = 1.0 if equal else rng.standard_normal(s)
    y = _matvec(phi, x)
    if snr_db is not None:
        sigma = np.linalg.norm(y) / math.sqrt(m) * 10.0 ** (-snr_db / 20.0)
        y = y + sigma * rng.standard_normal(m)
    return Problem(phi, y, x, sup, s, trial)


def gaussian_256x1024(seed=0):
    """Phi 256 x 1024 FP64 N(0, 1/256), s = 16, sigma_e = 1e-3."""
    return gaussian(256, 1024, 16, 1e-3, seed, np.float64)


def gaussian_8192x32768(seed=0, m=8192, n=32768, s=512):
    """Phi 8192 x 32768 FP32 N(0, 1/8192), s = 512, sigma_e = 1e-3."""
    return gaussian(m, n, s, 1e-3, seed, np.float32)


def complex_gaussian(m, n, s, sigma_e=1e-3, seed=0, dtype=np.complex64):
    """Complex instance with a complex unknown: Phi m x n with i.i.d.
    circular complex Gaussian entries of variance 1/m (real and imaginary
    parts N(0, 1/(2m))), an s-sparse x with circular complex N(0, 1)
    nonzeros, and circular complex noise of standard deviation sigma_e."""
    rng = np.random.default_rng(seed)
    sc = 1.0 / math.sqrt(2.0 * m)
    phi = (rng.standard_normal((m, n)) * sc + 1j * (rng.standard_normal((m, n)) * sc)).astype(dtype)
    sup = np.sort(rng.choice(n, s, replace=False))
    x = np.zeros(n, dtype=np.complex128)
    x[sup] = (rng.standard_normal(s) + 1j * rng.standard_normal(s)) / math.sqrt(2.0)
    e = sigma_e / math.sqrt(2.0) * (rng.standard_normal(m) + 1j * rng.standard_normal(m))
    y = _matvec(phi, x) + e
    return Problem(phi, y, x, sup, s, seed)


def interferometry(n_vis=32640, side=128, s=200, snr_db=30.0, seed=0,
                   dtype=np.complex64, complex_sky=False):
    """Fourier-sampled complex instance: n_vis visibilities of a side x side
    sky image (32640 x 16384 at the defaults), s point sources.  With
    ``complex_sky`` every source also gets a phase uniform in [0, 2 pi) (drawn
    after the noise), a complex unknown on the same matrix."""
    rng = np.random.default_rng(seed)
    rad = 0.5 * np.sqrt(rng.random(n_vis))
    th = 2.0 * np.pi * rng.random(n_vis)
    u = rad * np.cos(th)
    v = rad * np.sin(th)
    k = np.arange(side * side)
    lk = (k % side) - side // 2
    mk = (k // side) - side // 2
    n = side * side
    phi = np.empty((n_vis, n), dtype=dtype)
    step = 1024
    for r0 in range(0, n_vis, step):
        ph = np.outer(u[r0:r0 + step], lk) + np.outer(v[r0:r0 + step], mk)
        phi[r0:r0 + step] = np.exp(-2j * np.pi * ph)
    sup = np.sort(rng.choice(n, s, replace=False))
    x = np.zeros(n)
    x[sup] = 10.0 ** rng.uniform(-1.0, 1.0, s)
    clean = _matvec(phi, x)
    sig2 = float(np.vdot(clean, clean).real) / (n_vis * 10.0 ** (snr_db / 10.0))
    e = math.sqrt(sig2 / 2.0) * (rng.standard_normal(n_vis)
                                 + 1j * rng.standard_normal(n_vis))
    y = clean + e
    if complex_sky:
        x = x * np.exp(2j * np.pi * rng.random(n))
        x[np.setdiff1d(np.arange(n), sup)] = 0.0
        clean = _matvec(phi, x)
        y = clean + e
    p = Problem(phi, y, x, sup, s, seed)
    p.uv = np.stack([u, v], axis=1)
    p.lm = np.stack([lk, mk], axis=1)
    return p


def interferometry_visibilities(n_vis=32640, side=128, s=200, snr_db=30.0, seed=0):
    """The draws of ``interferometry`` (same order: baselines, support,
    fluxes, noise) without forming Phi: uv (n_vis, 2), the sky x, and the
    stacked visibilities y = [Re; Im] (2 n_vis, FP64), with Phi x evaluated
    over the s sources only.  For the kernels that compute Phi on the fly."""
    rng = np.random.default_rng(seed)
    rad = 0.5 * np.sqrt(rng.random(n_vis))
    th = 2.0 * np.pi * rng.random(n_vis)
    uv = np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)
    n = side * side
    sup = np.sort(rng.choice(n, s, replace=False))
    x = np.zeros(n)
    x[sup] = 10.0 ** rng.uniform(-1.0, 1.0, s)
    lk = (sup % side) - side // 2
    mk = (sup // side) - side // 2
    clean = np.zeros(n_vis, dtype=np.complex128)
    for t in range(s):
        clean += x[sup[t]] * np.exp(-2j * np.pi * (uv[:, 0] * lk[t] + uv[:, 1] * mk[t]))
    sig2 = float(np.vdot(clean, clean).real) / (n_vis * 10.0 ** (snr_db / 10.0))
    e = math.sqrt(sig2 / 2.0) * (rng.standard_normal(n_vis) + 1j * rng.standard_normal(n_vis))
    y = clean + e
    return uv, np.concatenate([y.real, y.imag]), x, sup


def batch_uneven(count=96, m_lo=1024, m_hi=8192, seed=0, sigma_e=1e-3,
                 dtype=np.float32):
    """Uneven independent Gaussian problems: m uniform in [m_lo, m_hi],
    n = 4m, s = m/16."""
    master = np.random.default_rng(seed)
    ms = master.integers(m_lo, m_hi + 1, size=count)
    probs = []
    for i, m in enumerate(ms):
        m = int(m)
        p = gaussian(m, 4 * m, max(1, m // 16), sigma_e, [seed, i], dtype,
                     qseed=i)
        probs.append(p)
    return probs


def shared_phi(m=8192, n=32768, nrhs=256, s=256, sigma_e=1e-3, seed=0,
               dtype=np.float32, equal=False):
    """One Gaussian Phi shared by nrhs sparse right-hand sides.

    ``s`` is the sparsity of every signal, or a sequence of nrhs sparsities;
    ``equal`` sets every nonzero to 1 (no draw) instead of N(0, 1).
    Returns (phi, Y (m, nrhs), X (n, nrhs), supports list)."""
    s_list = [int(s)] * nrhs if np.isscalar(s) else [int(v) for v in s]
    rng = np.random.default_rng(seed)
    if np.dtype(dtype) == np.float32:
        phi = rng.standard_normal((m, n), dtype=np.float32)
        phi *= np.float32(1.0 / math.sqrt(m))
    else:
        phi = rng.standard_normal((m, n)) * (1.0 / math.sqrt(m))
    X = np.zeros((n, nrhs))
    sups = []
    for j in range(nrhs):
        sup = np.sort(rng.choice(n, s_list[j], replace=False))
        X[sup, j] = 1.0 if equal else rng.standard_normal(s_list[j])
        sups.append(sup)
    E = sigma_e * rng.standard_normal((m, nrhs))
    Y = np.zeros((m, nrhs))
    for j in range(nrhs):
        Y[:, j] = _matvec(phi, X[:, j])
    return phi, Y + E, X, sups
