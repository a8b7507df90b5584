"""Pins of the Fourier-sampled gradient oracle (oracle/fourier.py) against
what the definition fixes, independently of the oracle's own formula:

* the complex product Re(Phi^H y) with Phi built by complex exponentials
  (brute force on a tiny sky);
* the interferometry workload generator's own Phi (its pixel layout and
  sign convention);
* the dirty-beam peak: for r the stacked column k of Phi, g_k = n_vis
  exactly and |g_k'| <= n_vis everywhere (Cauchy-Schwarz); a dropped or
  flipped sine term breaks the peak;
* translation invariance of the dirty beam: the beam of a source at k1
  seen at k1 + d equals that of a source at k2 seen at k2 + d.
"""

import numpy as np

import workloads
from oracle import fourier


def _uv(nv, seed):
    rng = np.random.default_rng(seed)
    rad = 0.5 * np.sqrt(rng.random(nv))
    th = 2.0 * np.pi * rng.random(nv)
    return np.stack([rad * np.cos(th), rad * np.sin(th)], axis=1)


def test_matches_complex_adjoint_brute_force():
    side, nv = 6, 17
    uv = _uv(nv, 1)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(nv) + 1j * rng.standard_normal(nv)
    phi = np.empty((nv, side * side), dtype=np.complex128)
    for j in range(nv):
        for k in range(side * side):
            lk, mk = k % side - side // 2, k // side - side // 2
            phi[j, k] = np.exp(-2j * np.pi * (uv[j, 0] * lk + uv[j, 1] * mk))
    want = (np.conj(phi).T @ y).real
    got = fourier.gradient(uv, side, np.concatenate([y.real, y.imag]))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_matches_the_workload_generator():
    p = workloads.interferometry(n_vis=300, side=16, s=5, seed=4, dtype=np.complex128)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(600)
    A = np.concatenate([p.phi.real, p.phi.imag], axis=0)
    want = A.T @ r
    np.testing.assert_allclose(fourier.gradient(p.uv, 16, r), want, rtol=0,
                               atol=1e-11 * np.abs(want).max())
    np.testing.assert_allclose(fourier.stacked_matrix(p.uv, 16), A, rtol=0, atol=1e-12)


def test_dirty_beam_peak_and_bound():
    side, nv = 12, 400
    uv = _uv(nv, 7)
    for k in (0, 77, side * side - 1):
        lk, mk = k % side - side // 2, k // side - side // 2
        e = np.exp(-2j * np.pi * (uv[:, 0] * lk + uv[:, 1] * mk))
        g = fourier.gradient(uv, side, np.concatenate([e.real, e.imag]))
        assert abs(g[k] - nv) <= 1e-9 * nv
        assert np.all(np.abs(g) <= nv * (1 + 1e-12))
        assert np.argmax(g) == k


def test_dirty_beam_translation_invariance():
    side, nv = 10, 250
    uv = _uv(nv, 9)

    def beam(k):
        lk, mk = k % side - side // 2, k // side - side // 2
        e = np.exp(-2j * np.pi * (uv[:, 0] * lk + uv[:, 1] * mk))
        return fourier.gradient(uv, side, np.concatenate([e.real, e.imag]))

    b1, b2 = beam(2 * side + 3), beam(5 * side + 4)   # (l, m) offsets differ by (1, 3)
    for dl, dm in ((0, 0), (1, 0), (2, 1), (-1, 2), (3, -1)):
        k1 = (2 + dm) * side + 3 + dl
        k2 = (5 + dm) * side + 4 + dl
        assert abs(b1[k1] - b2[k2]) <= 1e-9 * nv


def test_matrix_free_visibilities_are_the_workload_draws():
    uv, y, x, sup = workloads.interferometry_visibilities(300, 16, 5, 30.0, 4)
    p = workloads.interferometry(n_vis=300, side=16, s=5, seed=4, dtype=np.complex128)
    np.testing.assert_array_equal(uv, p.uv)
    np.testing.assert_array_equal(sup, p.support)
    np.testing.assert_array_equal(x, p.x_true)
    want = np.concatenate([p.y.real, p.y.imag])
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_pins_catch_planted_mistakes():
    """Each plausible mistake in the gradient's formula (planted here, in a
    copy on the CPU) breaks at least one of the checks above: the sine's
    sign, swapped pixel axes, the centre rounded up for odd sides, a
    dropped imaginary term."""
    def make(sign=-1.0, swap=False, centre=lambda s: s // 2, drop_im=False):
        def grad(uv, side, r):
            k = np.arange(side * side)
            lk, mk = (k % side) - centre(side), (k // side) - centre(side)
            if swap:
                lk, mk = mk, lk
            th = 2.0 * np.pi * (np.outer(uv[:, 0], lk) + np.outer(uv[:, 1], mk))
            nv = uv.shape[0]
            g = np.cos(th).T @ r[:nv]
            if not drop_im:
                g = g + sign * (np.sin(th).T @ r[nv:])
            return g
        return grad

    side, nv = 7, 60
    uv = _uv(nv, 21)
    rng = np.random.default_rng(22)
    y = rng.standard_normal(nv) + 1j * rng.standard_normal(nv)
    lk, mk = fourier.pixel_coords(side)
    phi = np.exp(-2j * np.pi * (np.outer(uv[:, 0], lk) + np.outer(uv[:, 1], mk)))
    want = (np.conj(phi).T @ y).real
    r = np.concatenate([y.real, y.imag])
    np.testing.assert_allclose(make()(uv, side, r), want, atol=1e-12 * np.abs(want).max())
    for bad in (make(sign=+1.0), make(swap=True), make(centre=lambda s: (s + 1) // 2),
                make(drop_im=True)):
        assert np.abs(bad(uv, side, r) - want).max() > 1e-3 * np.abs(want).max()
