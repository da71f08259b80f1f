"""Pins of the oracle's detector propagation (angular spectrum, a reading
where the paper gives no detector geometry).

* d = 0 is the identity; plane waves of the lateral grid are eigenfunctions
  with eigenvalue exp(j k_z d), k_z from the closed form (propagating and
  evanescent); P_{d1} P_{d2} = P_{d1 + d2}; <P a, b> = <a, P^H b>;
  propagating band-limited fields keep their norm;
* the gradient with a propagated detector matches central differences of
  the loss, which pins the adjoint chain detector_T = detector^H.
"""
import math

import numpy as np
import pytest

import synthetic as syn
from oracle import lsmodel

LAM0, NB = syn.LAMBDA0_UM, syn.N_B


def _geom(N, d=0.0):
    return lsmodel.Geometry(N=N, h=LAM0 / 4, lambda0=LAM0, n_b=NB, det_dist=d)


def _cfield(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_zero_distance_is_identity():
    g = _geom(16)
    a = _cfield((16, 16), 0)
    assert np.array_equal(lsmodel.transfer_function(g, 0.0), np.ones((16, 16), complex))
    np.testing.assert_allclose(lsmodel.propagate(a, g, 0.0), a, rtol=0, atol=1e-14)


@pytest.mark.parametrize("mx,my", [(0, 0), (1, 2), (-2, 1), (4, -3), (7, 7), (-8, 5)])
def test_plane_waves_are_eigenfunctions(mx, my):
    N, d = 16, 1.3
    g = _geom(N)
    h = g.h
    c = lsmodel.voxel_axis(N, h)
    kx, ky = 2 * math.pi * mx / (N * h), 2 * math.pi * my / (N * h)
    plane = np.exp(1j * (ky * c[:, None] + kx * c[None, :]))
    kp2 = kx * kx + ky * ky
    kz = math.sqrt(g.kb ** 2 - kp2) if kp2 <= g.kb ** 2 else 1j * math.sqrt(kp2 - g.kb ** 2)
    out = lsmodel.propagate(plane, g, d)
    np.testing.assert_allclose(out, np.exp(1j * kz * d) * plane, rtol=0, atol=1e-12)
    if kp2 > g.kb ** 2:
        assert np.max(np.abs(out)) < 1.0    # evanescent: decays


def test_semigroup_adjoint_and_norm():
    N = 24
    g = _geom(N)
    a, b = _cfield((N, N), 1), _cfield((N, N), 2)
    p12 = lsmodel.propagate(lsmodel.propagate(a, g, 0.7), g, 1.1)
    np.testing.assert_allclose(p12, lsmodel.propagate(a, g, 1.8), rtol=0, atol=1e-12)
    lhs = np.vdot(lsmodel.propagate(a, g, 0.9), b)
    rhs = np.vdot(a, lsmodel.propagate(b, g, 0.9, adjoint=True))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # band-limited to propagating frequencies: the norm is kept
    k = 2 * math.pi * np.fft.fftfreq(N, d=g.h)
    keep = (k[:, None] ** 2 + k[None, :] ** 2) < g.kb ** 2
    c = np.fft.ifft2(np.fft.fft2(a) * keep)
    assert np.linalg.norm(lsmodel.propagate(c, g, 2.5)) == pytest.approx(np.linalg.norm(c), rel=1e-13)


def test_gradient_with_propagated_detector_matches_central_differences():
    N = 12
    geom = _geom(N, d=1.5)
    model = lsmodel.LSModel(geom)
    rng = np.random.default_rng(21)
    dn = syn.phantom_ellipsoids(N, geom.h, rng, n_incl=3, dn_range=(0.01, 0.05))
    xt = syn.scattering_potential(dn)
    dirs = syn.illumination_directions(2, 35.0, np.random.default_rng(3))
    idx = [0, 1]
    yc, _ = model.forward(xt, dirs, idx, 1e-14, 500)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(4))
    x = 0.5 * xt
    g, f, _ = model.grad(x, y, dirs, idx, 0.5, 1e-14, 500)

    def loss(xx):
        H, _ = model.forward(xx, dirs, idx, 1e-14, 500)
        return 0.5 * 0.5 * float(np.sum(np.abs(H - y) ** 2))

    assert loss(x) == pytest.approx(f, rel=1e-12)
    step = 1e-4 * np.max(x)
    e = np.random.default_rng(6).standard_normal(x.shape)
    e /= np.linalg.norm(e)
    fd = (loss(x + step * e) - loss(x - step * e)) / (2 * step)
    an = float(np.sum(g * e))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
