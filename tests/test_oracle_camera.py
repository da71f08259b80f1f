"""Pins of the oracle's camera sampling (a reading: the paper's cameras have
their own pixel count and pitch, its geometry is not given).

* a camera on the window's own grid (M = N, pitch h) returns the window
  samples exactly;
* a lateral plane wave of the window's frequency grid is sampled exactly at
  arbitrary pixel positions (closed form), for cameras finer or coarser
  than the grid, larger or smaller than the window;
* <C a, r> = <a, C^H r>;
* the gradient of the loss with a camera (and a propagated detector plane)
  matches central differences, which pins the adjoint chain.
"""
import math

import numpy as np
import pytest

import synthetic as syn
from oracle import camera, lsmodel

LAM0, NB = syn.LAMBDA0_UM, syn.N_B
H = LAM0 / 4


def _cfield(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("N", [8, 12, 16])
def test_camera_on_the_grid_is_the_identity(N):
    a = _cfield((N, N), N)
    out = camera.sample(a, N, H, N, H)
    assert np.max(np.abs(out - a)) < 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("N,M,pitch", [(16, 40, 0.037), (16, 7, 0.31), (12, 150, 0.0123), (16, 23, H)])
@pytest.mark.parametrize("mx,my", [(0, 0), (1, -2), (-3, 5), (7, 0)])
def test_plane_waves_are_sampled_exactly(N, M, pitch, mx, my):
    if max(abs(mx), abs(my)) >= N // 2:
        pytest.skip("frequency at or past the window's Nyquist bin (aliased on the grid)")
    c = lsmodel.voxel_axis(N, H)
    kx, ky = 2 * math.pi * mx / (N * H), 2 * math.pi * my / (N * H)
    plane = np.exp(1j * (ky * c[:, None] + kx * c[None, :]))
    cc = camera.pixel_centres(M, pitch)
    ref = np.exp(1j * (ky * cc[:, None] + kx * cc[None, :]))
    out = camera.sample(plane, N, H, M, pitch)
    assert np.max(np.abs(out - ref)) < 1e-12


@pytest.mark.parametrize("N,M,pitch", [(16, 40, 0.037), (12, 9, 0.2)])
def test_adjoint_identity(N, M, pitch):
    a = _cfield((N, N), 1)
    r = _cfield((M, M), 2)
    lhs = np.vdot(camera.sample(a, N, H, M, pitch), r)
    rhs = np.vdot(a, camera.sample_adjoint(r, N, H, M, pitch))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.slow
@pytest.mark.parametrize("d", [0.0, 1.1])
def test_gradient_with_camera_matches_central_differences(d):
    N, M, pitch = 12, 20, 0.057
    geom = lsmodel.Geometry(N=N, h=H, lambda0=LAM0, n_b=NB, det_dist=d)
    model = camera.CameraLSModel(geom, M, pitch)
    rng = np.random.default_rng(7)
    xt = syn.scattering_potential(syn.phantom_ellipsoids(N, H, rng))
    dirs = syn.illumination_directions(2, 35.0, np.random.default_rng(8))
    idx = [0, 1]
    yc, _ = model.forward(xt, dirs, idx, 1e-14, 500)
    assert yc.shape == (2, M, M)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(9))
    x = 0.5 * xt
    g, f, _ = model.grad(x, y, dirs, idx, 0.5, 1e-14, 500)

    def loss(xx):
        Hh, _ = model.forward(xx, dirs, idx, 1e-14, 500)
        return 0.5 * 0.5 * float(np.sum(np.abs(Hh - y) ** 2))

    assert loss(x) == pytest.approx(f, rel=1e-12)
    step = 1e-4 * np.max(x)
    for seed in range(3):
        e = np.random.default_rng(20 + seed).standard_normal(x.shape)
        e /= np.linalg.norm(e)
        fd = (loss(x + step * e) - loss(x - step * e)) / (2 * step)
        an = float(np.sum(g * e))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.max(np.abs(g))), (fd, an)
