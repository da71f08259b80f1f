"""Camera sampling of the detector-plane field (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper records its measurements with cameras of their own size (512^2
pixels in the simulated experiment, 150^2 for the yeast cell; Section 6)
and gives no optical geometry, so the following reading is used: the
field on the detector plane (the exit plane, or the plane at det_dist
reached by angular-spectrum propagation) is known on the N x N lateral
window of the grid, periodic over that window and band limited to the
window's frequency grid; a square camera of M x M pixels with pitch p (in
the sample plane) centred on the optical axis samples the trigonometric
interpolant of that field at its pixel centres c_a = (a - (M-1)/2) p:

    f(c) = (1/N^2) sum_{ky, kx} F[ky, kx] exp(i (kx (c_x - x0) + ky (c_y - x0)))

with F the unnormalised 2-D DFT of the window samples, k = 2 pi fftfreq(N, h)
(signed frequencies, -pi/h for the Nyquist bin of an even N) and x0 the
first voxel centre.  The map is H = Ey F Ex^T / N^2 with E[a, k] =
exp(i k (c_a - x0)); its adjoint is r -> ifft2(Ey^H r conj(Ex)) (the fft2
adjoint being N^2 ifft2).  At M = N and p = h it is the identity.
"""
from __future__ import annotations

import math

import numpy as np

from . import lsmodel


def pixel_centres(M: int, pitch: float) -> np.ndarray:
    """Camera pixel centres along one axis, centred on the optical axis."""
    return (np.arange(M) - (M - 1) / 2.0) * pitch


def phase_matrix(N: int, h: float, M: int, pitch: float) -> np.ndarray:
    """E[a, k] = exp(i k (c_a - x0)) for the window's DFT frequencies k."""
    k = 2.0 * math.pi * np.fft.fftfreq(N, d=h)
    x0 = lsmodel.voxel_axis(N, h)[0]
    c = pixel_centres(M, pitch)
    return np.exp(1j * np.outer(c - x0, k))


def sample(plane: np.ndarray, N: int, h: float, M: int, pitch: float) -> np.ndarray:
    """Camera image (M, M) [y][x] of an (N, N) detector-plane field."""
    E = phase_matrix(N, h, M, pitch)
    return E @ np.fft.fft2(plane) @ E.T / (N * N)


def sample_adjoint(r: np.ndarray, N: int, h: float, M: int, pitch: float) -> np.ndarray:
    """Adjoint of `sample`: an (M, M) camera image back to the (N, N) window."""
    E = phase_matrix(N, h, M, pitch)
    return np.fft.ifft2(E.conj().T @ r @ E.conj())


class CameraLSModel(lsmodel.LSModel):
    """The oracle's scattering model with the detector images taken by an
    M x M camera of pitch `pitch` (um): H_l = C P_d S (u_l - u_in,l)."""

    def __init__(self, geom: lsmodel.Geometry, cam_n: int, cam_pitch: float, ghat_P=None, workers=None):
        super().__init__(geom, ghat_P=ghat_P, workers=workers)
        self.cam_n = int(cam_n)
        self.cam_pitch = float(cam_pitch)

    def detector(self, field):
        return sample(super().detector(field), self.geom.N, self.geom.h, self.cam_n, self.cam_pitch)

    def detector_T(self, r):
        return super().detector_T(sample_adjoint(r, self.geom.N, self.geom.h, self.cam_n, self.cam_pitch))
