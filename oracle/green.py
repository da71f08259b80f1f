"""Green's operator of the discretised Lippmann-Schwinger equation (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper defers the discretisation of the scattering model to its
supplement and to Pham et al. (2020) (Section 6, numerical experiments);
neither is available.  The reading implemented here is the standard one:

* the field obeys u = u_in + G (x . u), with the free-space Helmholtz Green's
  function g(r) = exp(j k_b r) / (4 pi r) of the background medium;
* g is truncated at R = sqrt(3) N h, the diameter of the cubic domain, which
  leaves the convolution unchanged for points inside the domain;
* the Fourier transform of the truncated kernel is known in closed form and
  is smooth, so it is sampled on an oversampled grid (Q = 4N points per
  axis), transformed back to get the discrete kernel at the lags
  -N..N-1, and that kernel is transformed on the 2N zero-padded grid
  (Vico, Greengard and Ferrando, 2016).  The voxel volume h^3 is part of the
  discrete kernel, so x is in um^-2 and G is dimensionless.

G v = crop(IFFT(ghat_P . FFT(pad v))) and G^H v uses conj(ghat_P).
ghat_P is even in every axis, so G^T = G.
"""
from __future__ import annotations

import math

import numpy as np


def truncation_radius(N: int, h: float) -> float:
    """Diameter of the N^3 voxel domain, the truncation radius of g."""
    return math.sqrt(3.0) * N * h


def _E(a: np.ndarray, R: float) -> np.ndarray:
    """Integral of exp(j a t) over t in [0, R], for real a (array)."""
    a = np.asarray(a, dtype=np.float64)
    z = a * R
    out = np.empty(a.shape, dtype=np.complex128)
    small = np.abs(z) < 0.5
    zb = z[~small]
    out[~small] = (np.exp(1j * zb) - 1.0) / (1j * a[~small])
    # power series R * sum_n (jz)^n / (n+1)!  for |z| < 0.5 (20 terms: < 1e-25)
    zs = 1j * z[small]
    acc = np.zeros(zs.shape, dtype=np.complex128)
    term = np.ones(zs.shape, dtype=np.complex128)
    for n in range(20):
        acc += term / math.factorial(n + 1)
        term = term * zs
    out[small] = R * acc
    return out


def ghat_truncated(s: np.ndarray, kb: float, R: float) -> np.ndarray:
    """Fourier transform of g(r) 1{r < R} at radial frequency s = |xi|.

    ghat(s) = (1/s) int_0^R exp(j kb t) sin(s t) dt.  Two exact forms are
    used so that no branch loses digits:
      s <  kb/2 : [1 + e^{j kb R}(j kb sin(sR)/s - cos(sR))] / (s^2 - kb^2)
      s >= kb/2 : [E(kb + s) - E(kb - s)] / (2 j s),  E(a) = int_0^R e^{j a t}dt
    The second form has no cancellation at the shell s = kb.
    """
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.complex128)
    lo = s < 0.5 * kb
    sl = s[lo]
    sinc_term = np.where(sl > 0, np.sin(sl * R) / np.where(sl > 0, sl, 1.0), R)
    eikR = np.exp(1j * kb * R)
    out[lo] = (1.0 + eikR * (1j * kb * sinc_term - np.cos(sl * R))) / (sl * sl - kb * kb)
    sh = s[~lo]
    out[~lo] = (_E(kb + sh, R) - _E(kb - sh, R)) / (2j * sh)
    return out


def oversampling(N: int) -> int:
    """Points per axis of the oversampled transform grid: 4N up to N = 128,
    3N above (both exceed the (1 + sqrt 3) N that keeps the periodic images
    of the truncated kernel off the domain; 3N keeps the 256^3 case at a
    768^3 transform)."""
    return 4 * N if N <= 128 else 3 * N


def kernel_lags_direct(N: int, h: float, kb: float, Q: int | None = None,
                       workers: int | None = None) -> np.ndarray:
    """The cropped kernel K of kernel_padded itself (lags -N..N-1 per axis in
    wrap-around order on the 2N grid), before its forward DFT: the discrete
    kernel of the padded convolution without the DFT round trip."""
    import scipy.fft as sfft

    Q = oversampling(N) if Q is None else Q
    R = truncation_radius(N, h)
    k = np.fft.fftfreq(Q, d=1.0 / Q).astype(np.int64)
    k2 = (k[:, None, None] ** 2 + k[None, :, None] ** 2) + k[None, None, :] ** 2
    dk = 2.0 * np.pi / (Q * h)
    table = ghat_truncated(dk * np.sqrt(np.arange(int(k2.max()) + 1, dtype=np.float64)), kb, R)
    gh = table[k2]
    del k2
    K = sfft.ifftn(gh, workers=workers, overwrite_x=True)
    del gh
    idx = np.r_[np.arange(0, N), np.arange(Q - N, Q)]
    return K[np.ix_(idx, idx, idx)]


def kernel_padded(N: int, h: float, kb: float, Q: int | None = None,
                  workers: int | None = None) -> np.ndarray:
    """ghat_P on the (2N)^3 padded grid (complex128, numpy FFT ordering).

    Steps: sample ghat_truncated at xi = 2 pi m / (Q h) on a Q^3 grid, take
    the inverse DFT (1/Q^3 normalisation) to obtain K[m] ~ h^3 g_R(m h), keep
    the lags -N..N-1 per axis in wrap-around order on the 2N grid, and take
    the forward DFT of that cropped kernel.
    """
    import scipy.fft as sfft

    Q = oversampling(N) if Q is None else Q
    R = truncation_radius(N, h)
    # |xi|^2 = (2 pi / (Q h))^2 (kx^2 + ky^2 + kz^2) with integer k: the radial
    # transform is evaluated once per distinct integer k^2 and gathered
    k = np.fft.fftfreq(Q, d=1.0 / Q).astype(np.int64)
    k2 = (k[:, None, None] ** 2 + k[None, :, None] ** 2) + k[None, None, :] ** 2
    dk = 2.0 * np.pi / (Q * h)
    table = ghat_truncated(dk * np.sqrt(np.arange(int(k2.max()) + 1, dtype=np.float64)), kb, R)
    gh = table[k2]
    del k2
    K = sfft.ifftn(gh, workers=workers)
    del gh
    idx = np.r_[np.arange(0, N), np.arange(Q - N, Q)]
    KP = K[np.ix_(idx, idx, idx)]
    del K
    return sfft.fftn(KP, workers=workers)


def _pad(v: np.ndarray) -> np.ndarray:
    N = v.shape[-1]
    out = np.zeros(v.shape[:-3] + (2 * N, 2 * N, 2 * N), dtype=np.complex128)
    out[..., :N, :N, :N] = v
    return out


def apply_G(ghat_P: np.ndarray, v: np.ndarray, workers: int | None = None) -> np.ndarray:
    """G v = crop(IFFT(ghat_P . FFT(pad v))) on the zero-padded grid."""
    import scipy.fft as sfft

    N = v.shape[-1]
    f = sfft.fftn(_pad(v), axes=(-3, -2, -1), workers=workers)
    f *= ghat_P
    return sfft.ifftn(f, axes=(-3, -2, -1), workers=workers)[..., :N, :N, :N]


def apply_GH(ghat_P: np.ndarray, v: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Adjoint G^H v, using the conjugate transfer function."""
    return apply_G(np.conj(ghat_P), v, workers=workers)


def kernel_lags(ghat_P: np.ndarray) -> np.ndarray:
    """Discrete kernel K on the 2N grid (inverse DFT of ghat_P)."""
    return np.fft.ifftn(ghat_P)


def apply_G_direct(K_P: np.ndarray, v: np.ndarray, points) -> np.ndarray:
    """(G v) at a few voxels by direct summation over the whole grid.

    (G v)[i] = sum_j K[i - j] v[j] with the lag taken modulo 2N.  Used to
    check single outputs of a large operator one at a time.
    """
    N = v.shape[-1]
    P = 2 * N
    j = np.arange(N)
    out = np.empty(len(points), dtype=np.complex128)
    for n, (iz, iy, ix) in enumerate(points):
        kz = (iz - j) % P
        ky = (iy - j) % P
        kx = (ix - j) % P
        out[n] = np.sum(K_P[np.ix_(kz, ky, kx)] * v)
    return out
