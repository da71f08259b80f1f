"""Lippmann-Schwinger data term and its mini-batch gradient (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Follows the problem statement of arXiv:2307.02043: the composite objective
(Section 1, eq. defMainPro) with f_l(x) = 1/2 ||H_l(x) - y_l||^2, the
mini-batch split F_s = (S/L) sum_{l in S_s} f_l (Section 4, eq. NewModelPro),
and the ODT setting of Section 6: evaluating H_l needs one Lippmann-Schwinger
solve and the gradient of f_l needs two, each solved with BiCGSTAB
(van der Vorst 1992).  Readings where the paper is silent (it defers the
model to its supplement):

* field equation (I - G diag(x)) u_l = u_in,l with u_in,l = exp(j k_l . r);
* H_l(x) = S (u_l - u_in,l), S = the z = N-1 plane (N x N detector);
  optionally the detector is a plane at distance d beyond it: the
  scattered field on the exit plane, taken as periodic over the N x N
  lateral window, is propagated by the angular spectrum
  P_d = F^-1 diag(exp(j k_z d)) F, k_z = sqrt(kb^2 - kx^2 - ky^2) for
  propagating and j sqrt(kx^2 + ky^2 - kb^2) for evanescent components
  (the paper's off-grid cameras need a geometry it does not give);
* BiCGSTAB started at the right-hand side, shadow residual r^ = r_0,
  relative recursive-residual stopping test, early exit on ||s||;
* gradient of f_l = Re(conj(u_l) . w_l) where w_l solves
  (I - G^H diag(x)) w_l = G^H S^T r_l  (J_l = S (I - G X)^-1 G diag(u_l),
  and G^H (I - X G^H)^-1 = (I - G^H X)^-1 G^H);
* first-Born variant: u_l := u_in,l, H_l = S G(x . u_in,l),
  gradient Re(conj(u_in,l) . G^H S^T r_l).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import green

# Solver status codes (mirrors the meaning, not the code, of the library's).
CONVERGED, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


@dataclass
class Geometry:
    N: int
    h: float          # voxel edge (um)
    lambda0: float    # vacuum wavelength (um)
    n_b: float        # background refractive index
    det_dist: float = 0.0  # detector distance beyond the exit plane (um); 0: the exit plane

    @property
    def k0(self) -> float:
        return 2.0 * math.pi / self.lambda0

    @property
    def kb(self) -> float:
        return self.n_b * self.k0


def voxel_axis(N: int, h: float) -> np.ndarray:
    """Voxel centres (i - (N-1)/2) h along one axis."""
    return (np.arange(N) - (N - 1) / 2.0) * h


def transfer_function(geom: Geometry, d: float) -> np.ndarray:
    """Angular-spectrum transfer function exp(j k_z d) on the N x N lateral
    frequency grid (FFT order, [ky][kx]), k_z = sqrt(kb^2 - |k_perp|^2) with
    the root j sqrt(|k_perp|^2 - kb^2) for evanescent components."""
    k = 2.0 * math.pi * np.fft.fftfreq(geom.N, d=geom.h)
    kp2 = k[:, None] ** 2 + k[None, :] ** 2
    kz2 = geom.kb ** 2 - kp2
    kz = np.where(kz2 >= 0, np.sqrt(np.maximum(kz2, 0.0)) + 0j, 1j * np.sqrt(np.maximum(-kz2, 0.0)))
    return np.exp(1j * kz * d)


def propagate(plane: np.ndarray, geom: Geometry, d: float, adjoint: bool = False) -> np.ndarray:
    """P_d (or its adjoint) applied to an (N, N) field [y][x]."""
    T = transfer_function(geom, d)
    return np.fft.ifft2((np.conj(T) if adjoint else T) * np.fft.fft2(plane))


def incident_field(geom: Geometry, direction) -> np.ndarray:
    """Plane wave exp(j kb d . r) on the grid, [z][y][x] (Section 6.1)."""
    c = voxel_axis(geom.N, geom.h)
    dx, dy, dz = direction
    ph = geom.kb * (dz * c[:, None, None] + dy * c[None, :, None]
                    + dx * c[None, None, :])
    return np.exp(1j * ph)


def bicgstab(apply_A, b, x0, tol, max_iter, breakdown=1e-300):
    """BiCGSTAB for A e = b (van der Vorst 1992), complex FP64.

    Inner product <a, b> = sum conj(a) b.  Returns (e, iterations, status,
    final relative recursive residual).  The solve stops with status
    BREAKDOWN when |rho|, |<rhat, v>| or |omega| falls below ``breakdown``.
    """
    e = np.array(x0, dtype=np.complex128, copy=True)
    r = b - apply_A(e)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(e), 0, CONVERGED, 0.0
    res = np.linalg.norm(r) / bnorm
    if res <= tol:
        return e, 0, CONVERGED, res
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0.0j
    v = np.zeros_like(r)
    p = np.zeros_like(r)
    for it in range(1, max_iter + 1):
        rho_new = np.vdot(rhat, r)
        if abs(rho_new) < breakdown:
            return e, it - 1, BREAKDOWN, res
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply_A(p)
        rv = np.vdot(rhat, v)
        if abs(rv) < breakdown or rv == 0:
            # counted as an iteration: its product A p was formed
            return e, it, BREAKDOWN, res
        alpha = rho_new / rv
        s = r - alpha * v
        res_s = np.linalg.norm(s) / bnorm
        if res_s <= tol:
            e = e + alpha * p
            return e, it, CONVERGED, res_s
        t = apply_A(s)
        tt = np.vdot(t, t)
        omega = np.vdot(t, s) / tt
        e = e + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        res = np.linalg.norm(r) / bnorm
        if res <= tol:
            return e, it, CONVERGED, res
        if abs(omega) < breakdown:
            return e, it, BREAKDOWN, res
    return e, max_iter, NOT_CONVERGED, res


class LSModel:
    """Discretised scattering model on an N^3 grid (oracle)."""

    def __init__(self, geom: Geometry, ghat_P: np.ndarray | None = None,
                 workers: int | None = None):
        self.geom = geom
        self.workers = workers
        if ghat_P is None:
            ghat_P = green.kernel_padded(geom.N, geom.h, geom.kb, workers=workers)
        self.ghat = ghat_P

    # operators --------------------------------------------------------------
    def G(self, v):
        return green.apply_G(self.ghat, v, workers=self.workers)

    def GH(self, v):
        return green.apply_GH(self.ghat, v, workers=self.workers)

    def detector(self, field):
        """S: the z = N-1 plane of a field, shape (N, N), propagated to the
        detector plane when det_dist > 0."""
        if self.geom.det_dist > 0:
            return propagate(field[-1], self.geom, self.geom.det_dist)
        return field[-1]

    def detector_T(self, r):
        """S^T (the adjoint of detector): embed an (N, N) detector image
        (propagated back by P_d^H when det_dist > 0) into the z = N-1 plane."""
        N = self.geom.N
        if self.geom.det_dist > 0:
            r = propagate(r, self.geom, self.geom.det_dist, adjoint=True)
        out = np.zeros((N, N, N), dtype=np.complex128)
        out[-1] = r
        return out

    # solves ----------------------------------------------------------------
    def solve_forward(self, x, uin, tol, max_iter, e0=None, breakdown=1e-300):
        """(I - G diag(x)) u = u_in, started from u_in (or from e0)."""
        return bicgstab(lambda e: e - self.G(x * e), uin, uin if e0 is None else e0, tol, max_iter,
                        breakdown)

    def solve_adjoint(self, x, z, tol, max_iter, e0=None, breakdown=1e-300):
        """(I - G^H diag(x)) w = z, started from z (or from e0)."""
        return bicgstab(lambda e: e - self.GH(x * e), z, z if e0 is None else e0, tol, max_iter,
                        breakdown)

    # model -----------------------------------------------------------------
    def forward(self, x, directions, idx, tol, max_iter, model="ls"):
        """H_l(x) for l in idx: (B, N, N) complex, plus per-illumination stats."""
        ys, stats = [], []
        for l in idx:
            uin = incident_field(self.geom, directions[l])
            if model == "born":
                ys.append(self.detector(self.G(x * uin)))
                stats.append((0, CONVERGED, 0.0))
                continue
            u, it, st, res = self.solve_forward(x, uin, tol, max_iter)
            ys.append(self.detector(u - uin))
            stats.append((it, st, res))
        return np.stack(ys), stats

    def grad(self, x, y, directions, idx, scale, tol, max_iter, model="ls", starts=None,
             return_fields=False):
        """scale * sum_l grad f_l(x) and scale * sum_l f_l(x) over the batch.

        y[b] is the measurement of illumination idx[b].  starts: None, or
        per batch element a pair (u0, w0) of starting points for the forward
        and adjoint solves (warm start, e.g. the fields of an earlier outer
        iteration).  Returns (g, loss, stats) with stats[b] = (it_fwd,
        it_adj, status_fwd, status_adj), and the fields [(u_b, w_b)] as a
        fourth element when return_fields is set.
        """
        g = np.zeros(x.shape)
        loss = 0.0
        stats = []
        fields = []
        for b, l in enumerate(idx):
            uin = incident_field(self.geom, directions[l])
            u0, w0 = (None, None) if starts is None else starts[b]
            if model == "born":
                u = uin
                H = self.detector(self.G(x * uin))
                itf, stf = 0, CONVERGED
            else:
                u, itf, stf, _ = self.solve_forward(x, uin, tol, max_iter, e0=u0)
                H = self.detector(u - uin)
            r = H - y[b]
            loss += 0.5 * np.vdot(r, r).real
            z = self.GH(self.detector_T(r))
            if model == "born":
                w, ita, sta = z, 0, CONVERGED
            else:
                w, ita, sta, _ = self.solve_adjoint(x, z, tol, max_iter, e0=w0)
            g += np.real(np.conj(u) * w)
            stats.append((itf, ita, stf, sta))
            fields.append((u, w))
        if return_fields:
            return scale * g, scale * loss, stats, fields
        return scale * g, scale * loss, stats

    def tangent(self, x, direction, dx, tol, max_iter):
        """J dx = S du with (I - G X) du = G(dx . u): directional derivative
        of H_l, computed by a forward-type solve (independent of the adjoint).
        """
        uin = incident_field(self.geom, direction)
        u, _, _, _ = self.solve_forward(x, uin, tol, max_iter)
        rhs = self.G(dx * u)
        du, _, _, _ = bicgstab(lambda e: e - self.G(x * e), rhs, rhs, tol, max_iter)
        return self.detector(du)

    def vjp(self, x, direction, rdet, tol, max_iter):
        """Re(J^H rdet) for one illumination (the gradient kernel)."""
        uin = incident_field(self.geom, direction)
        u, _, _, _ = self.solve_forward(x, uin, tol, max_iter)
        z = self.GH(self.detector_T(rdet))
        w, _, _, _ = self.solve_adjoint(x, z, tol, max_iter)
        return np.conj(u) * w
