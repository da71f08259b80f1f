"""Weighted proximal mapping of constrained TV (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Computes x = argmin_{x in C} 1/2 ||x - v||^2_B + lam TV(x) with
B = tau I + U U^T (U with r >= 0 columns), C = R^N_+ or R^N, TV isotropic or
anisotropic, following arXiv:2307.02043:

* discrete TV and its dual form (Section 3.2 eqs. TViso/TVl1, Section 3.3
  eqs. B&Tiso/B&Tl1): TV(x) = max_{P in Pset} d(P)^T x,
  d(P) = sum_d (D^d)^T q_d, with ||p_n||_2 <= 1 (iso) or ||p_n||_inf <= 1;
* D^d is read as the forward difference along array axis d with a zero last
  row (Neumann boundary), the operator of Beck and Teboulle (2009); the
  notation paragraph of Section 3.1 is garbled on the shift;
* the dual problem of Section 4.1 (eqs. SecondProximalMatrixnormV2_New):
  w(P) = v - lam B^-1 d(P), x(P) = prox^B_{iota_C}(w(P)), gradient of the
  dual objective -2 lam d^T(x(P)), Lipschitz constant 8 D lam^2 / omega_min
  (Lemma 4.1), minimised by the accelerated projected gradient (FISTA)
  iteration with step 1 / Lipschitz, output x(P_K);
* B^-1 applied with the Woodbury identity (Section 4.3):
  B^-1 = I / tau - U (I_r + U^T U / tau)^-1 U^T / tau^2;
* prox^B_{iota_C}(w) = max(w - U beta* / tau, 0) with beta* in R^r the root
  of phi(beta) = U^T (w - max(w - U beta / tau, 0)) + beta (Theorem 3.1 with
  Sigma = tau I).  For r = 1 phi is continuous, piecewise linear and
  increasing with slope >= 1; the oracle finds its root exactly from the
  sorted breakpoints.  For r >= 2 phi is the gradient of a strongly convex
  piecewise-quadratic function and the oracle takes Newton steps on its
  pieces with backtracking until a full step stays on its piece, where the
  step is the exact root (the library uses the semi-smooth Newton iteration
  of Algorithm 4.3 in both cases).
* omega_min = tau for B = tau I + U U^T when rank U < N.
"""
from __future__ import annotations

import math

import numpy as np

DIM = 3


# --------------------------------------------------------------------------
# finite differences and TV
# --------------------------------------------------------------------------

def diff(x: np.ndarray, axis: int) -> np.ndarray:
    """(D^d x): forward difference along `axis`, zero in the last slice."""
    out = np.zeros_like(x)
    n = x.shape[axis]
    sl_hi = [slice(None)] * x.ndim
    sl_lo = [slice(None)] * x.ndim
    sl_hi[axis] = slice(1, n)
    sl_lo[axis] = slice(0, n - 1)
    out[tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
    return out


def diff_T(q: np.ndarray, axis: int) -> np.ndarray:
    """(D^d)^T q, the exact transpose of `diff` (last slice of q ignored)."""
    n = q.shape[axis]
    qq = q.copy()
    sl_last = [slice(None)] * q.ndim
    sl_last[axis] = slice(n - 1, n)
    qq[tuple(sl_last)] = 0.0
    out = -qq
    sl_hi = [slice(None)] * q.ndim
    sl_lo = [slice(None)] * q.ndim
    sl_hi[axis] = slice(1, n)
    sl_lo[axis] = slice(0, n - 1)
    out[tuple(sl_hi)] += qq[tuple(sl_lo)]
    return out


def grad_op(x: np.ndarray) -> np.ndarray:
    """d^T(x) = (D^1 x, D^2 x, D^3 x), shape (3,) + x.shape."""
    return np.stack([diff(x, a) for a in range(DIM)])


def div_op(P: np.ndarray) -> np.ndarray:
    """d(P) = sum_d (D^d)^T q_d."""
    return sum(diff_T(P[a], a) for a in range(DIM))


def tv(x: np.ndarray, kind: str) -> float:
    g = grad_op(x)
    if kind == "iso":
        return float(np.sum(np.sqrt(np.sum(g * g, axis=0))))
    return float(np.sum(np.abs(g)))


def project_dual(P: np.ndarray, kind: str) -> np.ndarray:
    """Projection onto Pset: unit l2 ball per voxel (iso), unit box (aniso)."""
    if kind == "iso":
        nrm = np.sqrt(np.sum(P * P, axis=0))
        return P / np.maximum(1.0, nrm)
    return np.clip(P, -1.0, 1.0)


# --------------------------------------------------------------------------
# metric tau I + u u^T
# --------------------------------------------------------------------------

def _cols(u, shape):
    """The metric's low-rank factor as an (r, V) array (r = 0 for None).

    u is None, an image of the given shape (rank one) or an array of shape
    (r,) + shape (columns u_1 .. u_r).
    """
    if u is None:
        return np.zeros((0, int(np.prod(shape))))
    u = np.asarray(u, dtype=np.float64)
    if u.shape == tuple(shape):
        return u.reshape(1, -1)
    return u.reshape(u.shape[0], -1)


def apply_B(y, tau, u):
    """(tau I + U U^T) y."""
    U = _cols(u, y.shape)
    return tau * y + (U.T @ (U @ y.ravel())).reshape(y.shape)


def apply_B_inv(y, tau, u):
    """Woodbury: B^-1 = I/tau - U (I_r + U^T U / tau)^-1 U^T / tau^2."""
    U = _cols(u, y.shape)
    if U.shape[0] == 0:
        return y / tau
    M = np.eye(U.shape[0]) + (U @ U.T) / tau
    c = np.linalg.solve(M, U @ y.ravel())
    return y / tau - (U.T @ c).reshape(y.shape) / (tau * tau)


def phi(beta, w, tau, u):
    """phi(beta) = U^T (w - max(w - U beta / tau, 0)) + beta (Theorem 3.1).

    Scalar for a rank-one u given as an image, a vector of length r otherwise."""
    U = _cols(u, np.shape(w))
    wf = np.ravel(w)
    b = np.atleast_1d(np.asarray(beta, dtype=np.float64))
    out = U @ (wf - np.maximum(wf - U.T @ b / tau, 0.0)) + b
    if np.shape(u) == np.shape(w):
        return float(out[0])
    return out


def root_phi_exact(w, tau, u):
    """Exact root of the piecewise-linear increasing phi (rank one).

    Each voxel with u_n != 0 has one breakpoint b_n = tau w_n / u_n; between
    breakpoints phi(beta) = beta (1 + sum_{active} u_n^2 / tau)
    + sum_{inactive} u_n w_n with active = {w_n - u_n beta / tau > 0}.
    The breakpoints are sorted, phi is evaluated at all of them with prefix
    sums, and the root is found on the bracketing linear piece.
    """
    w = np.ravel(w)
    u = np.ravel(u)
    nz = u != 0.0
    w, u = w[nz], u[nz]
    if w.size == 0:
        return 0.0
    b = tau * w / u
    order = np.argsort(b, kind="stable")
    b, w, u = b[order], w[order], u[order]
    pos = u > 0
    u2 = u * u / tau
    uw = u * w
    # slope and intercept on the piece just above breakpoint b_k:
    # u>0 voxels with b_n <= beta are inactive, u<0 voxels with b_n <= beta active
    # beta below every breakpoint: u>0 active, u<0 inactive.
    slope0 = 1.0 + np.sum(u2[pos])
    inter0 = np.sum(uw[~pos])
    # crossing breakpoint n (ascending): u>0 -> leaves active set; u<0 -> joins
    dslope = np.where(pos, -u2, u2)
    dinter = np.where(pos, uw, -uw)
    slope = slope0 + np.cumsum(dslope)          # slope just above b_k
    inter = inter0 + np.cumsum(dinter)
    phi_at_b = slope * b + inter                # phi is continuous at b_k
    k = np.searchsorted(phi_at_b, 0.0, side="left")
    if k == 0:
        return float(-inter0 / slope0)           # root below every breakpoint
    # root lies on the piece just above breakpoint k-1
    return float(-inter[k - 1] / slope[k - 1])


def _psi_fn(beta, wf, tau, U):
    """Psi(beta) = 1/2 ||beta||^2 + beta^T U^T w + tau/2 ||max(w - U beta / tau, 0)||^2,
    whose gradient is phi (Theorem 3.1)."""
    z = np.maximum(wf - U.T @ beta / tau, 0.0)
    return 0.5 * float(beta @ beta) + float(beta @ (U @ wf)) + 0.5 * tau * float(z @ z)


def root_phi_rank(w, tau, u, max_iter=200):
    """Root of phi for a metric factor of any rank r >= 1 (Theorem 3.1).

    phi is the gradient of the strongly convex piecewise-quadratic Psi; on
    the piece with active set A = {w - U beta / tau > 0} it is affine with
    Jacobian H = I + U_A^T U_A / tau.  The full Newton step -H^-1 phi is
    taken when it stays on its piece: it then lands on the root of that
    affine piece, i.e. the exact root.  Otherwise the step is shortened by
    backtracking on Psi (Armijo, factor 1/2), which converges globally.
    """
    wf = np.ravel(w)
    U = _cols(u, np.shape(w))
    r = U.shape[0]
    beta = np.zeros(r)
    for _ in range(max_iter):
        z = wf - U.T @ beta / tau
        A = z > 0
        g = U @ (wf - np.maximum(z, 0.0)) + beta
        H = np.eye(r) + (U[:, A] @ U[:, A].T) / tau
        d = -np.linalg.solve(H, g)
        full = beta + d
        if np.array_equal(wf - U.T @ full / tau > 0, A):
            return full
        psi0 = _psi_fn(beta, wf, tau, U)
        slope = float(g @ d)
        t = 1.0
        while _psi_fn(beta + t * d, wf, tau, U) > psi0 + 1e-4 * t * slope:
            t *= 0.5
            if t < 1e-20:
                raise RuntimeError("root_phi_rank: no decrease along the Newton direction")
        beta = beta + t * d
    raise RuntimeError("root_phi_rank did not terminate")


def weighted_projection_nonneg(w, tau, u):
    """prox^B_{iota_{R+}}(w) for B = tau I + U U^T (Theorem 3.1).

    Returns (x, beta*): beta* scalar for a rank-one u given as an image, a
    vector of length r otherwise (r = 0: plain projection, beta* = 0)."""
    U = _cols(u, np.shape(w))
    if U.shape[0] == 0:
        return np.maximum(w, 0.0), 0.0
    if np.shape(u) == np.shape(w):
        beta = root_phi_exact(w, tau, u)
        return np.maximum(w - u * beta / tau, 0.0), beta
    if U.shape[0] == 1:
        b = root_phi_exact(w, tau, U[0].reshape(np.shape(w)))
        beta = np.array([b])
    else:
        beta = root_phi_rank(w, tau, u)
    x = np.maximum(np.ravel(w) - U.T @ beta / tau, 0.0).reshape(np.shape(w))
    return x, beta


# --------------------------------------------------------------------------
# weighted proximal mapping by the fast dual projected gradient method
# --------------------------------------------------------------------------

def _primal(P, v, tau, u, lam, cset):
    w = v - lam * apply_B_inv(div_op(P), tau, u)
    if cset == "nonneg":
        x, beta = weighted_projection_nonneg(w, tau, u)
    else:
        x, beta = w, 0.0
    return x, beta


def wprox(v, tau, u, lam, kind="iso", cset="nonneg", n_iter=50, P0=None,
          return_dual=False):
    """argmin_{x in C} 1/2 ||x - v||^2_{tau I + U U^T} + lam TV(x).

    u: None, a rank-one image, or the r columns of U as an (r,) + shape array.

    Accelerated projected gradient on the dual (Section 4.1), P_0 = R_1 = P0
    (zero by default), t_1 = 1, n_iter iterations, output x(P_K).
    """
    v = np.asarray(v, dtype=np.float64)
    sigma = tau / (4.0 * DIM * lam)        # 1 / Lipschitz of Lemma 4.1 (x 2 lam)
    P_prev = np.zeros((DIM,) + v.shape) if P0 is None else np.array(P0, float)
    R = P_prev.copy()
    t = 1.0
    for _ in range(n_iter):
        x, _ = _primal(R, v, tau, u, lam, cset)
        P = project_dual(R + sigma * grad_op(x), kind)
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        R = P + ((t - 1.0) / t_new) * (P - P_prev)
        P_prev, t = P, t_new
    x, _ = _primal(P_prev, v, tau, u, lam, cset)
    if return_dual:
        return x, P_prev
    return x


def wprox_objective(x, v, tau, u, lam, kind):
    d = x - v
    return 0.5 * float(np.sum(d * apply_B(d, tau, u))) + lam * tv(x, kind)
