"""Pins of the oracle's weighted TV proximal mapping.

* D and D^T are exact transposes; ||d||^2 <= 4D (Appendix B, proof of
  Lemma 4.1) and the bound is approached on a large grid;
* the dual representation of TV (Section 3.3): max over the dual set is
  attained at the normalised gradient;
* exact root of phi (Theorem 3.1, rank one) vs bisection to machine
  precision and a brute-force piece enumeration;
* weighted projection onto the nonnegative orthant under tau I + u u^T vs
  enumeration of all active sets with KKT multipliers (independent of
  Theorem 3.1);
* metrics tau I + U U^T of rank r >= 2: the root of phi (Theorem 3.1) and
  the projection vs active-set enumeration, the Woodbury inverse vs a dense
  inverse, a zero column changes nothing, rank one through the rank-r
  routine equals the breakpoint root;
* the weighted prox itself vs an independent ADMM solver with dense linear
  solves, on tiny grids, for iso/aniso TV, with and without the constraint,
  for metric ranks 0, 1 and 2;
* with u = 0 and tau = 1 the iteration is the Beck-Teboulle fast gradient
  projection for constrained TV denoising.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import tvprox as tp


def test_diff_transpose_and_norm_bound():
    rng = np.random.default_rng(0)
    shape = (5, 6, 7)
    x = rng.standard_normal(shape)
    P = rng.standard_normal((3,) + shape)
    lhs = np.sum(tp.grad_op(x) * P)
    rhs = np.sum(x * tp.div_op(P))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # power iteration on d d^T: largest eigenvalue -> 4D = 12 from below
    y = rng.standard_normal((24, 24, 24))
    lam = 0.0
    for _ in range(400):
        y = tp.div_op(tp.grad_op(y))
        lam = np.linalg.norm(y)
        y /= lam
    assert 11.8 < lam <= 12.0


def test_forward_difference_values():
    x = np.arange(2 * 3 * 4, dtype=float).reshape(2, 3, 4) ** 2
    g = tp.grad_op(x)
    assert g[2][1, 2, 1] == x[1, 2, 2] - x[1, 2, 1]
    assert g[1][0, 1, 3] == x[0, 2, 3] - x[0, 1, 3]
    assert g[0][0, 2, 2] == x[1, 2, 2] - x[0, 2, 2]
    assert np.all(g[2][..., -1] == 0) and np.all(g[1][:, -1] == 0) and np.all(g[0][-1] == 0)


@pytest.mark.parametrize("kind", ["iso", "aniso"])
def test_tv_dual_representation(kind):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 5, 4))
    g = tp.grad_op(x)
    if kind == "iso":
        nrm = np.sqrt(np.sum(g * g, axis=0))
        Pst = g / np.where(nrm > 0, nrm, 1.0)
    else:
        Pst = np.sign(g)
    assert np.sum(tp.div_op(Pst) * x) == pytest.approx(tp.tv(x, kind), rel=1e-13)
    for _ in range(20):
        P = tp.project_dual(3 * rng.standard_normal(g.shape), kind)
        assert np.sum(tp.div_op(P) * x) <= tp.tv(x, kind) + 1e-12


def _bisect_root(w, tau, u):
    lo, hi = -1.0, 1.0
    while tp.phi(lo, w, tau, u) > 0:
        lo *= 2
    while tp.phi(hi, w, tau, u) < 0:
        hi *= 2
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tp.phi(mid, w, tau, u) < 0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_exact_root_matches_bisection():
    rng = np.random.default_rng(2)
    for trial in range(20):
        n = int(rng.integers(1, 400))
        w = rng.standard_normal(n) * rng.uniform(0.01, 3)
        u = rng.standard_normal(n) * rng.uniform(0.01, 3)
        u[rng.random(n) < 0.1] = 0.0
        tau = float(rng.uniform(0.05, 5))
        b = tp.root_phi_exact(w, tau, u)
        ref = _bisect_root(w, tau, u)
        assert abs(b - ref) <= 1e-12 * max(1.0, abs(ref))
        assert abs(tp.phi(b, w, tau, u)) <= 1e-12 * (1 + np.sum(np.abs(u * w)))


def test_exact_root_tiny_brute_force():
    # every sign pattern of the 3 ramps: solve each linear piece, keep the
    # one whose active set is self-consistent
    w = np.array([0.7, -0.3, 0.2])
    u = np.array([0.9, 0.5, -1.1])
    tau = 0.4
    sols = []
    for act in itertools.product([False, True], repeat=3):
        a = np.array(act)
        slope = 1 + np.sum(u[a] ** 2) / tau
        beta = -np.sum((u * w)[~a]) / slope
        if np.array_equal(w - u * beta / tau > 0, a):
            sols.append(beta)
    assert len(sols) >= 1
    assert all(abs(s - sols[0]) < 1e-14 for s in sols)
    assert tp.root_phi_exact(w, tau, u) == pytest.approx(sols[0], abs=1e-15)


def test_weighted_projection_vs_active_set_enumeration():
    rng = np.random.default_rng(3)
    n = 10
    for _ in range(15):
        w = rng.standard_normal(n)
        u = rng.standard_normal(n) * rng.uniform(0.1, 2)
        tau = float(rng.uniform(0.1, 3))
        B = tau * np.eye(n) + np.outer(u, u)
        best = None
        for act in itertools.product([False, True], repeat=n):
            S = np.array(act)
            x = np.zeros(n)
            if S.any():
                x[S] = w[S] + np.linalg.solve(B[np.ix_(S, S)], B[np.ix_(S, ~S)] @ w[~S])
            mu = (B @ (x - w))[~S]
            if np.all(x[S] >= -1e-13) and np.all(mu >= -1e-13):
                best = x
                break
        assert best is not None
        got, beta = tp.weighted_projection_nonneg(w, tau, u)
        assert np.max(np.abs(got - best)) < 1e-12
        # KKT reading of Theorem 3.1: beta* = u^T (prox - w)
        assert beta == pytest.approx(float(u @ (got - w)), abs=1e-12)


def _dense_D(shape):
    n = int(np.prod(shape))
    rows = []
    for a in range(3):
        Da = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1
            Da[:, j] = tp.diff(e.reshape(shape), a).ravel()
        rows.append(Da)
    return rows


def _admm_wprox(v, tau, u, lam, kind, cset, iters=30000, rho=1.0):
    """Independent solver: ADMM on x with z = D x (TV) and y = x (C)."""
    shape = v.shape
    n = v.size
    Ds = _dense_D(shape)
    D = np.vstack(Ds)
    Uc = tp._cols(u, shape)
    B = tau * np.eye(n) + Uc.T @ Uc
    M = B + rho * (D.T @ D) + rho * np.eye(n)
    Minv = np.linalg.inv(M)
    vv = v.ravel()
    x = vv.copy()
    z = D @ x
    y = x.copy()
    a = np.zeros_like(z)
    b = np.zeros(n)
    Bv = B @ vv
    for _ in range(iters):
        x = Minv @ (Bv + rho * D.T @ (z - a) + rho * (y - b))
        Dx = D @ x
        q = (Dx + a).reshape(3, n)
        if kind == "iso":
            nrm = np.sqrt(np.sum(q * q, axis=0))
            shrink = np.maximum(1 - (lam / rho) / np.where(nrm > 0, nrm, 1), 0)
            z = (q * shrink).ravel()
        else:
            z = (np.sign(q) * np.maximum(np.abs(q) - lam / rho, 0)).ravel()
        y = np.maximum(x + b, 0) if cset == "nonneg" else x + b
        a += Dx - z
        b += x - y
    return y.reshape(shape) if cset == "nonneg" else x.reshape(shape)


@pytest.mark.slow
@pytest.mark.parametrize("kind,cset,shape,rank", [
    ("iso", "nonneg", (4, 4, 4), 1),
    ("aniso", "nonneg", (3, 3, 5), 1),
    ("iso", "none", (3, 4, 3), 1),
    ("aniso", "nonneg", (4, 3, 3), 0),
    ("iso", "nonneg", (3, 4, 4), 2),
    ("aniso", "nonneg", (3, 3, 4), 3),
])
def test_wprox_matches_admm(kind, cset, shape, rank):
    rng = np.random.default_rng(4)
    v = rng.standard_normal(shape) * 0.5 + 0.1
    if rank == 0:
        u = None
    elif rank == 1:
        u = 0.3 * rng.standard_normal(shape)
    else:
        u = 0.3 * rng.standard_normal((rank,) + shape)
    tau, lam = 0.7, 0.15
    x_fgp = tp.wprox(v, tau, u, lam, kind, cset, n_iter=20000)
    x_admm = _admm_wprox(v, tau, u, lam, kind, cset)
    assert np.max(np.abs(x_fgp - x_admm)) < 1e-10
    o1 = tp.wprox_objective(x_fgp, v, tau, u, lam, kind)
    o2 = tp.wprox_objective(np.maximum(x_admm, 0) if cset == "nonneg" else x_admm,
                            v, tau, u, lam, kind)
    assert o1 <= o2 + 1e-10
    if cset == "nonneg":
        assert np.all(x_fgp >= 0)


def test_unweighted_case_is_beck_teboulle():
    """u = None, tau = 1: x_k = P_C(b - lam d(R_k)), P_k = Proj(R_k +
    d^T(x_k) / (4 D lam)), FISTA momentum -- written out independently."""
    rng = np.random.default_rng(5)
    b = rng.standard_normal((5, 4, 6))
    lam = 0.2
    K = 30
    Pp = np.zeros((3,) + b.shape)
    R = Pp.copy()
    t = 1.0
    for _ in range(K):
        x = np.maximum(b - lam * tp.div_op(R), 0)
        P = tp.project_dual(R + tp.grad_op(x) / (12 * lam), "iso")
        tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
        R = P + (t - 1) / tn * (P - Pp)
        Pp, t = P, tn
    ref = np.maximum(b - lam * tp.div_op(Pp), 0)
    got = tp.wprox(b, 1.0, None, lam, "iso", "nonneg", n_iter=K)
    assert np.max(np.abs(got - ref)) < 1e-14
    # the rank-one code path with u = 0 gives the same iterates
    got0 = tp.wprox(b, 1.0, np.zeros_like(b), lam, "iso", "nonneg", n_iter=K)
    assert np.max(np.abs(got0 - ref)) < 1e-14


def _enumerate_projection(w, B):
    """argmin_{x >= 0} 1/2 (x - w)^T B (x - w) by enumerating the free set and
    checking the KKT multipliers (independent of Theorem 3.1)."""
    n = w.size
    for act in itertools.product([True, False], repeat=n):
        S = np.array(act)
        x = np.zeros(n)
        if S.any():
            x[S] = w[S] + np.linalg.solve(B[np.ix_(S, S)], B[np.ix_(S, ~S)] @ w[~S])
        mu = (B @ (x - w))[~S]
        if np.all(x[S] >= -1e-13) and np.all(mu >= -1e-13):
            return x
    raise AssertionError("no KKT point")


@pytest.mark.parametrize("r", [2, 3, 5])
def test_rank_r_projection_vs_active_set_enumeration(r):
    rng = np.random.default_rng(30 + r)
    n = 10
    for _ in range(8):
        w = rng.standard_normal((1, 2, 5))
        U = rng.standard_normal((r, 1, 2, 5)) * rng.uniform(0.1, 1.5)
        tau = float(rng.uniform(0.1, 3))
        Uc = U.reshape(r, n)
        B = tau * np.eye(n) + Uc.T @ Uc
        ref = _enumerate_projection(w.ravel(), B)
        got, beta = tp.weighted_projection_nonneg(w, tau, U)
        assert np.max(np.abs(got.ravel() - ref)) < 1e-12
        # KKT reading of Theorem 3.1: beta* = U^T (prox - w), and phi(beta*) = 0
        assert np.max(np.abs(beta - Uc @ (got.ravel() - w.ravel()))) < 1e-12
        assert np.max(np.abs(tp.phi(beta, w, tau, U))) < 1e-12


def test_rank_r_root_consistency():
    rng = np.random.default_rng(40)
    shape = (6, 7, 5)
    w = rng.standard_normal(shape)
    u = rng.standard_normal(shape) * 0.7
    tau = 0.4
    # rank one through the rank-r Newton routine equals the breakpoint root
    b1 = tp.root_phi_exact(w, tau, u)
    br = tp.root_phi_rank(w, tau, u[None])
    assert abs(br[0] - b1) < 1e-13 * max(1.0, abs(b1))
    # a zero column changes nothing (its beta component is 0)
    U2 = np.stack([u, np.zeros(shape)])
    x2, beta2 = tp.weighted_projection_nonneg(w, tau, U2)
    x1, _ = tp.weighted_projection_nonneg(w, tau, u)
    assert np.max(np.abs(x2 - x1)) < 1e-13 and abs(beta2[1]) < 1e-15
    # column order does not matter
    U3 = rng.standard_normal((3,) + shape)
    xa, ba = tp.weighted_projection_nonneg(w, tau, U3)
    xb, bb = tp.weighted_projection_nonneg(w, tau, U3[::-1])
    assert np.max(np.abs(xa - xb)) < 1e-12 and np.max(np.abs(ba - bb[::-1])) < 1e-12


@pytest.mark.parametrize("r", [1, 2, 4])
def test_woodbury_inverse_rank_r(r):
    rng = np.random.default_rng(50 + r)
    shape = (3, 4, 5)
    n = 60
    U = rng.standard_normal((r,) + shape)
    y = rng.standard_normal(shape)
    tau = 0.3
    B = tau * np.eye(n) + U.reshape(r, n).T @ U.reshape(r, n)
    ref = np.linalg.solve(B, y.ravel())
    got = tp.apply_B_inv(y, tau, U)
    assert np.max(np.abs(got.ravel() - ref)) < 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(tp.apply_B(got, tau, U) - y)) < 1e-12
