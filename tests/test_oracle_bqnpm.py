"""Pins of the oracle's SR1 metric (Algorithm 4.2) and outer iteration
(Algorithm 4.1 with the strategies of Section 4.3).

* SR1: every branch of Algorithm 4.2 on hand-built pairs with known
  outcome; the secant equation B s = m whenever the rank-one correction is
  kept; m = c s gives tau = c / gamma without correction;
* outer iteration: on separable quadratics F_s(x) = h/2 ||x - c_s||^2 with
  a negligible TV weight and no constraint, the first S iterations are
  gradient steps of length a / alpha and the later ones steps of length
  a S / tau* (SR1 finds B_s = (h / gamma) I for every subset revisited so
  far, the others keep alpha I) -- a closed-form recursion; strategy I
  visits the subsets
  cyclically; the metric handed to the prox has rank S once tau_max binds.
"""
import math

import numpy as np
import pytest

from oracle import bqnpm, tvprox


def test_sr1_proportional_pair():
    rng = np.random.default_rng(0)
    s = rng.standard_normal(50)
    for c, gamma in ((2.0, 0.8), (0.3, 0.5), (5.0, 1.0)):
        tau, u = bqnpm.sr1(s, c * s, gamma, 7.0, 1e8)
        assert u is None
        assert tau == pytest.approx(c / gamma, rel=1e-14)


def test_sr1_negative_curvature_resets_to_alpha():
    s = np.array([1.0, 0.0, 2.0])
    m = np.array([-1.0, 0.5, -0.3])       # <s, m> < 0
    assert bqnpm.sr1(s, m, 0.8, 3.5, 1e8) == (3.5, None)


def test_sr1_tau_max_keeps_correction_and_secant_equation():
    s = np.array([1.0, 0.0])
    m = np.array([1.0, 1.0])               # tau = 2 / 0.8 = 2.5 -> clipped to 0.5
    tau, u = bqnpm.sr1(s, m, 0.8, 1.0, 0.5)
    assert tau == 0.5
    np.testing.assert_allclose(u, np.array([0.5, 1.0]) / math.sqrt(0.5), rtol=1e-15)
    B = tau * np.eye(2) + np.outer(u, u)
    np.testing.assert_allclose(B @ s, m, rtol=1e-15, atol=1e-15)
    # random pairs: whenever u is kept, (tau I + u u^T) s = m
    rng = np.random.default_rng(1)
    kept = 0
    for _ in range(200):
        s = rng.standard_normal(20)
        m = s * rng.uniform(0.5, 2.0) + 0.3 * rng.standard_normal(20)
        tau, u = bqnpm.sr1(s, m, 0.8, 1.0, float(rng.uniform(0.05, 1.0)))
        if u is not None:
            kept += 1
            np.testing.assert_allclose(tau * s + u * (u @ s), m, rtol=1e-12, atol=1e-12)
    assert kept > 20


def test_sr1_angle_test_drops_correction():
    # <m - tau s, s> <= delta1 |s| |m - tau s| after clipping: u dropped, tau kept
    s = np.array([1.0, 0.0])
    m = np.array([0.5, 3.0])               # tau = 9.25 / 0.4 -> clipped to 0.5, r = (0, 3)
    tau, u = bqnpm.sr1(s, m, 0.8, 1.0, 0.5)
    assert tau == 0.5 and u is None


def test_sr1_curvature_loop_halves_tau():
    s = np.array([1.0, 0.0])
    tmax = 0.25
    m = np.array([tmax + 1e-13, 1e-13])    # <m - tmax s, s> = 1e-13 <= delta2 |s|^2
    tau, u = bqnpm.sr1(s, m, 0.8, 1.0, tmax)
    assert tau == tmax / 2
    r = m - tau * s
    np.testing.assert_allclose(u, r / math.sqrt(r @ s), rtol=1e-14)
    np.testing.assert_allclose(tau * s + u * (u @ s), m, rtol=1e-14)


def test_sr1_curvature_loop_resets_small_tau():
    s = np.array([1.0, 0.0])
    tmax = 4e-13                           # below delta2 = 1e-12 when the loop starts
    m = np.array([tmax + 1e-13, 1e-20])
    assert bqnpm.sr1(s, m, 0.8, 2.0, tmax) == (2.0, None)


def _quadratic_problem(S, shape, h, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((S,) + shape)

    def grad(s, x):
        return h * (x - c[s])
    return c, grad


@pytest.mark.parametrize("S", [1, 3, 4])
def test_outer_iteration_on_separable_quadratic(S):
    shape = (4, 5, 6)
    h, a, alpha, gamma = 1.7, 0.3, 2.0, 0.8
    c, grad = _quadratic_problem(S, shape, h, 10 + S)
    prm = bqnpm.BQNPMParams(S=S, a=a, lam=1e-13, alpha=alpha, gamma=gamma, tau_max=1e8,
                            cset="none", prox_iters=3)
    it = bqnpm.BQNPM(prm, grad)
    x = np.zeros(shape)
    xr = x.copy()
    for k in range(1, 3 * S + 3):
        x, sp, (tau, u) = it.step(x)
        assert sp == (k - 1) % S               # k <= S: s' = k; then strategy I
        if k <= S:
            step = a / alpha
        else:
            # subsets revisited so far have B_s = (h / gamma) I, the others alpha I
            nr = min(k - S, S)
            step = a * S / (nr * h / gamma + (S - nr) * alpha)
        xr = xr - step * h * (xr - c[sp])
        np.testing.assert_allclose(x, xr, rtol=1e-9, atol=1e-11)
        if k > S:
            assert u is None and tau == pytest.approx(h / gamma, rel=1e-12)


def test_outer_iteration_rank_S_metric_when_tau_max_binds():
    """A non-separable quadratic (F_s(x) = 1/2 |A_s x - b_s|^2 on a small
    image) with tau_max below the curvature scale: the subsets keep their
    rank-one corrections, and the prox receives tau* I + U U^T with S
    columns -- checked against a dense evaluation of step 10."""
    S, shape = 3, (2, 3, 4)
    n = 24
    rng = np.random.default_rng(5)
    A = rng.standard_normal((S, n, n)) / math.sqrt(n)
    b = rng.standard_normal((S, n))

    def grad(s, x):
        return (A[s].T @ (A[s] @ x.ravel() - b[s])).reshape(shape)
    prm = bqnpm.BQNPMParams(S=S, a=0.5, lam=1e-3, alpha=1.0, gamma=0.8, tau_max=0.05,
                            cset="nonneg", prox_iters=200)
    it = bqnpm.BQNPM(prm, grad)
    x = np.abs(rng.standard_normal(shape))
    for k in range(1, 2 * S + 2):
        xprev = x
        x, sp, (tau, u) = it.step(x)
        if k > 2 * S:
            subs = it.subsets
            assert all(sb.u is not None for sb in subs)
            taus = sum(sb.tau for sb in subs)
            U = np.stack([sb.u.ravel() for sb in subs])
            Bt = taus * np.eye(n) + U.T @ U
            g = grad(sp, xprev).ravel()
            v = xprev.ravel() - prm.a * S * np.linalg.solve(Bt, g)
            ref = tvprox.wprox(v.reshape(shape), taus, U.reshape((S,) + shape), prm.a * S * prm.lam,
                               "iso", "nonneg", n_iter=200)
            np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-13)
    assert np.all(x >= 0)


def test_subset_choice_strategies():
    """Section 4.3: the first S iterations visit the subsets in order; then
    strategy I cycles through them and strategy II takes the given draw."""
    prm = bqnpm.BQNPMParams(S=3, a=0.1, lam=1e-3, alpha=1.0)
    it = bqnpm.BQNPM(prm, lambda s, x: x)
    assert [it.pick(k) for k in range(1, 4)] == [0, 1, 2]
    assert [it.pick(k, draw=2) for k in range(1, 4)] == [0, 1, 2]   # draws ignored for k <= S
    assert [it.pick(k) for k in range(4, 10)] == [0, 1, 2, 0, 1, 2]
    assert [it.pick(k, draw=d) for k, d in zip(range(4, 8), [2, 2, 0, 1])] == [2, 2, 0, 1]
