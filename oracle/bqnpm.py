"""Mini-batch quasi-Newton proximal method (oracle, FP64).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

* sr1 -- Algorithm 4.2: the metric B = tau I + u u^T of one subset from its
  last pair (s, m) of iterate and gradient differences.
* BQNPM -- Algorithm 4.1 with the choices of Section 4.3: strategy I
  (subset s' = mod(k, S), read as k - 1 mod S + 1 so that s' runs 1..S) or
  strategy II (s' drawn uniformly; the draws are an input), x_s^k = x_{k-1}
  and g_s^k = grad F_{s'}(x_{k-1}) for every s, the pairs
  (xbar_s, gbar_s) updated for s' only.

Readings (the paper is silent or its listing is ambiguous):
* a subset whose pair has no earlier distinct value (it was visited once)
  keeps B_s = alpha_s I, the setting of the first S iterations;
* in Algorithm 4.2, u is formed from the final tau after the curvature loop
  (u = (m - tau s) / sqrt(<m - tau s, s>)); the listing assigns u only
  inside the loop, which leaves it unset when the loop condition is false at
  entry, where the plain SR1 correction with the unhalved tau is meant;
* with x_s^k = x_{k-1} and g_s^k = g for every s, step 10 of Algorithm 4.1
  is v_k = x_{k-1} - a S Btilde^-1 g, Btilde = tau* I + U U^T with
  tau* = sum_s tau_s and U = [u_1 .. u_S] (zero columns kept), and the WPM
  of step 11 has weight a S lambda;
* the first S iterations (step 6) take the WPM with metric alpha_s I and
  weight a lambda of v = x_{k-1} - a g / alpha_s; the first-order variant
  (a proximal stochastic-gradient baseline) takes that step at every k.

Algorithm 4.2 is implemented as listed.  Note that its initial
tau = <m,m> / (gamma <s,m>) with gamma <= 1 gives, by Cauchy-Schwarz,
<m - tau s, s> < 0 whenever <s,m> > 0, so the rank-one correction is kept
only when tau_max clips tau.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import tvprox

DELTA1 = 1e-8
DELTA2 = 1e-12


def sr1(s, m, gamma, alpha, tau_max):
    """Algorithm 4.2.  Returns (tau, u) with u None when the rank-one
    correction is dropped; s, m are the iterate and gradient differences."""
    s = np.ravel(np.asarray(s, dtype=np.float64))
    m = np.ravel(np.asarray(m, dtype=np.float64))
    tau = float(m @ m) / (gamma * float(s @ m))
    tau = min(tau, tau_max)
    if tau <= 0.0:
        return alpha, None
    r = m - tau * s
    if float(r @ s) <= DELTA1 * math.sqrt(float(s @ s)) * math.sqrt(float(r @ r)):
        return tau, None
    while float((m - tau * s) @ s) <= DELTA2 * float(s @ s):
        if tau < DELTA2:
            return alpha, None
        tau = tau / 2.0
    r = m - tau * s
    return tau, r / math.sqrt(float(r @ s))


@dataclass
class BQNPMParams:
    S: int
    a: float            # step size a_k (constant)
    lam: float          # TV weight lambda
    alpha: float        # alpha_s, the same for every subset
    gamma: float = 0.8
    tau_max: float = 1e8
    tv: str = "iso"
    cset: str = "nonneg"
    prox_iters: int = 50
    first_order: bool = False   # metric alpha I at every iteration (no SR1)


@dataclass
class _Subset:
    xbar: np.ndarray | None = None
    gbar: np.ndarray | None = None
    tau: float = 0.0
    u: np.ndarray | None = None


@dataclass
class BQNPM:
    """State of Algorithm 4.1.  grad(s, x) returns grad F_s(x) (F_s with
    its S / L weight) for subset s in 0..S-1."""
    prm: BQNPMParams
    grad: object
    k: int = 0
    subsets: list = field(default_factory=list)

    def __post_init__(self):
        self.subsets = [_Subset(tau=self.prm.alpha) for _ in range(self.prm.S)]

    def pick(self, k, draw=None):
        """Subset of iteration k (1-based): k for k <= S, then strategy I
        (draw None) or the given draw in 0..S-1 (strategy II)."""
        S = self.prm.S
        if k <= S:
            return k - 1
        if draw is None:
            return (k - 1) % S
        return int(draw)

    def step(self, x, draw=None):
        """x_{k-1} -> x_k.  Returns (x_k, chosen subset, its (tau, u))."""
        p = self.prm
        self.k += 1
        k = self.k
        sp = self.pick(k, draw)
        g = self.grad(sp, x)
        sub = self.subsets[sp]
        if not p.first_order and sub.xbar is not None and not np.array_equal(sub.xbar, x):
            tau, u = sr1(x - sub.xbar, g - sub.gbar, p.gamma, p.alpha, p.tau_max)
            sub.tau, sub.u = tau, (None if u is None else u.reshape(x.shape))
        sub.xbar, sub.gbar = x.copy(), g.copy()
        if k <= p.S or p.first_order:
            v = x - p.a * g / p.alpha
            xn = tvprox.wprox(v, p.alpha, None, p.a * p.lam, p.tv, p.cset, n_iter=p.prox_iters)
            return xn, sp, (sub.tau, sub.u)
        taus = sum(b.tau for b in self.subsets)
        U = np.stack([b.u if b.u is not None else np.zeros_like(x) for b in self.subsets])
        v = x - p.a * p.S * tvprox.apply_B_inv(g, taus, U)
        xn = tvprox.wprox(v, taus, U, p.a * p.S * p.lam, p.tv, p.cset, n_iter=p.prox_iters)
        return xn, sp, (sub.tau, sub.u)
