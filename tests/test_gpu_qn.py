"""GPU parity of the mini-batch quasi-Newton outer iteration (Algorithm 4.1,
SR1 metrics of Algorithm 4.2, strategies I/II of Section 4.3) against the
oracle's.

A 24^3 LS problem with L = 4 illuminations in S = 2 subsets, started from
x_0 = 0; every iterate x_k of the first 2S + 3 iterations is compared.
tau_max is set below the curvature scale so that Algorithm 4.2 keeps the
rank-one corrections for some subsets (mixed branches, rank-2 WPM metrics).
Both sides solve to tol 1e-13.  Tolerances: FP64 1e-9 relative per iterate
(gradient and prox parity are 1e-10 each; the SR1 scalars are ratios of
inner products of iterate and gradient differences); FP32 2e-3 (the 2e-4
per-call bound of the FP32 gradient and prox, accumulated over 7
iterations).
"""
import functools

import numpy as np
import pytest

import synthetic as syn
from oracle import bqnpm, lsmodel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, L, S = 24, 4, 2
H = syn.LAMBDA0_UM / 4
SUBSETS = [[0, 1], [2, 3]]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@functools.lru_cache(maxsize=None)
def _problem():
    rng = np.random.default_rng(21)
    xt = syn.scattering_potential(syn.phantom_ellipsoids(N, H, rng))
    dirs = syn.illumination_directions(L, 35.0, np.random.default_rng(22))
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B)
    m = lsmodel.LSModel(geom)
    y, _ = m.forward(xt, dirs, list(range(L)), 1e-13, 400)
    return xt, dirs, m, y


def _params(tau_max):
    xt, dirs, m, y = _problem()
    g0 = m.grad(np.zeros_like(xt), y[SUBSETS[0]], dirs, SUBSETS[0], S / L, 1e-13, 400)[0]
    alpha = float(np.abs(g0).max() / xt.max())
    return dict(S=S, a=0.5, lam=1e-5, alpha=alpha, gamma=0.8, tau_max=tau_max, prox_iters=30)


@functools.lru_cache(maxsize=None)
def _oracle_run(tau_max, draws, warm=False, first_order=False):
    xt, dirs, m, y = _problem()
    prm = bqnpm.BQNPMParams(**_params(tau_max), first_order=first_order)
    store = {}

    def grad(s, x):
        starts = store.get(s) if warm else None
        g, _, _, fields = m.grad(x, y[SUBSETS[s]], dirs, SUBSETS[s], S / L, 1e-13, 400, starts=starts,
                                 return_fields=True)
        store[s] = fields
        return g
    it = bqnpm.BQNPM(prm, grad)
    x = np.zeros_like(xt)
    out = []
    for k, d in enumerate(draws):
        x, sp, (tau, u) = it.step(x, None if d < 0 else d)
        out.append((x.copy(), sp, tau, u is not None))
    return out


def _gpu_run(dev, prec, tau_max, draws, warm=False, first_order=False):
    from paper_2307_02043_amd import LSContext, QNIteration, WProx
    xt, dirs, m, y = _problem()
    p = _params(tau_max)
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    ls = LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision=prec, tol=tol, max_iter=400)
    px = WProx((N, N, N), prec)
    qn = QNIteration(ls, px, SUBSETS, p["a"], p["lam"], p["alpha"], p["gamma"], p["tau_max"],
                     prox_iters=p["prox_iters"], warm_start=warm, first_order=first_order)
    x = torch.zeros((N, N, N), dtype=rd, device=dev)
    yt = torch.from_numpy(y).to(dev, cd)
    out = []
    for d in draws:
        info = qn.step(x, yt, int(d))
        out.append((x.cpu().numpy().astype(np.float64), info))
    qn.close()
    px.close()
    ls.close()
    return out


STRAT_I = (-1,) * (2 * S + 3)
STRAT_II = (-1, -1, 1, 1, 0, 1, 0)  # draws of strategy II for k > S (ignored for k <= S)


@pytest.mark.parametrize("tau_max,draws", [(5e-5, STRAT_I), (2e-5, STRAT_II)])
def test_qn_iteration_f64_matches_oracle(dev, tau_max, draws):
    ref = _oracle_run(tau_max, draws)
    got = _gpu_run(dev, "f64", tau_max, draws)
    kept = 0
    state = [0] * S  # whether each subset currently holds a rank-one correction
    for k, ((xr, sp, tau, uk), (xg, info)) in enumerate(zip(ref, got), start=1):
        assert info.k == k and info.subset == sp, (k, info.subset, sp)
        assert info.u_kept == uk, k
        assert abs(info.tau - tau) <= 1e-9 * abs(tau), (k, info.tau, tau)
        state[sp] = int(uk)
        # only the kept corrections enter the metric (the others are zero columns)
        assert info.metric_rank == (0 if k <= S else sum(state)), (k, info.metric_rank, state)
        err = _rel(xg, xr)
        assert err < 1e-9, (k, err)
        kept += uk
    assert kept >= 2   # the rank-one corrections were exercised
    assert np.all(got[-1][0] >= 0)


def test_qn_iteration_f32_matches_oracle(dev):
    ref = _oracle_run(5e-5, STRAT_I)
    got = _gpu_run(dev, "f32", 5e-5, STRAT_I)
    for k, ((xr, sp, tau, uk), (xg, info)) in enumerate(zip(ref, got), start=1):
        assert info.subset == sp
        err = _rel(xg, xr)
        assert err < 2e-3, (k, err)


def test_qn_rejects_bad_arguments(dev):
    from paper_2307_02043_amd import BQError, LSContext, QNIteration, WProx
    xt, dirs, m, y = _problem()
    ls = LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision="f64")
    px32 = WProx((N, N, N), "f32")
    with pytest.raises(BQError):          # precision mismatch
        QNIteration(ls, px32, SUBSETS, 0.5, 1e-5, 1.0)
    px = WProx((N, N, N), "f64")
    with pytest.raises(BQError):          # index out of range
        QNIteration(ls, px, [[0, 7]], 0.5, 1e-5, 1.0)
    with pytest.raises(BQError):          # gamma outside (0, 1]
        QNIteration(ls, px, SUBSETS, 0.5, 1e-5, 1.0, gamma=1.5)
    with pytest.raises(BQError):          # S above the largest metric rank
        QNIteration(ls, px, [[0]] * 9, 0.5, 1e-5, 1.0)
    qn = QNIteration(ls, px, SUBSETS, 0.5, 1e-5, 1.0, prox_iters=2)
    x = torch.zeros((N, N, N), dtype=torch.float64, device=dev)
    yt = torch.from_numpy(y).to(dev)
    qn.step(x, yt)
    qn.step(x, yt)
    with pytest.raises(BQError):          # draw outside 0..S-1
        qn.step(x, yt, 5)
    qn.close()
    px.close()
    px32.close()
    ls.close()


@pytest.mark.parametrize("warm,first_order", [(True, False), (False, True), (True, True)])
def test_qn_variants_f64_match_oracle(dev, warm, first_order):
    """Warm-started solves across outer iterations and the first-order
    (alpha I) variant of the outer loop, against the oracle."""
    ref = _oracle_run(5e-5, STRAT_I, warm, first_order)
    got = _gpu_run(dev, "f64", 5e-5, STRAT_I, warm, first_order)
    for k, ((xr, sp, tau, uk), (xg, info)) in enumerate(zip(ref, got), start=1):
        assert info.subset == sp
        if first_order:
            assert info.metric_rank == 0 and info.tau_sum == _params(5e-5)["alpha"]
        err = _rel(xg, xr)
        assert err < 1e-9, (k, err)


def test_qn_iteration_f32_single_steps_match_oracle(dev):
    """Per-step FP32 error, apart from its accumulation over iterations: the
    oracle follows the GPU's own trajectory (each of its steps starts from
    the GPU's x_{k-1}, so its subset pairs (xbar, gbar) and SR1 metrics are
    those exact arithmetic gives on that trajectory), and every GPU step is
    compared with the oracle step from the same point at 2e-4."""
    got = _gpu_run(dev, "f32", 5e-5, STRAT_I)
    xt, dirs, m, y = _problem()
    prm = bqnpm.BQNPMParams(**_params(5e-5))

    def grad(s, x):
        return m.grad(x, y[SUBSETS[s]], dirs, SUBSETS[s], S / L, 1e-13, 400)[0]
    it = bqnpm.BQNPM(prm, grad)
    x = np.zeros_like(xt)
    worst = 0.0
    for k, (xg, info) in enumerate(got, start=1):
        xr, sp, _ = it.step(x)
        assert info.subset == sp
        err = _rel(xg, xr)
        worst = max(worst, err)
        assert err < 2e-4, (k, err)
        x = xg
    print(f"FP32 outer iteration: worst single-step relative error {worst:.2e}")
