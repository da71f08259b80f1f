"""GPU parity of the weighted TV proximal mapping against the CPU oracle.

Same number of dual iterations on both sides; the oracle finds Theorem 3.1's
root exactly by sorting breakpoints, the GPU by safeguarded semi-smooth
Newton.  Tolerances (relative l2 on x): 1e-10 FP64, 2e-4 FP32.
"""
import numpy as np
import pytest

import synthetic as syn
from oracle import tvprox as tp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _inputs(shape, seed):
    rng = np.random.default_rng(seed)
    v = 0.02 * rng.random(shape) + 0.005 * rng.standard_normal(shape)
    u = 0.1 * rng.standard_normal(shape)
    return v, u


def _run(dev, shape, prec, v, tau, u, lam, tv, cset, n_iter, P=None):
    from paper_2307_02043_amd import WProx
    rd = torch.float64 if prec == "f64" else torch.float32
    px = WProx(shape, prec)
    Pt = None if P is None else torch.from_numpy(np.ascontiguousarray(P)).to(dev, rd)
    x, info = px(torch.from_numpy(v).to(dev, rd), tau,
                 None if u is None else torch.from_numpy(u).to(dev, rd),
                 lam, tv, cset, n_iter, P=Pt)
    out = x.cpu().numpy().astype(np.float64), info, (None if Pt is None else Pt.cpu().numpy())
    px.close()
    return out


@pytest.mark.parametrize("shape", [(13, 17, 19), (16, 16, 16)])
@pytest.mark.parametrize("tv", ["iso", "aniso"])
@pytest.mark.parametrize("cset", ["nonneg", "none"])
@pytest.mark.parametrize("rank", [1, 0])
def test_wprox_f64_matches_oracle(dev, shape, tv, cset, rank):
    v, u = _inputs(shape, sum(shape) + rank)
    u = u if rank else None
    ref = tp.wprox(v, 0.8, u, 2e-3, tv, cset, n_iter=30)
    got, info, _ = _run(dev, shape, "f64", v, 0.8, u, 2e-3, tv, cset, 30)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)
    if cset == "nonneg":
        assert np.all(got >= 0)
    if rank and cset == "nonneg":
        assert info.newton_max <= 8 and info.newton_total >= 31


@pytest.mark.parametrize("tv", ["iso", "aniso"])
def test_wprox_f32_matches_oracle(dev, tv):
    shape = (20, 24, 28)
    v, u = _inputs(shape, 77)
    ref = tp.wprox(v, 1.0, u, 1e-3, tv, "nonneg", n_iter=40)
    got, info, _ = _run(dev, shape, "f32", v, 1.0, u, 1e-3, tv, "nonneg", 40)
    assert _rel(got, ref) < 2e-4, _rel(got, ref)


def test_wprox_c1_workload(dev):
    """32^3 isotropic prox of the first workload: lambda 1e-3, 50 iterations,
    nonnegativity, metric tau I + u u^T."""
    w = syn.WORKLOADS["c1_ls32_f64"]
    v, tau, u = syn.prox_inputs(w)
    ref = tp.wprox(v, tau, u, w.prox_lambda, "iso", "nonneg", n_iter=w.prox_iters)
    for prec, tol in (("f64", 1e-10), ("f32", 2e-4)):
        got, info, _ = _run(dev, v.shape, prec, v, tau, u, w.prox_lambda, "iso", "nonneg", w.prox_iters)
        assert _rel(got, ref) < tol, (prec, _rel(got, ref))


@pytest.mark.slow
def test_wprox_c2_workload_aniso(dev):
    """64^3 anisotropic prox, 100 iterations (second workload)."""
    w = syn.WORKLOADS["c2_born64_f32"]
    v, tau, u = syn.prox_inputs(w)
    ref = tp.wprox(v, tau, u, w.prox_lambda, "aniso", "nonneg", n_iter=w.prox_iters)
    got, info, _ = _run(dev, v.shape, "f32", v, tau, u, w.prox_lambda, "aniso", "nonneg", w.prox_iters)
    assert _rel(got, ref) < 2e-4


def test_wprox_warm_start_and_zero_iterations(dev):
    shape = (12, 14, 10)
    v, u = _inputs(shape, 5)
    # n_iter = 0: x = prox^B_C(v) (Theorem 3.1 projection only)
    got0, _, _ = _run(dev, shape, "f64", v, 0.5, u, 1e-3, "iso", "nonneg", 0)
    ref0, _ = tp.weighted_projection_nonneg(v, 0.5, u)
    assert _rel(got0, ref0) < 1e-12
    # dual warm start: continue from P_20 for 15 more iterations
    x20, P20 = tp.wprox(v, 0.5, u, 1e-3, "iso", "nonneg", n_iter=20, return_dual=True)
    ref = tp.wprox(v, 0.5, u, 1e-3, "iso", "nonneg", n_iter=15, P0=P20)
    P = np.zeros((3,) + shape)
    got20, _, Pg = _run(dev, shape, "f64", v, 0.5, u, 1e-3, "iso", "nonneg", 20, P=P)
    assert _rel(got20, x20) < 1e-10 and _rel(Pg, P20) < 1e-10
    got, _, _ = _run(dev, shape, "f64", v, 0.5, u, 1e-3, "iso", "nonneg", 15, P=Pg)
    assert _rel(got, ref) < 1e-10


def test_wprox_rejects_bad_arguments(dev):
    from paper_2307_02043_amd import BQError, WProx
    px = WProx((8, 8, 8), "f64")
    v = torch.zeros((8, 8, 8), dtype=torch.float64, device=dev)
    with pytest.raises(BQError):
        px(v, -1.0, None, 1e-3)
    with pytest.raises(BQError):
        px(v, 1.0, None, 0.0)
    px.close()


def test_wprox_graph_replays_are_stable(dev):
    """The dual iteration runs as a captured graph replayed n_iter times;
    repeated calls with unrelated eager GPU work and synchronisations in
    between give bitwise identical results that match the oracle."""
    from paper_2307_02043_amd import WProx
    shape = (18, 20, 22)
    v, u = _inputs(shape, 9)
    ref = tp.wprox(v, 0.6, u, 1.5e-3, "iso", "nonneg", n_iter=25)
    px = WProx(shape, "f64")
    vt = torch.from_numpy(v).to(dev)
    ut = torch.from_numpy(u).to(dev)
    first = None
    for rep in range(4):
        junk = torch.randn(1 << 20, device=dev).cumsum(0)  # eager work between replays
        torch.cuda.synchronize()
        x, info = px(vt, 0.6, ut, 1.5e-3, "iso", "nonneg", 25)
        torch.cuda.synchronize()
        if first is None:
            first = x.clone()
            assert _rel(x.cpu().numpy(), ref) < 1e-10
        else:
            assert torch.equal(x, first), rep
        del junk
    px.close()


# ---- metrics tau I + U U^T of rank r >= 2 -----------------------------------

def _inputs_rank(shape, r, seed):
    rng = np.random.default_rng(seed)
    v = 0.02 * rng.random(shape) + 0.005 * rng.standard_normal(shape)
    U = 0.1 * rng.standard_normal((r,) + shape)
    return v, U


@pytest.mark.parametrize("r,tv,cset", [(2, "iso", "nonneg"), (3, "aniso", "nonneg"), (5, "iso", "nonneg"),
                                       (8, "aniso", "nonneg"), (4, "iso", "none")])
def test_wprox_rank_r_f64_matches_oracle(dev, r, tv, cset):
    shape = (13, 17, 19)
    v, U = _inputs_rank(shape, r, 100 + r)
    ref = tp.wprox(v, 0.8, U, 2e-3, tv, cset, n_iter=30)
    got, info, _ = _run(dev, shape, "f64", v, 0.8, U, 2e-3, tv, cset, 30)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)
    if cset == "nonneg":
        assert np.all(got >= 0)
        assert info.newton_max <= 12 and info.newton_total >= 31


def test_wprox_rank_r_f32_matches_oracle(dev):
    shape = (20, 24, 28)
    v, U = _inputs_rank(shape, 3, 7)
    ref = tp.wprox(v, 1.0, U, 1e-3, "iso", "nonneg", n_iter=40)
    got, info, _ = _run(dev, shape, "f32", v, 1.0, U, 1e-3, "iso", "nonneg", 40)
    assert _rel(got, ref) < 2e-4, _rel(got, ref)


def test_wprox_rank_r_projection_zero_column_and_warm_start(dev):
    shape = (12, 14, 10)
    v, U = _inputs_rank(shape, 3, 11)
    # n_iter = 0: x = prox^B_C(v), Theorem 3.1 with a rank-3 factor
    got0, _, _ = _run(dev, shape, "f64", v, 0.5, U, 1e-3, "iso", "nonneg", 0)
    ref0, _ = tp.weighted_projection_nonneg(v, 0.5, U)
    assert _rel(got0, ref0) < 1e-12
    # a zero column: the rank-2 path equals the rank-one path
    U2 = np.stack([U[0], np.zeros(shape)])
    a, _, _ = _run(dev, shape, "f64", v, 0.5, U2, 1e-3, "iso", "nonneg", 20)
    b, _, _ = _run(dev, shape, "f64", v, 0.5, U[0], 1e-3, "iso", "nonneg", 20)
    assert _rel(a, b) < 1e-11
    # dual warm start
    x20, P20 = tp.wprox(v, 0.5, U, 1e-3, "iso", "nonneg", n_iter=20, return_dual=True)
    ref = tp.wprox(v, 0.5, U, 1e-3, "iso", "nonneg", n_iter=15, P0=P20)
    got20, _, Pg = _run(dev, shape, "f64", v, 0.5, U, 1e-3, "iso", "nonneg", 20, P=np.zeros((3,) + shape))
    assert _rel(got20, x20) < 1e-10 and _rel(Pg, P20) < 1e-10
    got, _, _ = _run(dev, shape, "f64", v, 0.5, U, 1e-3, "iso", "nonneg", 15, P=Pg)
    assert _rel(got, ref) < 1e-10


def test_wprox_rank_r_rejects_bad_rank_and_replays_stably(dev):
    from paper_2307_02043_amd import WProx
    from paper_2307_02043_amd import _lib as L
    shape = (10, 12, 14)
    v, U = _inputs_rank(shape, 4, 13)
    px = WProx(shape, "f64")
    vt = torch.from_numpy(v).to(dev)
    Ut = torch.from_numpy(U).to(dev)
    x = torch.empty_like(vt)
    lib = L.load()
    st = L.ProxStats()
    P = L.ct.c_void_p
    for r, Up in ((L.BQ_PROX_MAX_RANK + 1, Ut), (-1, Ut), (2, None)):
        s = lib.bq_wprox(px._h, P(vt.data_ptr()), 0.5, None if Up is None else P(Up.data_ptr()), r, 1e-3,
                         L.BQ_TV_ISO, L.BQ_SET_NONNEG, 5, P(x.data_ptr()), None, L.ct.byref(st))
        assert s == L.BQ_EINVAL, r
    ref = tp.wprox(v, 0.5, U, 1e-3, "iso", "nonneg", n_iter=25)
    first = None
    for rep in range(3):
        junk = torch.randn(1 << 20, device=dev).cumsum(0)
        torch.cuda.synchronize()
        y, _ = px(vt, 0.5, Ut, 1e-3, "iso", "nonneg", 25)
        torch.cuda.synchronize()
        if first is None:
            first = y.clone()
            assert _rel(y.cpu().numpy(), ref) < 1e-10
        else:
            assert torch.equal(y, first), rep
        del junk
    px.close()


def test_wprox_root_pass_budget_rerun(dev):
    """A call first launches two root passes per dual iteration; the cold start
    of this input needs four evaluations, so the call runs again with the full
    pass budget.  The result matches the oracle, a second call on the same
    object (which keeps the larger budget) gives the same bits, and a caller's
    starting dual point is restored before the rerun."""
    from paper_2307_02043_amd import WProx
    shape = (12, 14, 10)
    rng = np.random.default_rng(5)
    v = 0.02 * rng.standard_normal(shape) + 0.002 * rng.random(shape)
    u = 0.1 * rng.standard_normal(shape)
    ref, Pref = tp.wprox(v, 0.8, u, 1e-3, "iso", "nonneg", n_iter=20, return_dual=True)
    vt, ut = torch.from_numpy(v).to(dev), torch.from_numpy(u).to(dev)
    px = WProx(shape, "f64")
    x1, i1 = px(vt, 0.8, ut, 1e-3, "iso", "nonneg", 20)
    assert i1.newton_max >= 4, i1
    x2, i2 = px(vt, 0.8, ut, 1e-3, "iso", "nonneg", 20)
    assert torch.equal(x1, x2) and i2.newton_total == i1.newton_total
    assert _rel(x1.cpu().numpy(), ref) < 1e-10
    px.close()
    px = WProx(shape, "f64")
    P = torch.zeros((3,) + shape, dtype=torch.float64, device=dev)
    x3, _ = px(vt, 0.8, ut, 1e-3, "iso", "nonneg", 20, P=P)
    assert torch.equal(x3, x1)
    assert _rel(P.cpu().numpy(), Pref) < 1e-10
    px.close()


def test_wprox_rank_r_pass_budget_is_transparent(dev):
    """Rank 3: calls on a fresh object and on one that already raised its root
    pass budget agree bit for bit and match the oracle."""
    from paper_2307_02043_amd import WProx
    shape = (13, 17, 19)
    v, U = _inputs_rank(shape, 3, 21)
    ref = tp.wprox(v, 0.8, U, 2e-3, "aniso", "nonneg", n_iter=25)
    vt, Ut = torch.from_numpy(v).to(dev), torch.from_numpy(U).to(dev)
    px = WProx(shape, "f64")
    x1, i1 = px(vt, 0.8, Ut, 2e-3, "aniso", "nonneg", 25)
    x2, i2 = px(vt, 0.8, Ut, 2e-3, "aniso", "nonneg", 25)
    assert torch.equal(x1, x2) and i1.newton_total == i2.newton_total
    assert _rel(x1.cpu().numpy(), ref) < 1e-10
    px.close()


@pytest.mark.parametrize("shape", [(3, 5, 300), (2, 3, 256), (4, 6, 128), (2, 2, 2), (2, 3, 2)])
@pytest.mark.parametrize("r,tv", [(1, "iso"), (3, "aniso")])
def test_wprox_row_lengths(dev, shape, r, tv):
    """Rows longer than, equal to and half a workgroup (one row over several
    steps of the threads / one row per step / two rows per step), and the
    smallest images (every voxel on a face, 128 rows per step)."""
    if r == 1:
        v, U = _inputs(shape, 31)
    else:
        v, U = _inputs_rank(shape, r, 31)
    ref = tp.wprox(v, 0.7, U, 2e-3, tv, "nonneg", n_iter=20)
    got, info, _ = _run(dev, shape, "f64", v, 0.7, U, 2e-3, tv, "nonneg", 20)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)


@pytest.mark.parametrize("shape", [(101, 96, 130), (37, 97, 300)])
@pytest.mark.parametrize("r", [0, 1, 3])
def test_wprox_column_walk_ragged_chunks(dev, shape, r):
    """The dual kernels of every rank walk x columns through chunks of z
    planes (4 planes per thread at these sizes): a last chunk of one plane,
    rows shorter than a workgroup (130) and longer than one (300), FP64
    against the oracle."""
    rng = np.random.default_rng(200 + r + shape[2])
    v = 0.02 * rng.random(shape) + 0.005 * rng.standard_normal(shape)
    U = None if r == 0 else 0.1 * rng.standard_normal(((r,) if r > 1 else ()) + shape)
    ref = tp.wprox(v, 0.8, U, 2e-3, "iso", "nonneg", n_iter=12)
    got, _, _ = _run(dev, shape, "f64", v, 0.8, U, 2e-3, "iso", "nonneg", 12)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)


# ---- metric tau I (no u): one fused kernel per dual iteration ---------------

@pytest.mark.parametrize("n_iter", [0, 1, 2, 7, 20])
@pytest.mark.parametrize("shape", [(3, 5, 300), (2, 3, 256), (4, 6, 128), (2, 2, 2), (5, 7, 9)])
@pytest.mark.parametrize("tv,cset", [("iso", "nonneg"), ("aniso", "none")])
def test_wprox_tau_metric_iteration_counts_and_rows(dev, n_iter, shape, tv, cset):
    """Odd and even iteration counts (pairs of dual iterations replayed as one
    graph, an odd count ending with one launch alone, zero iterations giving
    x(P_0)) on rows longer than, equal to and shorter than a workgroup."""
    v, _ = _inputs(shape, 41 + n_iter)
    ref = tp.wprox(v, 0.9, None, 2e-3, tv, cset, n_iter=n_iter)
    got, info, _ = _run(dev, shape, "f64", v, 0.9, None, 2e-3, tv, cset, n_iter)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)
    assert info.newton_total == 0 and info.newton_max == 0 and info.status == 0
    if cset == "nonneg":
        assert np.all(got >= 0)


def test_wprox_tau_metric_warm_start_dual_point(dev):
    """The dual point left in P after K iterations is the oracle's P_K, and a
    call started from it continues the oracle's sequence."""
    shape = (9, 10, 11)
    v, _ = _inputs(shape, 57)
    x13, P13 = tp.wprox(v, 0.5, None, 1e-3, "iso", "nonneg", n_iter=13, return_dual=True)
    got13, _, Pg = _run(dev, shape, "f64", v, 0.5, None, 1e-3, "iso", "nonneg", 13, P=np.zeros((3,) + shape))
    assert _rel(got13, x13) < 1e-10
    assert _rel(Pg, P13) < 1e-10
    ref = tp.wprox(v, 0.5, None, 1e-3, "iso", "nonneg", n_iter=8, P0=P13)
    got, _, _ = _run(dev, shape, "f64", v, 0.5, None, 1e-3, "iso", "nonneg", 8, P=Pg)
    assert _rel(got, ref) < 1e-10, _rel(got, ref)


def test_wprox_tau_metric_f32_and_repeatable(dev):
    """FP32 at 64^3 within 2e-4 of the oracle; three calls on one object give
    the same bits (the second momentum buffer and both t slots are set up
    afresh by every call)."""
    shape = (64, 64, 64)
    v, _ = _inputs(shape, 63)
    ref = tp.wprox(v, 1.0, None, 1e-3, "iso", "nonneg", n_iter=25)
    from paper_2307_02043_amd import WProx
    px = WProx(shape, "f32")
    vt = torch.from_numpy(v).to(dev, torch.float32)
    outs = [px(vt, 1.0, None, 1e-3, "iso", "nonneg", 25)[0].clone() for _ in range(3)]
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    assert _rel(outs[0].cpu().numpy().astype(np.float64), ref) < 2e-4
    px.close()
