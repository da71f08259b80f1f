"""GPU parity of the Lippmann-Schwinger path against the CPU oracle.

All inputs are seeded synthetic data (see the synthetic package); every
expected value comes from the oracle.  Tolerances: 1e-10 relative (l2 over
the whole output) for FP64 and 2e-4 for FP32 on gradients; the Green's
operator alone is checked tighter (1e-12 FP64, 1e-5 FP32).  Solver parity
runs both sides to tol 1e-13 (FP64) so that the difference measures the
arithmetic, not where two correct iterations stop.
"""
import functools

import numpy as np
import pytest

import synthetic as syn
from oracle import green, lsmodel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = syn.LAMBDA0_UM / 4
KB = syn.N_B * 2 * np.pi / syn.LAMBDA0_UM


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@functools.lru_cache(maxsize=None)
def _ghat(N):
    return green.kernel_padded(N, H, KB)


@functools.lru_cache(maxsize=None)
def _model(N):
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B)
    return lsmodel.LSModel(geom, ghat_P=_ghat(N))


def _ctx(N, dirs, prec="f64", **kw):
    from paper_2307_02043_amd import LSContext
    return LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision=prec, **kw)


@pytest.mark.parametrize("N", [8, 12, 16, 24, 32, 48, 64])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_green_apply_matches_oracle(dev, N, prec):
    rng = np.random.default_rng(N)
    v = syn.random_field((2, N, N, N), rng)
    dirs = np.array([[0.0, 0.0, 1.0]])
    ctx = _ctx(N, dirs, prec)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    tol = 1e-12 if prec == "f64" else 1e-5
    vt = torch.from_numpy(v).to(dev, cd)
    for adj in (False, True):
        out = ctx.green(vt, adjoint=adj).cpu().numpy()
        ref = np.stack([(green.apply_GH if adj else green.apply_G)(_ghat(N), v[b]) for b in range(2)])
        assert _rel(out, ref) < tol, (N, prec, adj, _rel(out, ref))
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_green_apply_96_matches_oracle(dev, prec):
    """The radix-3 grid of the 96^3 workload, element by element, three
    systems: in complex64 the y pass is the padded register pass with
    24-point DFTs (192-point lines of 24 x 8), in complex128 the LDS
    Stockham pass; the other passes are the LDS Stockham ones in both."""
    N = 96
    rng = np.random.default_rng(960)
    v = syn.random_field((3, N, N, N), rng)
    ctx = _ctx(N, np.array([[0.0, 0.0, 1.0]]), prec)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    tol = 1e-12 if prec == "f64" else 1e-5
    vt = torch.from_numpy(v).to(dev, cd)
    for adj in (False, True):
        out = ctx.green(vt, adjoint=adj).cpu().numpy()
        for b in range(3):
            ref = (green.apply_GH if adj else green.apply_G)(_ghat(N), v[b])
            assert _rel(out[b], ref) < tol, (prec, adj, b, _rel(out[b], ref))
    ctx.close()


@pytest.mark.parametrize("N,prec", [(96, "f64"), (96, "f32"), (128, "f64"), (128, "f32")])
def test_green_apply_sampled_direct_sum(dev, N, prec):
    """Larger grids (128^3 is the benchmark grid, in its launch
    configuration): single outputs by direct summation with the oracle's
    discrete kernel."""
    rng = np.random.default_rng(100 + N)
    v = syn.random_field((2, N, N, N), rng)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    ctx = _ctx(N, np.array([[0.0, 0.0, 1.0]]), prec)
    out = ctx.green(torch.from_numpy(v).to(dev, cd)).cpu().numpy()[1]
    K = green.kernel_lags(_ghat(N))
    pts = [tuple(int(t) for t in rng.integers(0, N, 3)) for _ in range(6)] + [(0, 0, 0), (N - 1, N - 1, N - 1)]
    ref = green.apply_G_direct(K, v[1], pts)
    got = np.array([out[p] for p in pts])
    assert _rel(got, ref) < (1e-11 if prec == "f64" else 1e-5)
    ctx.close()


@functools.lru_cache(maxsize=None)
def _lags(N):
    return green.kernel_lags_direct(N, H, KB, workers=16)


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_green_apply_sampled_direct_sum_256(dev, prec):
    """256^3 (the parity-split register passes): single outputs by direct
    summation with the oracle's discrete kernel (its lags taken without the
    DFT round trip)."""
    N = 256
    rng = np.random.default_rng(256)
    v = syn.random_field((1, N, N, N), rng)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    ctx = _ctx(N, np.array([[0.0, 0.0, 1.0]]), prec)
    out = ctx.green(torch.from_numpy(v).to(dev, cd)).cpu().numpy()[0]
    ctx.close()
    pts = [tuple(int(t) for t in rng.integers(0, N, 3)) for _ in range(4)] + [(0, 0, 0), (N - 1, N - 1, N - 1)]
    ref = green.apply_G_direct(_lags(N), v[0], pts)
    got = np.array([out[p] for p in pts])
    assert _rel(got, ref) < (1e-11 if prec == "f64" else 1e-5), _rel(got, ref)


@pytest.mark.parametrize("N,prec", [(16, "f64"), (32, "f32"), (64, "f64"), (64, "f32"), (128, "f32")])
def test_fused_plane_pass_equals_split_passes(dev, N, prec):
    """The LDS-resident x/y pass and the three-pass path compute the same G
    (consistency between two GPU paths; each is also checked vs the oracle)."""
    rng = np.random.default_rng(7 * N)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    v = torch.from_numpy(syn.random_field((3, N, N, N), rng)).to(dev, cd)
    d = np.array([[0.0, 0.0, 1.0]])
    a = _ctx(N, d, prec, fused_xy=True).green(v)
    b = _ctx(N, d, prec).green(v)
    err = float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    assert err < (1e-13 if prec == "f64" else 3e-6), err


def _c1_like(N, L, seed):
    rng = np.random.default_rng(seed)
    dn = syn.phantom_ellipsoids(N, H, rng)
    xt = syn.scattering_potential(dn)
    dirs = syn.illumination_directions(L, 35.0, np.random.default_rng(seed + 1))
    return xt, dirs


@pytest.mark.parametrize("N", [16, 24])
def test_forward_and_fields_match_oracle(dev, N):
    xt, dirs = _c1_like(N, 3, 7 + N)
    idx = [2, 0]
    m = _model(N)
    yref, _ = m.forward(xt, dirs, idx, 1e-13, 400)
    ctx = _ctx(N, dirs, "f64", tol=1e-13, max_iter=400)
    x = torch.from_numpy(xt).to(dev)
    y, info = ctx.forward(x, idx)
    assert info.status == 0 and all(s == 0 for s in info.status_fwd)
    assert _rel(y.cpu().numpy(), yref) < 1e-10
    u, _ = ctx.fields(x, idx)
    uref = m.solve_forward(xt, lsmodel.incident_field(m.geom, dirs[2]), 1e-13, 400)[0]
    assert _rel(u[0].cpu().numpy(), uref) < 1e-10
    ctx.close()


@functools.lru_cache(maxsize=None)
def _c1_reference():
    w = syn.WORKLOADS["c1_ls32_f64"]
    N = w.N
    xt = syn.scattering_potential(syn.make_phantom(w))
    dirs = syn.workload_directions(w)
    idx = syn.batch_indices(w)
    m = _model(N)
    yc, _ = m.forward(xt, dirs, idx, 1e-13, 400)
    y = syn.add_noise(yc, w.snr_db, np.random.default_rng(w.seed("noise")))
    x = 0.5 * xt
    g, f, st = m.grad(x, y, dirs, idx, 1.0 / len(idx), 1e-13, 400)
    return x, y, dirs, idx, g, f


@pytest.mark.parametrize("plain", [False, True])
def test_grad_c1_f64_matches_oracle(dev, plain):
    x, y, dirs, idx, gref, fref = _c1_reference()
    ctx = _ctx(x.shape[0], dirs, "f64", tol=1e-13, max_iter=400, plain=plain)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), idx, 1.0 / len(idx))
    assert info.status == 0
    assert _rel(g.cpu().numpy(), gref) < 1e-10
    assert abs(f - fref) / fref < 1e-10
    ctx.close()


def test_grad_c1_f32_matches_oracle(dev):
    x, y, dirs, idx, gref, fref = _c1_reference()
    ctx = _ctx(x.shape[0], dirs, "f32", tol=1e-6, max_iter=400)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev, torch.float32),
                          torch.from_numpy(y).to(dev, torch.complex64), idx, 1.0 / len(idx))
    assert info.status == 0
    err = _rel(g.cpu().numpy(), gref)
    assert err < 2e-4, err
    assert abs(f - fref) / fref < 2e-4
    ctx.close()


def test_batched_equals_plain_f64(dev):
    x, y, dirs, idx, _, _ = _c1_reference()
    out = []
    for plain in (False, True):
        ctx = _ctx(x.shape[0], dirs, "f64", tol=1e-13, max_iter=400, plain=plain)
        g, f, info = ctx.grad(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), idx, 0.25)
        out.append((g.cpu().numpy(), f, info.iters_fwd, info.iters_adj))
        ctx.close()
    assert out[0][2] == out[1][2] and out[0][3] == out[1][3]
    assert _rel(out[0][0], out[1][0]) < 1e-13


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32", 2e-4)])
def test_born_grad_matches_oracle(dev, prec, tol):
    N = 24
    xt, dirs = _c1_like(N, 5, 31)
    idx = [4, 1, 3]
    m = _model(N)
    yc, _ = m.forward(xt, dirs, idx, 0, 0, model="born")
    y = syn.add_noise(yc, 30.0, np.random.default_rng(5))
    x = 0.5 * xt
    gref, fref, _ = m.grad(x, y, dirs, idx, 1 / 3, 0, 0, model="born")
    ctx = _ctx(N, dirs, prec, model="born")
    rd = torch.float64 if prec == "f64" else torch.float32
    cd = torch.complex128 if prec == "f64" else torch.complex64
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd), idx, 1 / 3)
    assert _rel(g.cpu().numpy(), gref) < tol
    assert abs(f - fref) / fref < tol
    yb, _ = ctx.forward(torch.from_numpy(xt).to(dev, rd), idx)
    assert _rel(yb.cpu().numpy(), yc) < tol
    ctx.close()


def test_status_and_errors(dev):
    from paper_2307_02043_amd import BQError
    x, y, dirs, idx, _, _ = _c1_reference()
    ctx = _ctx(x.shape[0], dirs, "f64", tol=1e-13, max_iter=1)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), idx, 0.25)
    assert info.status == 1 and all(s == 1 for s in info.status_fwd)
    assert all(i == 1 for i in info.iters_fwd)
    with pytest.raises(BQError):
        ctx.grad(torch.from_numpy(x).to(dev), torch.from_numpy(y[:2]).to(dev), [0, 9], 0.5)
    # x = 0: LS reduces to Born, no iterations
    z = torch.zeros_like(torch.from_numpy(x)).to(dev)
    g0, _, info0 = ctx.grad(z, torch.from_numpy(y).to(dev), idx, 0.25)
    assert info0.status == 0 and all(i == 0 for i in info0.iters_fwd + info0.iters_adj)
    ctx.close()


def test_pass_timing_mask(dev):
    """bq_timing times exactly the passes of its mask; out-of-range masks fail."""
    from paper_2307_02043_amd import _lib as L
    lib = L.load()
    N = 32
    ctx = _ctx(N, np.array([[0.0, 0.0, 1.0]]), "f32")
    v = torch.randn(2, N, N, N, dtype=torch.complex64, device=dev)
    yc = L.PASS_NAMES.index("yc")
    assert lib.bq_timing(ctx._h, 1 << yc) == 0
    ctx.green(v)
    ctx.green(v)
    assert lib.bq_timing(ctx._h, 0) == 0
    for pid, name in enumerate(L.PASS_NAMES):
        ms, n = L.ct.c_double(), L.ct.c_longlong()
        assert lib.bq_timing_get(ctx._h, pid, L.ct.byref(ms), L.ct.byref(n)) == 0
        if name == "yc":
            assert n.value == 2 and ms.value > 0
        else:
            assert n.value == 0
    assert lib.bq_timing(ctx._h, L.BQ_TIMING_ALL + 1) == L.BQ_EINVAL
    assert lib.bq_timing(ctx._h, -1) == L.BQ_EINVAL
    ctx.close()


@pytest.mark.parametrize("prec,plain", [("f64", False), ("f64", True), ("f32", False)])
def test_warm_started_grad_matches_oracle(dev, prec, plain):
    """bq_grad_ws: the fields of a gradient at x start the solves of the
    gradient at a nearby x1; gradient, loss and fields match the oracle's
    warm-started computation, with fewer iterations than a cold start."""
    x, y, dirs, idx, _, _ = _c1_reference()
    N = x.shape[0]
    m = _model(N)
    x1 = 1.02 * x
    _, _, _, fields = m.grad(x, y, dirs, idx, 0.25, 1e-13, 400, return_fields=True)
    gref, fref, stref, fref1 = m.grad(x1, y, dirs, idx, 0.25, 1e-13, 400, starts=fields, return_fields=True)
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    ctx = _ctx(N, dirs, prec, tol=tol, max_iter=400, plain=plain)
    B = len(idx)
    u = torch.zeros((B, N, N, N), dtype=cd, device=dev)
    w = torch.zeros_like(u)
    yt = torch.from_numpy(y).to(dev, cd)
    ctx.grad_ws(torch.from_numpy(x).to(dev, rd), yt, idx, 0.25, u, w, start=False)
    gc, fc, ic = ctx.grad(torch.from_numpy(x1).to(dev, rd), yt, idx, 0.25)
    g, f, info = ctx.grad_ws(torch.from_numpy(x1).to(dev, rd), yt, idx, 0.25, u, w, start=True)
    assert info.status == 0
    lim = 1e-10 if prec == "f64" else 2e-4
    assert _rel(g.cpu().numpy(), gref) < lim
    assert abs(f - fref) / fref < lim
    for b in range(B):
        assert _rel(u[b].cpu().numpy(), fref1[b][0]) < lim
        # the library keeps the conjugated adjoint field (it solves the conjugate system)
        assert _rel(w[b].cpu().numpy(), np.conj(fref1[b][1])) < lim
    assert sum(info.iters_fwd) + sum(info.iters_adj) < sum(ic.iters_fwd) + sum(ic.iters_adj)
    if prec == "f64":
        assert list(info.iters_fwd) == [s[0] for s in stref]
        assert list(info.iters_adj) == [s[1] for s in stref]
    ctx.close()


@pytest.mark.parametrize("N,prec,model", [(24, "f64", "ls"), (32, "f64", "ls"), (32, "f32", "ls"),
                                          (24, "f64", "born")])
def test_propagated_detector_matches_oracle(dev, N, prec, model):
    """Detector plane 1.3 um beyond the exit plane (angular-spectrum
    propagation): forward images, loss and gradient vs the oracle."""
    d = 1.3
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B, det_dist=d)
    m = lsmodel.LSModel(geom, ghat_P=_ghat(N))
    xt, dirs = _c1_like(N, 3, 50 + N)
    idx = [2, 0]
    yc, _ = m.forward(xt, dirs, idx, 1e-13, 400, model=model)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(9))
    x = 0.5 * xt
    gref, fref, _ = m.grad(x, y, dirs, idx, 0.5, 1e-13, 400, model=model)
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    lim = 1e-10 if prec == "f64" else 2e-4
    ctx = _ctx(N, dirs, prec, tol=tol, max_iter=400, model=model, det_dist_um=d)
    yg, _ = ctx.forward(torch.from_numpy(xt).to(dev, rd), idx)
    assert _rel(yg.cpu().numpy(), yc) < lim
    yt = torch.from_numpy(y).to(dev, cd)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev, rd), yt, idx, 0.5)
    assert info.status == 0
    assert _rel(g.cpu().numpy(), gref) < lim
    assert abs(f - fref) / fref < lim
    fl, _ = ctx.loss(torch.from_numpy(x).to(dev, rd), yt, idx, 0.5)
    assert abs(fl - fref) / fref < lim
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replayed_iterations_equal_kernel_by_kernel_launches(dev, prec):
    """With BQ_FLAG_GRAPH, batched solves replay one captured BiCGSTAB
    iteration as a HIP graph.  Repeated calls, with eager torch work and synchronisations between them,
    a batch-size change (new graph, same buffers) and warm-started solves
    into caller-owned fields give exactly the results of the path that
    launches every kernel itself."""
    x, y, dirs, idx, _, _ = _c1_reference()
    N = x.shape[0]
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    eager = _ctx(N, dirs, prec, tol=tol, max_iter=400)
    graph = _ctx(N, dirs, prec, tol=tol, max_iter=400, graphs=True)
    xt = torch.from_numpy(x).to(dev, rd)
    yt = torch.from_numpy(y).to(dev, cd)
    B = len(idx)
    ref = {}
    for nb in (B, 2):
        ref[nb] = eager.grad(xt, yt[:nb], idx[:nb], 0.25)
    for rep, nb in enumerate((B, B, 2, B, 2)):
        g, f, info = graph.grad(xt, yt[:nb], idx[:nb], 0.25)
        ge, fe, ie = ref[nb]
        assert torch.equal(g, ge), (rep, nb)
        assert f == fe and list(info.iters_fwd) == list(ie.iters_fwd), (rep, nb)
        assert list(info.iters_adj) == list(ie.iters_adj), (rep, nb)
        float((xt * 2.0).sum())  # eager work and a synchronisation between replays
    for ctx in (eager, graph):
        ctx.u = torch.zeros((B, N, N, N), dtype=cd, device=dev)
        ctx.w = torch.zeros_like(ctx.u)
        ctx.grad_ws(xt, yt, idx, 0.25, ctx.u, ctx.w, start=False)
    ge, fe, _ = eager.grad_ws(1.02 * xt, yt, idx, 0.25, eager.u, eager.w, start=True)
    g, f, _ = graph.grad_ws(1.02 * xt, yt, idx, 0.25, graph.u, graph.w, start=True)
    assert torch.equal(g, ge) and f == fe
    assert torch.equal(graph.u, eager.u) and torch.equal(graph.w, eager.w)
    eager.close()
    graph.close()


@pytest.mark.parametrize("case", ["c1_f64", "c1_f32", "c4_f32"])
def test_launch_shapes_change_no_value(dev, case):
    """Every launch shape the autotuner may choose (x-pass tile rows, width
    of the z-forward pass) gives the same gradient bit for bit; the tuner
    returns one of them; shapes not available are rejected."""
    from paper_2307_02043_amd import BQError
    if case.startswith("c1"):
        x, y, dirs, idx, _, _ = _c1_reference()
        prec = case[3:]
        N = x.shape[0]
        ctx = _ctx(N, dirs, prec, tol=1e-13 if prec == "f64" else 1e-6, max_iter=400)
    else:
        w = syn.WORKLOADS["c4_ls128_f32"]
        prec, N = "f32", w.N
        dirs = syn.workload_directions(w)
        idx = syn.batch_indices(w)[:4]
        x = 0.5 * syn.scattering_potential(syn.make_phantom(w))
        ctx = _ctx(N, dirs, prec, tol=w.tol, max_iter=w.max_iter)
        y = ctx.forward(torch.from_numpy(2 * x).to(dev, torch.float32), idx)[0].cpu().numpy()
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    xt, yt = torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd)
    g0, f0, i0 = ctx.grad(xt, yt, idx, 0.25)
    tried = 0
    for xr in (0, 8, 16, 32):
        for zt in (0, 256, 1024):
            try:
                ctx.set_plan(xr, zt)
            except BQError:
                continue
            g, f, info = ctx.grad(xt, yt, idx, 0.25)
            assert torch.equal(g, g0) and f == f0, (xr, zt)
            assert list(info.iters_fwd) == list(i0.iters_fwd), (xr, zt)
            tried += 1
    assert tried >= 3
    with pytest.raises(BQError):
        ctx.set_plan(5, 0)
    with pytest.raises(BQError):
        ctx.set_plan(0, 512)
    r = ctx.autotune(len(idx))
    assert r["ms_tuned"] <= r["ms_default"] and r["ms_default"] > 0
    g, f, _ = ctx.grad(xt, yt, idx, 0.25)
    assert torch.equal(g, g0) and f == f0
    ctx.close()


@pytest.mark.parametrize("prec,model", [("f64", "ls"), ("f32", "ls"), ("f64", "born")])
def test_sub_batches_equal_one_launch_set(dev, prec, model):
    """A batch run as consecutive sub-batches (a limit of 2 and of 3 systems
    per launch set for 4 systems) gives the same per-system fields, images
    and iteration counts bit for bit, and the same gradient and loss up to
    the order of the additions."""
    x, y, dirs, idx, _, _ = _c1_reference()
    N = x.shape[0]
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    ctx = _ctx(N, dirs, prec, tol=tol, max_iter=400, model=model)
    xt, yt = torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd)
    g0, f0, i0 = ctx.grad(xt, yt, idx, 0.25)
    h0, _ = ctx.forward(xt, idx)
    u0, _ = ctx.fields(xt, idx)
    l0, _ = ctx.loss(xt, yt, idx, 0.25)
    lim = 1e-13 if prec == "f64" else 1e-6
    for m in (2, 3):
        ctx.set_batch_limit(m)
        g, f, info = ctx.grad(xt, yt, idx, 0.25)
        assert float(torch.linalg.norm(g - g0) / torch.linalg.norm(g0)) < lim, m
        assert abs(f - f0) <= lim * abs(f0), m
        assert list(info.iters_fwd) == list(i0.iters_fwd) and list(info.iters_adj) == list(i0.iters_adj)
        h, _ = ctx.forward(xt, idx)
        u, _ = ctx.fields(xt, idx)
        assert torch.equal(h, h0) and torch.equal(u, u0), m
        l, _ = ctx.loss(xt, yt, idx, 0.25)
        assert abs(l - l0) <= lim * abs(l0), m
    ctx.set_batch_limit(0)
    from paper_2307_02043_amd import BQError
    with pytest.raises(BQError):
        ctx.set_batch_limit(-1)
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graphs_follow_the_launch_plan(dev, prec):
    """Replayed iteration graphs are keyed on the launch shapes: after
    bq_set_plan the next solve captures its graphs again (a cached graph of
    the old shapes is not replayed), going back to cached shapes captures
    nothing, bq_autotune drops the graphs, and the gradient stays the same
    bit for bit throughout."""
    from paper_2307_02043_amd import BQError
    x, y, dirs, idx, _, _ = _c1_reference()
    N = x.shape[0]
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    ctx = _ctx(N, dirs, prec, tol=1e-13 if prec == "f64" else 1e-6, max_iter=400, graphs=True)
    xt, yt = torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd)
    g0, f0, _ = ctx.grad(xt, yt, idx, 0.25)
    n0 = ctx.info()["graph_captures"]
    assert n0 >= 1
    g, f, _ = ctx.grad(xt, yt, idx, 0.25)
    assert torch.equal(g, g0) and ctx.info()["graph_captures"] == n0
    other = None
    for xr, zt in ((8, 0), (16, 0), (32, 0), (0, 256), (0, 1024)):
        try:
            ctx.set_plan(xr, zt)
        except BQError:
            continue
        other = (xr, zt)
        break
    assert other is not None
    g, f, _ = ctx.grad(xt, yt, idx, 0.25)
    info = ctx.info()
    assert (info["x_tile_rows"], info["zf_threads"]) == other
    assert info["graph_captures"] == 2 * n0
    assert torch.equal(g, g0) and f == f0
    ctx.set_plan(0, 0)
    g, f, _ = ctx.grad(xt, yt, idx, 0.25)
    assert ctx.info()["graph_captures"] == 2 * n0 and torch.equal(g, g0)
    ctx.autotune(len(idx))
    assert ctx.info()["graphs_cached"] == 0
    g, f, _ = ctx.grad(xt, yt, idx, 0.25)
    assert torch.equal(g, g0) and f == f0
    ctx.close()
