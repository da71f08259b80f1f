"""GPU parity of the camera sampling of the detector plane against the
oracle (oracle/camera.py): forward images, loss and gradient with an M x M
camera of its own pitch, at the exit plane and after angular-spectrum
propagation, LS and first-Born models, FP64 (1e-10) and FP32 (2e-4); a
camera on the window's own grid gives the images of the window; the outer
iteration runs on camera measurements."""
import functools

import numpy as np
import pytest

import synthetic as syn
from oracle import bqnpm, camera, green, lsmodel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = syn.LAMBDA0_UM / 4
KB = syn.N_B * 2 * np.pi / syn.LAMBDA0_UM


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@functools.lru_cache(maxsize=None)
def _ghat(N):
    return green.kernel_padded(N, H, KB)


def _ctx(N, dirs, prec, **kw):
    from paper_2307_02043_amd import LSContext
    return LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision=prec, **kw)


def _problem(N, L, seed):
    rng = np.random.default_rng(seed)
    xt = syn.scattering_potential(syn.phantom_ellipsoids(N, H, rng))
    dirs = syn.illumination_directions(L, 35.0, np.random.default_rng(seed + 1))
    return xt, dirs


# (N, M, pitch): finer and wider than the window (the paper's 512^2 camera
# over a few micrometres), coarser and narrower, and an odd pixel count
CAMS = [(24, 60, 0.05), (24, 15, 0.13), (32, 37, 0.07)]


@pytest.mark.parametrize("N,M,pitch", CAMS)
@pytest.mark.parametrize("d", [0.0, 1.3])
@pytest.mark.parametrize("prec,model", [("f64", "ls"), ("f32", "ls"), ("f64", "born")])
def test_camera_matches_oracle(dev, N, M, pitch, d, prec, model):
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B, det_dist=d)
    m = camera.CameraLSModel(geom, M, pitch, ghat_P=_ghat(N))
    xt, dirs = _problem(N, 3, 40 + N + M)
    idx = [2, 0]
    yc, _ = m.forward(xt, dirs, idx, 1e-13, 400, model=model)
    assert yc.shape == (2, M, M)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(3))
    x = 0.5 * xt
    gref, fref, _ = m.grad(x, y, dirs, idx, 0.5, 1e-13, 400, model=model)
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    tol = 1e-13 if prec == "f64" else 1e-6
    lim = 1e-10 if prec == "f64" else 2e-4
    ctx = _ctx(N, dirs, prec, tol=tol, max_iter=400, model=model, det_dist_um=d, cam_n=M, cam_pitch_um=pitch)
    yg, _ = ctx.forward(torch.from_numpy(xt).to(dev, rd), idx)
    assert tuple(yg.shape) == (2, M, M)
    assert _rel(yg.cpu().numpy(), yc) < lim
    yt = torch.from_numpy(y).to(dev, cd)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev, rd), yt, idx, 0.5)
    assert info.status == 0
    assert _rel(g.cpu().numpy(), gref) < lim, _rel(g.cpu().numpy(), gref)
    assert abs(f - fref) < lim * fref
    fl, _ = ctx.loss(torch.from_numpy(x).to(dev, rd), yt, idx, 0.5)
    assert abs(fl - fref) < lim * fref
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_camera_on_the_window_grid_is_the_window(dev, prec):
    N = 24
    xt, dirs = _problem(N, 2, 9)
    rd = torch.float64 if prec == "f64" else torch.float32
    x = torch.from_numpy(xt).to(dev, rd)
    plain = _ctx(N, dirs, prec, tol=1e-13, max_iter=400)
    cam = _ctx(N, dirs, prec, tol=1e-13, max_iter=400, cam_n=N, cam_pitch_um=H)
    a, _ = plain.forward(x, [0, 1])
    b, _ = cam.forward(x, [0, 1])
    err = float(torch.linalg.norm(a - b) / torch.linalg.norm(a))
    assert err < (1e-13 if prec == "f64" else 1e-6), err
    plain.close()
    cam.close()


def test_camera_arguments_are_checked(dev):
    from paper_2307_02043_amd import BQError
    _, dirs = _problem(16, 1, 1)
    for n, p in ((-1, 0.1), (5000, 0.1), (8, 0.0), (8, float("nan"))):
        with pytest.raises(BQError):
            _ctx(16, dirs, "f64", cam_n=n, cam_pitch_um=p)
    ctx = _ctx(16, dirs, "f64", cam_n=20, cam_pitch_um=0.08)
    with pytest.raises(ValueError):  # measurements of the window's size
        ctx.grad(torch.zeros((16, 16, 16), dtype=torch.float64, device=dev),
                 torch.zeros((1, 16, 16), dtype=torch.complex128, device=dev), [0], 1.0)
    ctx.close()


def test_outer_iteration_on_camera_measurements(dev):
    """Three outer iterations (Algorithm 4.1) with camera measurements
    (L x M x M), against the oracle's, FP64."""
    from paper_2307_02043_amd import LSContext, QNIteration, WProx
    N, M, pitch, L, S = 16, 30, 0.06, 4, 2
    subsets = [[0, 1], [2, 3]]
    xt, dirs = _problem(N, L, 77)
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B)
    m = camera.CameraLSModel(geom, M, pitch, ghat_P=_ghat(N))
    y, _ = m.forward(xt, dirs, list(range(L)), 1e-13, 400)
    g0 = m.grad(np.zeros_like(xt), y[subsets[0]], dirs, subsets[0], S / L, 1e-13, 400)[0]
    alpha = float(np.abs(g0).max() / xt.max())
    prm = bqnpm.BQNPMParams(S=S, a=0.5, lam=1e-5, alpha=alpha, prox_iters=20)
    it = bqnpm.BQNPM(prm, lambda s, x: m.grad(x, y[subsets[s]], dirs, subsets[s], S / L, 1e-13, 400)[0])
    ls = LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision="f64", tol=1e-13, max_iter=400, cam_n=M,
                   cam_pitch_um=pitch)
    px = WProx((N, N, N), "f64")
    qn = QNIteration(ls, px, subsets, prm.a, prm.lam, alpha, prox_iters=20)
    xg = torch.zeros((N, N, N), dtype=torch.float64, device=dev)
    yt = torch.from_numpy(y).to(dev)
    xr = np.zeros_like(xt)
    for k in range(3):
        xr, _, _ = it.step(xr)
        qn.step(xg, yt)
        assert _rel(xg.cpu().numpy(), xr) < 1e-9, k
    qn.close()
    px.close()
    ls.close()
