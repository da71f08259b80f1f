"""Status paths of the Lippmann-Schwinger calls on the GPU, each reached by
a constructed input and checked against the oracle where the oracle defines
the result:

* BQ_NOTCONV: an iteration cap below what the tolerance needs; the
  gradient then equals the oracle's with the same cap;
* BQ_BREAKDOWN: a breakdown floor on |rho|, |<rhat, A p>|, |omega| (BiCGSTAB,
  van der Vorst 1992) that the scalars cross after a few iterations; the
  iteration counts, fields and gradient equal the oracle's with the same
  floor; a floor above every scalar stops before the first iteration;
* BQ_NONFINITE: a NaN in the potential (every forward solve) or in one
  measurement (that system's adjoint solve only);
* x = 0: the Lippmann-Schwinger gradient takes no iteration and equals the
  oracle's first-Born gradient;
* BQ_EINVAL / BQ_EUNSUPPORTED / BQ_ENOMEM from argument and size checks.

No input here makes a kernel read or write out of bounds: the non-finite
values are ordinary floating-point data, and the breakdown floor is a host
setting read by the scalar steps.
"""
import functools

import numpy as np
import pytest

import synthetic as syn
from oracle import lsmodel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

H = syn.LAMBDA0_UM / 4


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _ctx(N, dirs, prec="f64", **kw):
    from paper_2307_02043_amd import LSContext
    return LSContext(N, H, syn.LAMBDA0_UM, syn.N_B, dirs, precision=prec, **kw)


@functools.lru_cache(maxsize=None)
def _case(N=16):
    rng = np.random.default_rng(1000 + N)
    xt = syn.scattering_potential(syn.phantom_ellipsoids(N, H, rng))
    dirs = syn.illumination_directions(3, 35.0, np.random.default_rng(2000 + N))
    geom = lsmodel.Geometry(N=N, h=H, lambda0=syn.LAMBDA0_UM, n_b=syn.N_B)
    m = lsmodel.LSModel(geom)
    idx = [0, 2, 1]
    yc, _ = m.forward(xt, dirs, idx, 1e-13, 300)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(3000 + N))
    return m, 0.5 * xt, y, dirs, idx


def _oracle_grad(m, x, y, dirs, idx, scale, tol, max_iter, breakdown=1e-300, model="ls"):
    """The oracle's gradient with a given iteration cap and breakdown floor
    (its grad() runs the default floor)."""
    g = np.zeros(x.shape)
    loss = 0.0
    st = []
    for b, l in enumerate(idx):
        uin = lsmodel.incident_field(m.geom, dirs[l])
        u, itf, sf, _ = m.solve_forward(x, uin, tol, max_iter, breakdown=breakdown)
        r = m.detector(u - uin) - y[b]
        loss += 0.5 * np.vdot(r, r).real
        w, ita, sa, _ = m.solve_adjoint(x, m.GH(m.detector_T(r)), tol, max_iter, breakdown=breakdown)
        g += np.real(np.conj(u) * w)
        st.append((itf, ita, sf, sa))
    return scale * g, scale * loss, st


def test_iteration_cap_gives_notconv_and_the_capped_oracle_gradient(dev):
    m, x, y, dirs, idx = _case()
    ctx = _ctx(16, dirs, "f64", tol=1e-13, max_iter=2)
    g, f, info = ctx.grad(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), idx, 1 / 3)
    assert info.status == 1  # BQ_NOTCONV
    assert info.status_fwd == [1, 1, 1] and info.iters_fwd == [2, 2, 2]
    gref, fref, st = _oracle_grad(m, x, y, dirs, idx, 1 / 3, 1e-13, 2)
    assert [s[2] for s in st] == [lsmodel.NOT_CONVERGED] * 3
    assert _rel(g.cpu().numpy(), gref) < 1e-10 and abs(f - fref) < 1e-10 * fref
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_breakdown_floor_matches_oracle(dev, prec):
    m, x, y, dirs, idx = _case()
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    ctx = _ctx(16, dirs, prec, tol=1e-13, max_iter=300)
    xt, yt = torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd)
    # a floor above every scalar: no iteration, the fields are the starts
    ctx.set_breakdown_floor(1e300)
    assert ctx.info()["breakdown_floor"] == 1e300
    u, info = ctx.fields(xt, idx)
    assert info.status == 2 and info.status_fwd == [2, 2, 2] and info.iters_fwd == [0, 0, 0]
    for b, l in enumerate(idx):
        err = _rel(u[b].cpu().numpy(), lsmodel.incident_field(m.geom, dirs[l]))
        assert err < (1e-13 if prec == "f64" else 1e-6), err
    # |rho| of the forward solves falls from about 15 by a factor of hundreds
    # per iteration, that of the adjoint solves from about 4e-6: 1e-4 stops the
    # forward solves after two iterations and the adjoint ones at the start,
    # 1e-9 (FP64 only: FP32 residuals stall above it) after four and two
    floors = (1e-4, 1e-9) if prec == "f64" else (1e-4,)
    for floor in floors:
        ctx.set_breakdown_floor(floor)
        g, f, info = ctx.grad(xt, yt, idx, 1 / 3)
        gref, fref, st = _oracle_grad(m, x, y, dirs, idx, 1 / 3, 1e-13, 300, breakdown=floor)
        assert [s[2] for s in st] == [lsmodel.BREAKDOWN] * 3
        assert info.status == 2 and info.status_fwd == [2, 2, 2]
        assert info.iters_fwd == [s[0] for s in st]
        assert info.iters_adj == [s[1] for s in st]
        assert info.status_adj == [s[3] for s in st]
        lim = 1e-10 if prec == "f64" else 2e-4
        assert _rel(g.cpu().numpy(), gref) < lim and abs(f - fref) < lim * fref
    ctx.set_breakdown_floor(1e-300)
    g2, f2, info2 = ctx.grad(xt, yt, idx, 1 / 3)
    assert info2.status == 0
    from paper_2307_02043_amd import BQError
    with pytest.raises(BQError):
        ctx.set_breakdown_floor(-1.0)
    with pytest.raises(BQError):
        ctx.set_breakdown_floor(float("inf"))
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nonfinite_inputs_are_reported_per_system(dev, prec):
    m, x, y, dirs, idx = _case()
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    ctx = _ctx(16, dirs, prec, tol=1e-13 if prec == "f64" else 1e-6, max_iter=300)
    xt, yt = torch.from_numpy(x).to(dev, rd), torch.from_numpy(y).to(dev, cd)
    xn = xt.clone()
    xn[3, 7, 11] = float("nan")
    g, f, info = ctx.grad(xn, yt, idx, 1 / 3)
    assert info.status == 3  # BQ_NONFINITE
    # the first residual G(x u_in) is NaN everywhere: every forward and
    # adjoint solve stops before its first iteration
    assert info.status_fwd == [3, 3, 3] and info.status_adj == [3, 3, 3]
    assert info.iters_fwd == [0, 0, 0]
    # NaN in one measurement: the forward solves converge, only that
    # system's adjoint solve meets it
    yn = yt.clone()
    yn[1, 5, 5] = complex(float("nan"), 0.0)
    g, f, info = ctx.grad(xt, yn, idx, 1 / 3)
    assert info.status == 3
    assert info.status_fwd == [0, 0, 0]
    assert info.status_adj[1] == 3 and info.status_adj[0] == 0 and info.status_adj[2] == 0
    # the context stays usable and exact afterwards
    g, f, info = ctx.grad(xt, yt, idx, 1 / 3)
    gref, fref, _ = m.grad(x, y, dirs, idx, 1 / 3, 1e-13, 300)
    assert info.status == 0
    assert _rel(g.cpu().numpy(), gref) < (1e-10 if prec == "f64" else 2e-4)
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gradient_at_zero_is_the_oracle_born_gradient(dev, prec):
    """At x = 0 the total field is the incident wave: no iteration runs and
    the Lippmann-Schwinger gradient is the first-Born one."""
    m, x, y, dirs, idx = _case()
    rd, cd = (torch.float64, torch.complex128) if prec == "f64" else (torch.float32, torch.complex64)
    ctx = _ctx(16, dirs, prec, tol=1e-13, max_iter=300)
    z = torch.zeros((16, 16, 16), dtype=rd, device=dev)
    g, f, info = ctx.grad(z, torch.from_numpy(y).to(dev, cd), idx, 1 / 3)
    assert info.status == 0 and info.iters_fwd == [0, 0, 0] and info.iters_adj == [0, 0, 0]
    gref, fref, _ = m.grad(np.zeros_like(x), y, dirs, idx, 1 / 3, 0, 0, model="born")
    lim = 1e-10 if prec == "f64" else 2e-4
    assert _rel(g.cpu().numpy(), gref) < lim and abs(f - fref) < lim * fref
    ctx.close()


def test_error_statuses(dev):
    from paper_2307_02043_amd import BQError, WProx
    from paper_2307_02043_amd import _lib as L
    m, x, y, dirs, idx = _case()
    ctx = _ctx(16, dirs, "f64")
    xt, yt = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    with pytest.raises(BQError) as e:
        ctx.grad(xt, yt[:2], [0, 3], 0.5)  # index out of range
    assert e.value.status == L.BQ_EINVAL
    lib = L.load()
    loss = L.ct.c_double()
    assert lib.bq_grad(ctx._h, None, None, None, 0, 1.0, None, L.ct.byref(loss), None) == L.BQ_EINVAL
    with pytest.raises(ValueError):
        ctx.grad(xt, yt, idx, 0.5, out=torch.empty((16, 16, 16), dtype=torch.float32, device=dev))
    ctx.close()
    with pytest.raises(BQError) as e:
        _ctx(20, dirs, "f64")
    assert e.value.status == L.BQ_EUNSUPPORTED
    # an image far larger than the device memory: the first allocation fails
    with pytest.raises(BQError) as e:
        WProx((4096, 4096, 4096), "f64")
    assert e.value.status == L.BQ_ENOMEM
