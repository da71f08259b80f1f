"""Pins of the oracle's Lippmann-Schwinger data term.

* BiCGSTAB agrees with a dense LU solve of I - G diag(x) built column by
  column from the operator (8^3, 12^3);
* first-Born limit: (u(eps x) - u_in)/eps -> G(x u_in) with error O(eps);
* at x = 0 the LS gradient is exactly the first-Born gradient;
* adjoint identity <J v, w> = <v, J^H w>, with J v from an independent
  tangent solve;
* the gradient matches FP64 central finite differences of the loss on 16^3;
* warm-started solves (a given starting point) reach the dense solutions,
  return the start unchanged when it is exact and zero for a zero
  right-hand side; the warm-started gradient equals the cold one.
"""
import math

import numpy as np
import pytest

import synthetic as syn
from oracle import green, lsmodel

LAM0, NB = syn.LAMBDA0_UM, syn.N_B


def _geom(N):
    return lsmodel.Geometry(N=N, h=LAM0 / 4, lambda0=LAM0, n_b=NB)


def _phantom(N, seed):
    rng = np.random.default_rng(seed)
    dn = syn.phantom_ellipsoids(N, LAM0 / 4, rng, n_incl=3, dn_range=(0.01, 0.05))
    return syn.scattering_potential(dn)


def _dense_operator(model, x):
    N = model.geom.N
    n = N ** 3
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        col = e.reshape(N, N, N)
        A[:, j] = (col - model.G(x * col)).ravel()
    return A


@pytest.mark.parametrize("N", [8, 12])
def test_bicgstab_matches_dense_lu(N):
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    x = _phantom(N, 100 + N) + 5.0
    d = syn.illumination_directions(1, 35.0, np.random.default_rng(N))[0]
    uin = lsmodel.incident_field(geom, d)
    u, it, st, _ = model.solve_forward(x, uin, 1e-14, 500)
    assert st == lsmodel.CONVERGED and it > 2
    A = _dense_operator(model, x)
    ud = np.linalg.solve(A, uin.ravel()).reshape(u.shape)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-12


def test_born_limit_is_first_order():
    N = 12
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    x = _phantom(N, 5)
    d = (0.2, -0.1, math.sqrt(1 - 0.05))
    uin = lsmodel.incident_field(geom, d)
    born = model.G(x * uin)
    eps = np.array([1e-1, 1e-2, 1e-3, 1e-4])
    err = []
    for e in eps:
        u, _, st, _ = model.solve_forward(e * x, uin, 1e-15, 500)
        err.append(np.linalg.norm((u - uin) / e - born) / np.linalg.norm(born))
    slope = np.polyfit(np.log(eps), np.log(err), 1)[0]
    assert abs(slope - 1.0) < 0.05, (slope, err)


def test_gradient_at_zero_equals_born_gradient():
    N = 12
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    dirs = syn.illumination_directions(3, 35.0, np.random.default_rng(1))
    rng = np.random.default_rng(2)
    y = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    idx = [0, 1, 2]
    x0 = np.zeros((N, N, N))
    g_ls, f_ls, st = model.grad(x0, y, dirs, idx, 1 / 3, 1e-12, 100, model="ls")
    g_b, f_b, _ = model.grad(x0, y, dirs, idx, 1 / 3, 1e-12, 100, model="born")
    assert all(s[0] == 0 and s[1] == 0 for s in st)
    assert np.max(np.abs(g_ls - g_b)) <= 1e-14 * np.max(np.abs(g_b))
    assert f_ls == pytest.approx(f_b, rel=1e-15)
    # At x = 0 the prediction is zero, so r_l = -y_l and the gradient is
    # (1/3) sum_l Re(conj(u_in,l) G^H S^T (-y_l)).
    ref = np.zeros((N, N, N))
    for l in idx:
        uin = lsmodel.incident_field(geom, dirs[l])
        ref += np.real(np.conj(uin) * green.apply_GH(model.ghat, model.detector_T(-y[l])))
    assert np.max(np.abs(g_b - ref / 3)) <= 1e-14 * np.max(np.abs(ref))
    assert f_b == pytest.approx(0.5 / 3 * float(np.sum(np.abs(y) ** 2)), rel=1e-14)


def test_adjoint_identity():
    N = 12
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    x = _phantom(N, 9)
    d = syn.illumination_directions(1, 35.0, np.random.default_rng(4))[0]
    rng = np.random.default_rng(8)
    v = rng.standard_normal((N, N, N))
    w = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    Jv = model.tangent(x, d, v, 1e-14, 500)
    JHw = model.vjp(x, d, w, 1e-14, 500)
    lhs = np.vdot(Jv, w)
    rhs = np.sum(v * JHw)
    assert abs(lhs - rhs) / abs(lhs) < 1e-11


@pytest.mark.slow
def test_gradient_matches_central_differences():
    N = 16
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    xt = _phantom(N, 21)
    dirs = syn.illumination_directions(2, 35.0, np.random.default_rng(3))
    idx = [0, 1]
    yc, _ = model.forward(xt, dirs, idx, 1e-14, 500)
    y = syn.add_noise(yc, 30.0, np.random.default_rng(4))
    x = 0.5 * xt
    scale = 0.5
    g, f, _ = model.grad(x, y, dirs, idx, scale, 1e-14, 500)

    def loss(xx):
        H, _ = model.forward(xx, dirs, idx, 1e-14, 500)
        return scale * 0.5 * float(np.sum(np.abs(H - y) ** 2))

    assert loss(x) == pytest.approx(f, rel=1e-12)
    # step 1e-4 max(x): smaller steps are limited by the 1e-14 solver
    # tolerance (loss differences of ~1e-11), larger ones by O(step^2).
    step = 1e-4 * np.max(x)
    rng = np.random.default_rng(6)
    checks = []
    for _ in range(3):
        e = rng.standard_normal(x.shape)
        e /= np.linalg.norm(e)
        fd = (loss(x + step * e) - loss(x - step * e)) / (2 * step)
        checks.append((fd, float(np.sum(g * e))))
    big = np.argsort(-np.abs(g).ravel())[:4]
    for flat in big:
        e = np.zeros(x.size)
        e[flat] = 1.0
        e = e.reshape(x.shape)
        fd = (loss(x + step * e) - loss(x - step * e)) / (2 * step)
        checks.append((fd, float(g.ravel()[flat])))
    for fd, an in checks:
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.max(np.abs(g))), (fd, an)


def test_warm_started_solves():
    """Warm start: from the exact solution no iteration is taken and the
    start is returned; from a perturbed start the solve reaches the dense
    solution of the forward and adjoint systems; a zero right-hand side
    gives zero whatever the start."""
    N = 8
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    x = _phantom(N, 7) + 3.0
    d = syn.illumination_directions(1, 35.0, np.random.default_rng(3))[0]
    uin = lsmodel.incident_field(geom, d)
    A = _dense_operator(model, x)
    ud = np.linalg.solve(A, uin.ravel()).reshape(uin.shape)
    u, it, st, _ = model.solve_forward(x, uin, 1e-12, 500, e0=ud)
    assert it == 0 and st == lsmodel.CONVERGED and np.array_equal(u, ud)
    rng = np.random.default_rng(4)
    start = ud + 0.05 * (rng.standard_normal(ud.shape) + 1j * rng.standard_normal(ud.shape))
    u, it, st, _ = model.solve_forward(x, uin, 1e-14, 500, e0=start)
    assert st == lsmodel.CONVERGED and it > 0
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-12
    # adjoint system (I - G^H X) w = z from a random start, vs the dense solve
    z = rng.standard_normal(ud.shape) + 1j * rng.standard_normal(ud.shape)
    AH = np.empty_like(A)
    e = np.zeros(N ** 3, dtype=np.complex128)
    for j in range(N ** 3):
        e[:] = 0
        e[j] = 1
        col = e.reshape(N, N, N)
        AH[:, j] = (col - model.GH(x * col)).ravel()
    wd = np.linalg.solve(AH, z.ravel()).reshape(z.shape)
    w, it, st, _ = model.solve_adjoint(x, z, 1e-14, 500, e0=start)
    assert st == lsmodel.CONVERGED
    assert np.linalg.norm(w - wd) / np.linalg.norm(wd) < 1e-12
    w0, it0, st0, _ = model.solve_adjoint(x, np.zeros_like(z), 1e-14, 500, e0=start)
    assert it0 == 0 and st0 == lsmodel.CONVERGED and not np.any(w0)


def test_warm_started_gradient_equals_cold_gradient():
    """The gradient does not depend on where the solves start (to the solve
    tolerance), and a start near the solution saves iterations."""
    N = 12
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    xt = _phantom(N, 11)
    dirs = syn.illumination_directions(3, 35.0, np.random.default_rng(12))
    idx = [0, 2]
    y, _ = model.forward(xt, dirs, idx, 1e-13, 400)
    x = 0.5 * xt
    g0, f0, st0, fields = model.grad(x, y, dirs, idx, 0.5, 1e-13, 400, return_fields=True)
    x1 = x * 1.02
    gc, fc, stc = model.grad(x1, y, dirs, idx, 0.5, 1e-13, 400)
    gw, fw, stw = model.grad(x1, y, dirs, idx, 0.5, 1e-13, 400, starts=fields)
    assert np.linalg.norm(gw - gc) / np.linalg.norm(gc) < 1e-10
    assert abs(fw - fc) < 1e-10 * fc
    assert sum(s[0] + s[1] for s in stw) < sum(s[0] + s[1] for s in stc)


@pytest.mark.parametrize("N", [7, 8, 13])
def test_incident_field_is_the_plane_wave_of_the_background(N):
    """The illumination of Section 6.1 is a plane wave in the background
    medium: a unit-modulus field whose phase advances by k_b d_a h per voxel
    along axis a (k_b = 2 pi n_b / lambda0, not the vacuum k0), that
    satisfies the discrete Helmholtz equation of the background exactly, and
    whose phase origin is the centre of the domain.  Each check fails for
    one plausible misreading: k0 for k_b, a flipped or permuted direction
    component, an origin at a corner or half a voxel off."""
    geom = _geom(N)
    h, kb = geom.h, 2 * math.pi * NB / LAM0
    assert abs(geom.kb - kb) < 1e-12 * kb
    d = np.array([0.31, -0.22, 0.0])
    d[2] = math.sqrt(1 - d[0] ** 2 - d[1] ** 2)
    u = lsmodel.incident_field(geom, tuple(d))
    assert u.shape == (N, N, N)
    assert np.max(np.abs(np.abs(u) - 1)) < 1e-14
    # per-voxel phase advance along x (array axis 2), y (1), z (0)
    for axis, comp in ((2, d[0]), (1, d[1]), (0, d[2])):
        ratio = np.take(u, np.arange(1, N), axis=axis) / np.take(u, np.arange(N - 1), axis=axis)
        assert np.max(np.abs(ratio - np.exp(1j * kb * comp * h))) < 1e-12
    # the 7-point Laplacian of exp(i k.r) is exactly
    # -sum_a (4/h^2) sin^2(k_a h / 2) times the field, and that factor tends
    # to -k_b^2 as h -> 0 (O(h^2))
    lap = (u[2:, 1:-1, 1:-1] + u[:-2, 1:-1, 1:-1] + u[1:-1, 2:, 1:-1] + u[1:-1, :-2, 1:-1]
           + u[1:-1, 1:-1, 2:] + u[1:-1, 1:-1, :-2] - 6 * u[1:-1, 1:-1, 1:-1]) / h ** 2
    fac = -sum(4 / h ** 2 * math.sin(kb * c * h / 2) ** 2 for c in d)
    assert np.max(np.abs(lap - fac * u[1:-1, 1:-1, 1:-1])) < 1e-9 * kb ** 2
    # (k_b h is about 2.1 here, a quarter wavelength per voxel in vacuum, so
    # the O(h^2) term is about a quarter of k_b^2 at the grid's own spacing)
    assert abs(fac + kb ** 2) < 0.3 * kb ** 2
    # on finer grids the oracle's field's Laplacian tends to -k_b^2 u at O(h^2)
    errs = []
    for hh in (h / 8, h / 16):
        g2 = lsmodel.Geometry(N=N, h=hh, lambda0=LAM0, n_b=NB)
        w = lsmodel.incident_field(g2, tuple(d))
        lw = (w[2:, 1:-1, 1:-1] + w[:-2, 1:-1, 1:-1] + w[1:-1, 2:, 1:-1] + w[1:-1, :-2, 1:-1]
              + w[1:-1, 1:-1, 2:] + w[1:-1, 1:-1, :-2] - 6 * w[1:-1, 1:-1, 1:-1]) / hh ** 2
        errs.append(np.max(np.abs(lw / w[1:-1, 1:-1, 1:-1] + kb ** 2)))
    assert errs[0] < 0.02 * kb ** 2 and abs(errs[0] / errs[1] - 4) < 0.1, errs
    # phase origin at the domain centre: u(-r) = conj(u(r)) for every voxel,
    # and for odd N the centre voxel has phase 0
    assert np.max(np.abs(u[::-1, ::-1, ::-1] - np.conj(u))) < 1e-12
    if N % 2:
        c = (N - 1) // 2
        assert abs(u[c, c, c] - 1) < 1e-15
    # a corner voxel sits at r = -(N-1)/2 h on every axis
    corner = np.exp(-1j * kb * (N - 1) / 2 * h * d.sum())
    assert abs(u[0, 0, 0] - corner) < 1e-12


def test_breakdown_floor_stops_where_an_iteration_cap_would():
    """BiCGSTAB with a breakdown floor stops at the first |rho| below it;
    its iterate is then the one a run capped at that many iterations
    returns, and a floor above every scalar stops before the first
    iteration with the starting point."""
    N = 12
    geom = _geom(N)
    model = lsmodel.LSModel(geom)
    x = _phantom(N, 5)
    d = syn.illumination_directions(1, 35.0, np.random.default_rng(2))[0]
    uin = lsmodel.incident_field(geom, d)
    u, it, st, _ = model.solve_forward(x, uin, 1e-15, 50, breakdown=1e300)
    assert st == lsmodel.BREAKDOWN and it == 0 and np.array_equal(u, uin)
    # |rho_k| = |<rhat, r_{k-1}>| falls geometrically with k, so each floor
    # is crossed after some iterations, later for a lower floor
    ref_it = None
    for floor in (1e-2, 1e-4, 1e-6):
        u, it, st, _ = model.solve_forward(x, uin, 0.0, 40, breakdown=floor)
        assert st == lsmodel.BREAKDOWN and 0 < it < 40
        uc, itc, stc, _ = model.solve_forward(x, uin, 0.0, it)
        assert itc == it and stc == lsmodel.NOT_CONVERGED and np.array_equal(u, uc)
        assert ref_it is None or it >= ref_it
        ref_it = it
