"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds the input recipe only: refractive-index phantoms, illumination
directions, mini-batch draws, measurement noise and the inputs of the weighted
proximal mapping.  It contains none of the reconstruction method's arithmetic
(no Green's operator, no solver, no gradient, no TV proximal step), so that the
CPU oracle and the GPU path can both consume it without sharing code.

The paper's phantoms and its yeast-cell data are not available; the workloads
below are stand-ins with the shapes of its experiments (Section 6: a cube of a
few micrometres discretised at a fraction of the wavelength, background index
1.333, tens of tilted plane waves inside a cone of 35-42 degrees, index
contrast of a few hundredths).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Section 6.1: illumination wavelength 406 nm in a medium of index 1.333.
LAMBDA0_UM = 0.406
N_B = 1.333


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: grid, illuminations, solver and prox settings."""

    name: str
    index: int                 # 1-based configuration number (seeds derive from it)
    N: int                     # grid edge (voxels); padded edge is 2N
    L: int                     # number of illuminations
    B: int                     # mini-batch size
    model: str                 # "ls" (Lippmann-Schwinger) or "born"
    precision: str             # "f64" or "f32"
    tol: float                 # BiCGSTAB relative tolerance
    max_iter: int
    phantom: str               # "ellipsoids", "beads", "cell"
    contrast_scale: float = 1.0
    max_polar_deg: float = 35.0
    lambda0_um: float = LAMBDA0_UM
    n_b: float = N_B
    snr_db: float = 30.0
    prox_tv: str | None = None     # "iso" / "aniso" / None
    prox_lambda: float = 1e-3
    prox_iters: int = 0
    prox_tau: float = 1.0
    x_eval_scale: float = 0.5      # gradients are evaluated at this multiple of x_true
    extra: dict = field(default_factory=dict)

    @property
    def h_um(self) -> float:
        """Voxel edge: a quarter of the vacuum wavelength."""
        return self.lambda0_um / 4.0

    def seed(self, what: str) -> int:
        base = {"phantom": 1000, "illum": 2000, "noise": 3000,
                "batch": 4000, "prox": 5000}[what]
        return base + self.index


WORKLOADS = {
    "c1_ls32_f64": Workload("c1_ls32_f64", 1, N=32, L=4, B=4, model="ls",
                            precision="f64", tol=1e-8, max_iter=100,
                            phantom="ellipsoids", prox_tv="iso",
                            prox_lambda=1e-3, prox_iters=50),
    "c2_born64_f32": Workload("c2_born64_f32", 2, N=64, L=32, B=32,
                              model="born", precision="f32", tol=0.0,
                              max_iter=0, phantom="beads", prox_tv="aniso",
                              prox_lambda=1e-3, prox_iters=100),
    "c3_ls96_f32": Workload("c3_ls96_f32", 3, N=96, L=60, B=8, model="ls",
                            precision="f32", tol=1e-5, max_iter=300,
                            phantom="cell"),
    "c4_ls128_f32": Workload("c4_ls128_f32", 4, N=128, L=120, B=16,
                             model="ls", precision="f32", tol=1e-5,
                             max_iter=300, phantom="cell"),
    "c5_ls256_f32": Workload("c5_ls256_f32", 5, N=256, L=120, B=32,
                             model="ls", precision="f32", tol=1e-5,
                             max_iter=300, phantom="cell", contrast_scale=1.5,
                             prox_tv="iso", prox_lambda=1e-3, prox_iters=200),
    # stand-in for the strongly scattering simulated sample of Section 6.1
    # (maximal index 1.43 in a 1.333 medium, 60 illuminations in a 42 degree
    # cone, mini-batches of 15 = 60 / 4 subsets), on the 128^3 grid of
    # quarter-wavelength voxels: a solid cell body of delta n 0.06 with 20
    # nucleoli of 0.097, gradient evaluated at the phantom itself
    "c6_ls128_strong": Workload("c6_ls128_strong", 6, N=128, L=60, B=15,
                                model="ls", precision="f32", tol=1e-5,
                                max_iter=300, phantom="cell_solid",
                                max_polar_deg=42.0, x_eval_scale=1.0),
    # the 256^3 configuration in its strong multiple-scattering regime: a
    # solid cell body of delta n 0.037 with nucleoli of 0.06 (the largest
    # contrast that configuration names), gradient at the phantom itself
    "c7_ls256_strong": Workload("c7_ls256_strong", 7, N=256, L=120, B=32,
                                model="ls", precision="f32", tol=1e-5,
                                max_iter=300, phantom="cell_solid",
                                contrast_scale=0.06 / 0.097, x_eval_scale=1.0),
}


def voxel_centres(N: int, h: float) -> np.ndarray:
    """Voxel-centre coordinates along one axis, centred on the origin."""
    return (np.arange(N, dtype=np.float64) - (N - 1) / 2.0) * h


# --------------------------------------------------------------------------
# Refractive-index phantoms (delta n, C-order [z][y][x])
# --------------------------------------------------------------------------

def _coords(N: int, h: float):
    c = voxel_centres(N, h)
    return np.meshgrid(c, c, c, indexing="ij")  # Z, Y, X


def phantom_ellipsoids(N: int, h: float, rng: np.random.Generator,
                       n_incl: int = 3, dn_range=(0.01, 0.05)) -> np.ndarray:
    """Axis-aligned ellipsoidal inclusions; overlaps take the larger value."""
    Z, Y, X = _coords(N, h)
    ext = N * h
    dn = np.zeros((N, N, N))
    for _ in range(n_incl):
        c = rng.uniform(-0.25, 0.25, size=3) * ext
        a = rng.uniform(0.10, 0.25, size=3) * ext
        val = rng.uniform(*dn_range)
        inside = (((X - c[0]) / a[0]) ** 2 + ((Y - c[1]) / a[1]) ** 2
                  + ((Z - c[2]) / a[2]) ** 2) <= 1.0
        dn = np.where(inside, np.maximum(dn, val), dn)
    return dn


def phantom_beads(N: int, h: float, rng: np.random.Generator,
                  n_beads: int = 20, r_vox=(2.0, 6.0),
                  dn_range=(0.005, 0.03)) -> np.ndarray:
    """Spherical beads of random radius and contrast, fully inside the grid."""
    Z, Y, X = _coords(N, h)
    dn = np.zeros((N, N, N))
    half = (N / 2.0) * h
    for _ in range(n_beads):
        r = rng.uniform(*r_vox) * h
        lim = max(half - r - h, 0.0)
        c = rng.uniform(-lim, lim, size=3)
        val = rng.uniform(*dn_range)
        inside = ((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= r * r
        dn = np.where(inside, np.maximum(dn, val), dn)
    return dn


def phantom_cell(N: int, h: float, rng: np.random.Generator,
                 scale: float = 1.0) -> np.ndarray:
    """Hollow ellipsoidal shell (delta n 0.02) holding 20 nucleoli (0.04)."""
    Z, Y, X = _coords(N, h)
    ext = N * h
    a_out = np.array([0.40, 0.35, 0.30]) * ext
    thick = math.ceil(N / 24) * h
    a_in = a_out - thick
    q_out = (X / a_out[0]) ** 2 + (Y / a_out[1]) ** 2 + (Z / a_out[2]) ** 2
    q_in = (X / a_in[0]) ** 2 + (Y / a_in[1]) ** 2 + (Z / a_in[2]) ** 2
    dn = np.where((q_out <= 1.0) & (q_in > 1.0), 0.02, 0.0)
    for _ in range(20):
        r = rng.uniform(1.5, 4.0) * (N / 96.0) * h
        # centre drawn inside the inner ellipsoid, shrunk so the nucleolus fits
        while True:
            c = rng.uniform(-1.0, 1.0, size=3) * (a_in - r) * 0.8
            if np.sum((c / a_in) ** 2) <= 0.64:
                break
        inside = ((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= r * r
        dn = np.where(inside, np.maximum(dn, 0.04), dn)
    return dn * scale


def phantom_cell_solid(N: int, h: float, rng: np.random.Generator,
                       body_dn: float = 0.06, nucleolus_dn: float = 0.097) -> np.ndarray:
    """Solid ellipsoidal cell body (semi-axes 0.40, 0.35, 0.30 of the
    domain edge) holding 20 nucleoli of a higher index."""
    Z, Y, X = _coords(N, h)
    a = np.array([0.40, 0.35, 0.30]) * N * h
    q = (X / a[0]) ** 2 + (Y / a[1]) ** 2 + (Z / a[2]) ** 2
    dn = np.where(q <= 1.0, body_dn, 0.0)
    for _ in range(20):
        r = rng.uniform(1.5, 4.0) * (N / 96.0) * h
        c = rng.uniform(-1.0, 1.0, size=3) * (a - r) * 0.6
        inside = ((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) <= r * r
        dn = np.where(inside, nucleolus_dn, dn)
    return dn


def make_phantom(w: Workload) -> np.ndarray:
    rng = np.random.default_rng(w.seed("phantom"))
    if w.phantom == "ellipsoids":
        return phantom_ellipsoids(w.N, w.h_um, rng) * w.contrast_scale
    if w.phantom == "beads":
        return phantom_beads(w.N, w.h_um, rng) * w.contrast_scale
    if w.phantom == "cell":
        return phantom_cell(w.N, w.h_um, rng, scale=w.contrast_scale)
    if w.phantom == "cell_solid":
        return phantom_cell_solid(w.N, w.h_um, rng) * w.contrast_scale
    raise ValueError(w.phantom)


def scattering_potential(dn: np.ndarray, n_b: float = N_B,
                         lambda0_um: float = LAMBDA0_UM) -> np.ndarray:
    """Unknown of the reconstruction, k0^2 ((n_b + dn)^2 - n_b^2), in um^-2.

    This is how the synthetic refractive-index phantom is expressed in the
    variable the method optimises over (nonnegative for dn >= 0).
    """
    k0 = 2.0 * math.pi / lambda0_um
    return k0 * k0 * ((n_b + dn) ** 2 - n_b * n_b)


# --------------------------------------------------------------------------
# Illuminations, mini-batches, noise
# --------------------------------------------------------------------------

def illumination_directions(L: int, max_polar_deg: float,
                            rng: np.random.Generator) -> np.ndarray:
    """Unit propagation directions (L, 3) as (dx, dy, dz), dz > 0.

    Polar angles are uniform in [0, max_polar_deg]; azimuths are evenly spaced
    on the circle.
    """
    theta = np.deg2rad(rng.uniform(0.0, max_polar_deg, size=L))
    phi = 2.0 * np.pi * np.arange(L) / L
    return np.stack([np.sin(theta) * np.cos(phi),
                     np.sin(theta) * np.sin(phi),
                     np.cos(theta)], axis=1)


def workload_directions(w: Workload) -> np.ndarray:
    return illumination_directions(w.L, w.max_polar_deg,
                                   np.random.default_rng(w.seed("illum")))


def batch_indices(w: Workload) -> np.ndarray:
    """Mini-batch of B distinct illumination indices (all of them if B == L)."""
    if w.B >= w.L:
        return np.arange(w.L, dtype=np.int32)
    rng = np.random.default_rng(w.seed("batch"))
    return np.sort(rng.choice(w.L, size=w.B, replace=False)).astype(np.int32)


def add_noise(y_clean: np.ndarray, snr_db: float,
              rng: np.random.Generator) -> np.ndarray:
    """Circular complex Gaussian noise at the given SNR, per illumination.

    y_clean has shape (B, M...); each row gets variance
    ||y_l||^2 / (M 10^(snr/10)), split evenly between real and imaginary parts.
    """
    y = np.asarray(y_clean, dtype=np.complex128)
    out = np.empty_like(y)
    for l in range(y.shape[0]):
        m = y[l].size
        sig2 = np.vdot(y[l], y[l]).real / (m * 10.0 ** (snr_db / 10.0))
        s = math.sqrt(sig2 / 2.0)
        out[l] = y[l] + s * (rng.standard_normal(y[l].shape)
                             + 1j * rng.standard_normal(y[l].shape))
    return out


def prox_inputs(w: Workload, dn: np.ndarray | None = None):
    """(v, tau, u) for the weighted TV proximal mapping of a workload.

    v is the phantom plus N(0, 0.005^2) noise (so that the nonnegativity
    constraint is active), the metric is tau I + u u^T with u ~ 0.1 N(0, 1).
    """
    if dn is None:
        dn = make_phantom(w)
    rng = np.random.default_rng(w.seed("prox"))
    v = dn + 0.005 * rng.standard_normal(dn.shape)
    u = 0.1 * rng.standard_normal(dn.shape)
    return v, float(w.prox_tau), u


def random_field(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex normal test vector."""
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def detector_images(B: int, N: int, rng: np.random.Generator, scale: float = 0.1) -> np.ndarray:
    """Stand-in measurements (B, N, N): circular complex Gaussian images of
    the size of a scattered field on the detector, for parity tests of the
    gradient, which is defined for any measurement."""
    return scale * (rng.standard_normal((B, N, N)) + 1j * rng.standard_normal((B, N, N))) / math.sqrt(2.0)
