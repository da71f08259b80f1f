"""Writes the oracle's results at the 256^3 configuration for the GPU parity
tests that the oracle cannot finish inside a test (hours of FP64 CPU work
otherwise repeated on every run).  Calls only oracle/ and synthetic/.

    python tests/golden/make_fullsize_refs.py [grad|fields|strong|strong_fields|strong256_fields|prox|prox_tau|qn_step|all] [workers]

grad: the 256^3 workload with contrast x1.5 (c5_ls256_f32), the first two
      illuminations of its mini-batch.  Measurements y = H(x_true) (oracle
      forward solves at tol 1e-11) plus 30 dB noise, stored as complex64 (the
      GPU's FP32 path reads them as they are; the oracle uses the same values
      widened to complex128).  The gradient and loss at x = 0.5 x_true with
      scale 1/2 (oracle solves at tol 1e-11), kept at 8192 seeded voxels
      together with whole-array sums.
strong: the strongly scattering 128^3 workload (c6_ls128_strong), its first
      two mini-batch illuminations: measurements H(x_true) (tol 1e-13) plus
      30 dB noise, stored as complex128, and the FP64 gradient and loss at
      x_true with scale 1/2 (tol 1e-13 on both sides of the comparison),
      kept at 8192 seeded voxels, with the iteration counts.
fields: the 256^3 workload's whole launch set of 32 illuminations with
      stand-in detector images (synthetic.detector_images, stored as
      complex64) at x = 0.5 x_true (in float32 values): the forward and the
      adjoint fields of the first and the last system (oracle solves at tol
      1e-12), kept at 8192 seeded voxels with their whole-array norms.
strong_fields: the strongly scattering workload's whole launch set of 15
      with stand-in detector images (complex64) at its evaluation point (in
      float32 values): forward and adjoint fields of the first and the last
      system (tol 1e-13), kept at 8192 seeded voxels with their norms.
strong256_fields: the strongly scattering 256^3 workload (c7_ls256_strong)
      in the same way, oracle tol 1e-11.
prox: the weighted TV prox of the same workload: iso TV, nonnegativity,
      metric tau I + u u^T (rank one), lambda 1e-3, 200 dual iterations
      (Section 4.1 iteration, Theorem 3.1 projection), kept at 8192 seeded
      voxels together with whole-array sums.
prox_tau: the same prox under the metric tau I (no u).
qn_step: the first outer iteration (Algorithm 4.1, S = 4 subsets of 16) on the
      128^3 workload from x_0 = 0.5 x_true (in float32 values) with stand-in
      detector images for its first subset: the subset gradient (oracle
      solves at tol 1e-13) and the iterate x_1, kept at 8192 seeded voxels
      with their norms.
Each file records a digest of the oracle sources it was made with and one
of its input arrays; the tests refuse a file whose oracle digest no longer
matches, or whose inputs differ from those the synthetic generators give.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthetic as syn  # noqa: E402
from oracle import bqnpm, lsmodel, tvprox  # noqa: E402

SAMPLES = 8192


def source_digest(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def array_digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


GRAD_SOURCES = ("oracle/green.py", "oracle/lsmodel.py")
PROX_SOURCES = ("oracle/tvprox.py",)


def sample_index(V: int, seed: int) -> np.ndarray:
    return np.sort(np.random.default_rng(seed).choice(V, size=SAMPLES, replace=False)).astype(np.int64)


def make_grad(workers: int) -> None:
    w = syn.WORKLOADS["c5_ls256_f32"]
    N = w.N
    geom = lsmodel.Geometry(N=N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    print(f"kernel {time.time() - t0:.0f} s", flush=True)
    xt = syn.scattering_potential(syn.make_phantom(w))
    dirs = syn.workload_directions(w)
    idx = [int(i) for i in syn.batch_indices(w)[:2]]
    yc, st = m.forward(xt, dirs, idx, 1e-11, 500)
    print(f"forward {time.time() - t0:.0f} s, iterations {[s[0] for s in st]}", flush=True)
    y = syn.add_noise(yc, w.snr_db, np.random.default_rng(w.seed("noise"))).astype(np.complex64)
    x = 0.5 * xt
    g, f, st = m.grad(x, y.astype(np.complex128), dirs, idx, 0.5, 1e-11, 500)
    print(f"gradient {time.time() - t0:.0f} s, iterations {st}", flush=True)
    sel = sample_index(g.size, 7256)
    np.savez(os.path.join(HERE, "c5_grad256_b2.npz"), idx=np.array(idx, np.int32), y=y, loss=f,
             sel=sel, g_sel=g.ravel()[sel], g_norm=np.linalg.norm(g), g_sum=g.sum(),
             iters=np.array(st, np.int32), digest=source_digest(GRAD_SOURCES),
             inputs=array_digest(x, dirs))


def c5_field_inputs():
    """x, y, directions and batch of the 256^3 launch-set field references
    (the GPU test rebuilds them the same way)."""
    w = syn.WORKLOADS["c5_ls256_f32"]
    x = (0.5 * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 100)).astype(np.complex64)
    return x, y, syn.workload_directions(w), [int(i) for i in syn.batch_indices(w)]


def make_fields(workers: int) -> None:
    w = syn.WORKLOADS["c5_ls256_f32"]
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    x, y, dirs, idx = c5_field_inputs()
    sel = sample_index(x.size, 7259)
    out = {}
    for b in (0, w.B - 1):
        uin = lsmodel.incident_field(geom, dirs[idx[b]])
        u, itf, sf, _ = m.solve_forward(x, uin, 1e-12, 500)
        r = m.detector(u - uin) - y[b].astype(np.complex128)
        wv, ita, sa, _ = m.solve_adjoint(x, m.GH(m.detector_T(r)), 1e-12, 500)
        assert sf == lsmodel.CONVERGED and sa == lsmodel.CONVERGED
        print(f"system {b}: {time.time() - t0:.0f} s, iterations {itf} / {ita}", flush=True)
        out[f"u{b}_sel"] = u.ravel()[sel]
        out[f"w{b}_sel"] = wv.ravel()[sel]
        out[f"u{b}_norm"] = np.linalg.norm(u)
        out[f"w{b}_norm"] = np.linalg.norm(wv)
        out[f"loss{b}"] = 0.5 * float(np.vdot(r, r).real)
        out[f"iters{b}"] = np.array([itf, ita], np.int32)
    np.savez(os.path.join(HERE, "c5_fields256_b32.npz"), sel=sel, systems=np.array([0, w.B - 1], np.int32),
             digest=source_digest(GRAD_SOURCES), inputs=array_digest(x, y, dirs), **out)


def c6_field_inputs():
    """x, y, directions and batch of the strongly scattering launch-set field
    references (the GPU test rebuilds them the same way)."""
    w = syn.WORKLOADS["c6_ls128_strong"]
    x = (w.x_eval_scale * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 100)).astype(np.complex64)
    return x, y, syn.workload_directions(w), [int(i) for i in syn.batch_indices(w)]


def make_strong_fields(workers: int) -> None:
    w = syn.WORKLOADS["c6_ls128_strong"]
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    x, y, dirs, idx = c6_field_inputs()
    sel = sample_index(x.size, 7260)
    out = {}
    for b in (0, w.B - 1):
        uin = lsmodel.incident_field(geom, dirs[idx[b]])
        u, itf, sf, _ = m.solve_forward(x, uin, 1e-13, 1000)
        r = m.detector(u - uin) - y[b].astype(np.complex128)
        wv, ita, sa, _ = m.solve_adjoint(x, m.GH(m.detector_T(r)), 1e-13, 1000)
        assert sf == lsmodel.CONVERGED and sa == lsmodel.CONVERGED
        print(f"system {b}: {time.time() - t0:.0f} s, iterations {itf} / {ita}", flush=True)
        out[f"u{b}_sel"] = u.ravel()[sel]
        out[f"w{b}_sel"] = wv.ravel()[sel]
        out[f"u{b}_norm"] = np.linalg.norm(u)
        out[f"w{b}_norm"] = np.linalg.norm(wv)
        out[f"iters{b}"] = np.array([itf, ita], np.int32)
    np.savez(os.path.join(HERE, "c6_fields128_strong_b15.npz"), sel=sel,
             systems=np.array([0, w.B - 1], np.int32), digest=source_digest(GRAD_SOURCES),
             inputs=array_digest(x, y, dirs), **out)


def c7_field_inputs():
    """x, y, directions and batch of the strongly scattering 256^3
    launch-set field references (the GPU test rebuilds them the same way)."""
    w = syn.WORKLOADS["c7_ls256_strong"]
    x = (w.x_eval_scale * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 100)).astype(np.complex64)
    return x, y, syn.workload_directions(w), [int(i) for i in syn.batch_indices(w)]


def make_strong256_fields(workers: int) -> None:
    w = syn.WORKLOADS["c7_ls256_strong"]
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    x, y, dirs, idx = c7_field_inputs()
    sel = sample_index(x.size, 7261)
    out = {}
    for b in (0, w.B - 1):
        uin = lsmodel.incident_field(geom, dirs[idx[b]])
        u, itf, sf, _ = m.solve_forward(x, uin, 1e-11, 1000)
        print(f"system {b} forward: {time.time() - t0:.0f} s, iterations {itf}", flush=True)
        r = m.detector(u - uin) - y[b].astype(np.complex128)
        wv, ita, sa, _ = m.solve_adjoint(x, m.GH(m.detector_T(r)), 1e-11, 1000)
        assert sf == lsmodel.CONVERGED and sa == lsmodel.CONVERGED
        print(f"system {b}: {time.time() - t0:.0f} s, iterations {itf} / {ita}", flush=True)
        out[f"u{b}_sel"] = u.ravel()[sel]
        out[f"w{b}_sel"] = wv.ravel()[sel]
        out[f"u{b}_norm"] = np.linalg.norm(u)
        out[f"w{b}_norm"] = np.linalg.norm(wv)
        out[f"iters{b}"] = np.array([itf, ita], np.int32)
    np.savez(os.path.join(HERE, "c7_fields256_strong_b32.npz"), sel=sel,
             systems=np.array([0, w.B - 1], np.int32), digest=source_digest(GRAD_SOURCES),
             inputs=array_digest(x, y, dirs), **out)


def make_strong(workers: int) -> None:
    w = syn.WORKLOADS["c6_ls128_strong"]
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    xt = syn.scattering_potential(syn.make_phantom(w))
    dirs = syn.workload_directions(w)
    idx = [int(i) for i in syn.batch_indices(w)[:2]]
    yc, st = m.forward(xt, dirs, idx, 1e-13, 1000)
    print(f"forward {time.time() - t0:.0f} s, iterations {[s[0] for s in st]}", flush=True)
    y = syn.add_noise(yc, w.snr_db, np.random.default_rng(w.seed("noise")))
    x = w.x_eval_scale * xt
    g, f, st = m.grad(x, y, dirs, idx, 0.5, 1e-13, 1000)
    print(f"gradient {time.time() - t0:.0f} s, iterations {st}", flush=True)
    sel = sample_index(g.size, 7128)
    np.savez(os.path.join(HERE, "c6_grad128_strong_b2.npz"), idx=np.array(idx, np.int32), y=y, loss=f,
             sel=sel, g_sel=g.ravel()[sel], g_norm=np.linalg.norm(g), iters=np.array(st, np.int32),
             digest=source_digest(GRAD_SOURCES), inputs=array_digest(x, dirs))


def make_prox() -> None:
    w = syn.WORKLOADS["c5_ls256_f32"]
    v, tau, u = syn.prox_inputs(w)
    t0 = time.time()
    x = tvprox.wprox(v, tau, u, w.prox_lambda, "iso", "nonneg", n_iter=w.prox_iters)
    print(f"prox {time.time() - t0:.0f} s", flush=True)
    sel = sample_index(x.size, 7257)
    np.savez(os.path.join(HERE, "c5_prox256_k200.npz"), x_sel=x.ravel()[sel], sel=sel,
             x_norm=np.linalg.norm(x), x_sum=x.sum(), x_pos=int(np.count_nonzero(x > 0)),
             n_iter=w.prox_iters, lam=w.prox_lambda, tau=tau, digest=source_digest(PROX_SOURCES),
             inputs=array_digest(v, u))


QN_SOURCES = GRAD_SOURCES + PROX_SOURCES + ("oracle/bqnpm.py",)


def qn_step_inputs():
    """x_0, the first subset's stand-in detector images, directions and the
    subsets of the full-size outer-iteration reference (the GPU test
    rebuilds them the same way)."""
    w = syn.WORKLOADS["c4_ls128_f32"]
    x0 = (0.5 * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y0 = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 200)).astype(np.complex64)
    subsets = [list(range(s * w.B, (s + 1) * w.B)) for s in range(4)]
    return x0, y0, syn.workload_directions(w), subsets


def make_qn_step(workers: int) -> None:
    w = syn.WORKLOADS["c4_ls128_f32"]
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t0 = time.time()
    m = lsmodel.LSModel(geom, workers=workers)
    x0, y0, dirs, subsets = qn_step_inputs()
    S = len(subsets)
    xt = syn.scattering_potential(syn.make_phantom(w))
    g0, f0, st = m.grad(x0, y0.astype(np.complex128), dirs, subsets[0], S / w.L, 1e-13, 300)
    print(f"gradient {time.time() - t0:.0f} s, iterations {st}", flush=True)
    alpha = float(np.abs(g0).max() / xt.max())
    prm = bqnpm.BQNPMParams(S=S, a=1.0 / 20, lam=1.0 / w.N ** 3, alpha=alpha, prox_iters=50)
    # the first outer iteration takes subset 0, whose gradient is g0
    it = bqnpm.BQNPM(prm, lambda s, x: g0)
    x1, sp, _ = it.step(x0)
    assert sp == 0
    print(f"outer step {time.time() - t0:.0f} s", flush=True)
    sel = sample_index(x0.size, 7263)
    np.savez(os.path.join(HERE, "c4_qn_step128_b16.npz"), sel=sel, g_sel=g0.ravel()[sel],
             g_norm=np.linalg.norm(g0), loss=f0, x1_sel=x1.ravel()[sel], x1_norm=np.linalg.norm(x1),
             alpha=alpha, a=prm.a, lam=prm.lam, S=S, prox_iters=prm.prox_iters,
             iters=np.array(st, np.int32), digest=source_digest(QN_SOURCES), inputs=array_digest(x0, y0, dirs))


def make_prox_tau() -> None:
    w = syn.WORKLOADS["c5_ls256_f32"]
    v, tau, _ = syn.prox_inputs(w)
    t0 = time.time()
    x = tvprox.wprox(v, tau, None, w.prox_lambda, "iso", "nonneg", n_iter=w.prox_iters)
    print(f"prox (metric tau I) {time.time() - t0:.0f} s", flush=True)
    sel = sample_index(x.size, 7262)
    np.savez(os.path.join(HERE, "c5_prox256_tau_k200.npz"), x_sel=x.ravel()[sel], sel=sel,
             x_norm=np.linalg.norm(x), x_sum=x.sum(), x_pos=int(np.count_nonzero(x > 0)),
             n_iter=w.prox_iters, lam=w.prox_lambda, tau=tau, digest=source_digest(PROX_SOURCES),
             inputs=array_digest(v))


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    workers = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    if what in ("grad", "all"):
        make_grad(workers)
    if what in ("fields", "all"):
        make_fields(workers)
    if what in ("strong", "all"):
        make_strong(workers)
    if what in ("strong_fields", "all"):
        make_strong_fields(workers)
    if what in ("strong256_fields", "all"):
        make_strong256_fields(workers)
    if what in ("prox", "all"):
        make_prox()
    if what in ("prox_tau", "all"):
        make_prox_tau()
    if what in ("qn_step", "all"):
        make_qn_step(workers)
