"""The stored oracle results under tests/golden/ are still those of the
current oracle and inputs: each file's digest of the oracle sources it was
made with, and of the input arrays, against the sources and the seeded
generators as they are now (the GPU parity tests refuse a stale file; this
check finds one without a GPU).  The inputs are rebuilt exactly as the
generator script builds them."""
import hashlib
import os

import numpy as np
import pytest

import synthetic as syn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")
GRAD = ("oracle/green.py", "oracle/lsmodel.py")
PROX = ("oracle/tvprox.py",)


def _digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _array_digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def _field_inputs(name):
    w = syn.WORKLOADS[name]
    x = (w.x_eval_scale * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 100)).astype(np.complex64)
    return x, y, syn.workload_directions(w)


def _grad_inputs(name):
    w = syn.WORKLOADS[name]
    return w.x_eval_scale * syn.scattering_potential(syn.make_phantom(w)), syn.workload_directions(w)


def _prox_inputs(name):
    v, _, u = syn.prox_inputs(syn.WORKLOADS[name])
    return v, u


def _qn_step_inputs():
    w = syn.WORKLOADS["c4_ls128_f32"]
    x0 = (0.5 * syn.scattering_potential(syn.make_phantom(w))).astype(np.float32).astype(np.float64)
    y0 = syn.detector_images(w.B, w.N, np.random.default_rng(w.seed("noise") + 200)).astype(np.complex64)
    return x0, y0, syn.workload_directions(w)


CASES = [
    ("c4_qn_step128_b16.npz", GRAD + PROX + ("oracle/bqnpm.py",), _qn_step_inputs),
    ("c5_grad256_b2.npz", GRAD, lambda: _grad_inputs("c5_ls256_f32")),
    ("c5_fields256_b32.npz", GRAD, lambda: _field_inputs("c5_ls256_f32")),
    ("c5_prox256_k200.npz", PROX, lambda: _prox_inputs("c5_ls256_f32")),
    ("c5_prox256_tau_k200.npz", PROX, lambda: _prox_inputs("c5_ls256_f32")[:1]),
    ("c6_grad128_strong_b2.npz", GRAD, lambda: _grad_inputs("c6_ls128_strong")),
    ("c6_fields128_strong_b15.npz", GRAD, lambda: _field_inputs("c6_ls128_strong")),
    ("c7_fields256_strong_b32.npz", GRAD, lambda: _field_inputs("c7_ls256_strong")),
]


@pytest.mark.parametrize("name,sources,inputs", CASES, ids=[c[0] for c in CASES])
def test_stored_oracle_results_are_current(name, sources, inputs):
    path = os.path.join(GOLDEN, name)
    assert os.path.exists(path), f"{name} missing: run tests/golden/make_fullsize_refs.py"
    d = np.load(path, allow_pickle=False)
    assert str(d["digest"]) == _digest(sources), f"{name}: made with other oracle sources"
    assert str(d["inputs"]) == _array_digest(*inputs()), f"{name}: made from other inputs"


def test_every_stored_file_is_checked():
    stored = sorted(f for f in os.listdir(GOLDEN) if f.endswith(".npz"))
    assert stored == sorted(c[0] for c in CASES)
