"""bq_wprox_noalloc (no device allocation; a static per-GPU scratch array)
against bq_wprox on the same inputs, through the C ABI: two calls in a row
(the second on a smaller image, so that it runs over what the first left in
the array), plus ranks 0 and 3 and the size limit.  Bar: 1e-10 relative
(FP64) and 2e-4 (FP32), as for the prox against the oracle; the root passes
and the partial sums are the same in both, so they agree bit for bit in
practice."""
import numpy as np
import pytest

import synthetic as syn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _rel(a, b):
    return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))


def _inputs(shape, r, seed, dt, dev):
    rng = np.random.default_rng(seed)
    v = 0.03 * rng.random(shape) + 0.005 * rng.standard_normal(shape)
    u = 0.1 * rng.standard_normal(((r,) if r > 1 else ()) + shape) if r else None
    P0 = 0.3 * rng.standard_normal((3,) + shape)
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)  # noqa: E731
    return t(v), t(u), t(P0)


def _pair(dev, shape, prec, r, tv, cset, n_iter, seed, warm):
    from paper_2307_02043_amd import WProx
    from paper_2307_02043_amd.api import wprox_noalloc
    dt = torch.float32 if prec == "f32" else torch.float64
    v, u, P0 = _inputs(shape, r, seed, dt, dev)
    px = WProx(shape, prec)
    Pa = P0.clone() if warm else None
    xa, ia = px(v, 1.0, u, 2e-3, tv, cset, n_iter, P=Pa)
    px.close()
    Pb = P0.clone() if warm else None
    out = torch.full_like(v, float("nan"))
    xb, ib, status = wprox_noalloc(v, 1.0, u, 2e-3, tv, cset, n_iter, P=Pb, out=out)
    assert xb.data_ptr() == out.data_ptr() and status == 0
    torch.cuda.synchronize()
    lim = 1e-10 if prec == "f64" else 2e-4
    assert _rel(xb, xa) < lim, (shape, prec, r, _rel(xb, xa))
    if warm:
        assert _rel(Pb, Pa) < lim
    assert ib.newton_total >= 0 and ia.newton_max <= ib.newton_max + 1
    return xb


def test_noalloc_matches_wprox_on_two_calls_in_a_row(dev):
    # first call: rank one, FP64, warm-started dual point, 64 x 48 x 40
    _pair(dev, (64, 48, 40), "f64", 1, "iso", "nonneg", 30, 1, warm=True)
    # second call, smaller: it reads nothing the first call left behind
    _pair(dev, (20, 18, 16), "f64", 1, "iso", "nonneg", 25, 2, warm=False)


@pytest.mark.parametrize("prec,r,tv,cset", [("f32", 0, "iso", "nonneg"), ("f32", 3, "aniso", "nonneg"),
                                             ("f64", 2, "iso", "none"), ("f32", 1, "iso", "nonneg")])
def test_noalloc_matches_wprox_ranks(dev, prec, r, tv, cset):
    _pair(dev, (32, 24, 40), prec, r, tv, cset, 17, 10 + r, warm=(r == 0))
    _pair(dev, (12, 10, 8), prec, r, tv, cset, 9, 20 + r, warm=False)


def test_noalloc_full_size_and_limit(dev):
    from paper_2307_02043_amd import BQError
    from paper_2307_02043_amd.api import wprox_noalloc
    # 128^3 FP32 rank one fits the array
    w = syn.WORKLOADS["c4_ls128_f32"]
    x = _pair(dev, (w.N, w.N, w.N), "f32", 1, "iso", "nonneg", 20, 5, warm=False)
    assert torch.all(x >= 0)
    # 128^3 FP64 rank zero does not: a clear error, nothing launched
    v = torch.zeros((128, 128, 128), dtype=torch.float64, device=dev)
    with pytest.raises(BQError) as e:
        wprox_noalloc(v, 1.0, None, 1e-3, n_iter=3)
    assert e.value.status == -1 and "maximum" in str(e.value)
