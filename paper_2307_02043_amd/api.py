"""Python binding of the bq library: argument marshalling only.

Every step of the data-term gradient and of the weighted prox runs in the
HIP kernels of libbq.so; torch is used for device memory and streams.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L


class BQError(RuntimeError):
    """A negative status from the library."""

    def __init__(self, status: int, msg: str):
        super().__init__(f"bq status {status}: {msg}")
        self.status = status


@dataclass
class SolveInfo:
    status: int                 # library return value (0 or a positive warning)
    iters_fwd: list
    iters_adj: list
    status_fwd: list
    status_adj: list
    relres_fwd: list
    relres_adj: list
    green_apps: list


def _stats(arr, B, status) -> SolveInfo:
    return SolveInfo(status, [arr[i].iters_fwd for i in range(B)],
                     [arr[i].iters_adj for i in range(B)],
                     [arr[i].status_fwd for i in range(B)],
                     [arr[i].status_adj for i in range(B)],
                     [arr[i].relres_fwd for i in range(B)],
                     [arr[i].relres_adj for i in range(B)],
                     [arr[i].green_apps for i in range(B)])


def _ptr(t: torch.Tensor | None):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


class LSContext:
    """Green's operator, Lippmann-Schwinger solves and the mini-batch
    gradient for one grid and a set of illumination directions."""

    def __init__(self, N: int, h_um: float, lambda0_um: float, n_b: float,
                 directions, precision: str = "f32", model: str = "ls",
                 tol: float = 1e-5, max_iter: int = 300, plain: bool = False,
                 fused_xy: bool = False, stream: torch.cuda.Stream | None = None,
                 det_dist_um: float = 0.0, graphs: bool = False, cam_n: int = 0,
                 cam_pitch_um: float = 0.0):
        """graphs=True replays one captured BiCGSTAB iteration as a HIP graph
        instead of launching its kernels one by one (same results).
        cam_n > 0: detector images are taken by a cam_n x cam_n camera of
        pitch cam_pitch_um (um) centred on the axis."""
        self._lib = L.load()
        self.N = int(N)
        self.precision = precision
        self.rdtype = torch.float32 if precision == "f32" else torch.float64
        self.cdtype = torch.complex64 if precision == "f32" else torch.complex128
        self.device = torch.device("cuda", torch.cuda.current_device())
        d = np.ascontiguousarray(np.asarray(directions, dtype=np.float64).reshape(-1, 3))
        self.L = d.shape[0]
        g = L.Geom(self.N, float(h_um), float(lambda0_um), float(n_b),
                   L.BQ_F32 if precision == "f32" else L.BQ_F64,
                   L.BQ_MODEL_LS if model == "ls" else L.BQ_MODEL_BORN,
                   float(tol), int(max_iter),
                   (L.BQ_FLAG_PLAIN if plain else 0) | (L.BQ_FLAG_FUSED_XY if fused_xy else 0)
                   | (L.BQ_FLAG_GRAPH if graphs else 0),
                   float(det_dist_um), int(cam_n), float(cam_pitch_um))
        self.ndet = int(cam_n) if cam_n > 0 else self.N
        ill = (L.Illum * self.L)(*[L.Illum(*row) for row in d])
        self._stream = stream
        h = ct.c_void_p()
        s = self._lib.bq_create(ct.byref(g), ill, self.L, _stream_handle(stream), ct.byref(h))
        if s != L.BQ_OK:
            raise BQError(s, self._lib.bq_last_error(None).decode())
        self._h = h

    # ------------------------------------------------------------------
    def autotune(self, B: int) -> dict:
        """Choose the launch shapes of the FFT passes for batches of B by
        timing (bq_autotune); later calls compute the same values."""
        r = L.TuneResult()
        self._check(self._lib.bq_autotune(self._h, int(B), ct.byref(r)))
        return {"x_tile_rows": r.x_tile_rows, "zf_threads": r.zf_threads,
                "ms_default": r.ms_default, "ms_tuned": r.ms_tuned}

    def set_batch_limit(self, max_systems: int = 0):
        """Systems per launch set (0: as many as the free device memory
        holds); larger batches run as consecutive sub-batches."""
        self._check(self._lib.bq_set_batch_limit(self._h, int(max_systems)))

    def set_plan(self, x_tile_rows: int = 0, zf_threads: int = 0):
        """Set the launch shapes of the FFT passes directly (0 = default)."""
        self._check(self._lib.bq_set_plan(self._h, int(x_tile_rows), int(zf_threads)))

    def set_breakdown_floor(self, floor: float):
        """|rho|, |<rhat, A p>| or |omega| below floor stops a BiCGSTAB
        solve with status breakdown (default 1e-300)."""
        self._check(self._lib.bq_set_breakdown_floor(self._h, float(floor)))

    def info(self) -> dict:
        """Workspace capacity, launch shapes and graph-cache counters."""
        r = L.CtxInfo()
        self._check(self._lib.bq_get_info(self._h, ct.byref(r)))
        return {f: getattr(r, f) for f, _ in L.CtxInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s):
        if s < 0:
            raise BQError(s, self._lib.bq_last_error(self._h).decode())
        return s

    def _real(self, x: torch.Tensor, shape) -> torch.Tensor:
        if x.dtype != self.rdtype or x.device.type != "cuda" or tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected {self.rdtype} cuda tensor of shape {shape}")
        return x.contiguous()

    def _cplx(self, v: torch.Tensor, shape) -> torch.Tensor:
        if v.dtype != self.cdtype or v.device.type != "cuda" or tuple(v.shape) != tuple(shape):
            raise ValueError(f"expected {self.cdtype} cuda tensor of shape {shape}")
        return v.contiguous()

    def _out(self, out: torch.Tensor | None, shape) -> torch.Tensor:
        if out is None:
            return torch.empty(shape, dtype=self.rdtype, device=self.device)
        if (out.dtype != self.rdtype or out.device.type != "cuda" or tuple(out.shape) != tuple(shape)
                or not out.is_contiguous()):
            raise ValueError(f"out must be a contiguous {self.rdtype} cuda tensor of shape {shape}")
        return out

    @staticmethod
    def _idx(idx):
        a = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1))
        return a, a.ctypes.data_as(ct.POINTER(ct.c_int)), a.size

    # ------------------------------------------------------------------
    def forward(self, x: torch.Tensor, idx):
        N = self.N
        x = self._real(x, (N, N, N))
        a, pidx, B = self._idx(idx)
        D = self.ndet
        y = torch.empty((B, D, D), dtype=self.cdtype, device=x.device)
        st = (L.SolveStats * B)()
        s = self._check(self._lib.bq_forward(self._h, _ptr(x), pidx, B, _ptr(y), st))
        return y, _stats(st, B, s)

    def fields(self, x: torch.Tensor, idx):
        N = self.N
        x = self._real(x, (N, N, N))
        a, pidx, B = self._idx(idx)
        u = torch.empty((B, N, N, N), dtype=self.cdtype, device=x.device)
        st = (L.SolveStats * B)()
        s = self._check(self._lib.bq_fields(self._h, _ptr(x), pidx, B, _ptr(u), st))
        return u, _stats(st, B, s)

    def grad(self, x: torch.Tensor, y: torch.Tensor, idx, scale: float,
             out: torch.Tensor | None = None):
        N = self.N
        x = self._real(x, (N, N, N))
        a, pidx, B = self._idx(idx)
        y = self._cplx(y, (B, self.ndet, self.ndet))
        g = self._out(out, (N, N, N))
        loss = ct.c_double(0.0)
        st = (L.SolveStats * B)()
        s = self._check(self._lib.bq_grad(self._h, _ptr(x), _ptr(y), pidx, B, float(scale),
                                          _ptr(g), ct.byref(loss), st))
        return g, loss.value, _stats(st, B, s)

    def grad_ws(self, x: torch.Tensor, y: torch.Tensor, idx, scale: float, u: torch.Tensor,
                w: torch.Tensor, start: bool, out: torch.Tensor | None = None):
        """grad with the fields kept in u, w ((B, N, N, N) complex) and, when
        start is set, used as the starting points of the solves."""
        N = self.N
        x = self._real(x, (N, N, N))
        a, pidx, B = self._idx(idx)
        y = self._cplx(y, (B, self.ndet, self.ndet))
        for f in (u, w):
            if f.dtype != self.cdtype or tuple(f.shape) != (B, N, N, N) or not f.is_contiguous():
                raise ValueError("u, w must be contiguous (B, N, N, N) tensors of the context's complex type")
        g = self._out(out, (N, N, N))
        loss = ct.c_double(0.0)
        st = (L.SolveStats * B)()
        s = self._check(self._lib.bq_grad_ws(self._h, _ptr(x), _ptr(y), pidx, B, float(scale), _ptr(g),
                                             ct.byref(loss), st, _ptr(u), _ptr(w), int(bool(start))))
        return g, loss.value, _stats(st, B, s)

    def loss(self, x: torch.Tensor, y: torch.Tensor, idx, scale: float):
        N = self.N
        x = self._real(x, (N, N, N))
        a, pidx, B = self._idx(idx)
        y = self._cplx(y, (B, self.ndet, self.ndet))
        loss = ct.c_double(0.0)
        st = (L.SolveStats * B)()
        s = self._check(self._lib.bq_loss(self._h, _ptr(x), _ptr(y), pidx, B, float(scale),
                                          ct.byref(loss), st))
        return loss.value, _stats(st, B, s)

    def green(self, v: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
        N = self.N
        if v.dim() == 3:
            v = v.unsqueeze(0)
        B = v.shape[0]
        v = self._cplx(v, (B, N, N, N))
        out = torch.empty_like(v)
        self._check(self._lib.bq_green_apply(self._h, _ptr(v), _ptr(out), B, int(bool(adjoint))))
        return out


@dataclass
class ProxInfo:
    newton_total: int
    newton_max: int
    beta_last: float
    phi_last: float
    # BQ_OK, or BQ_NOTCONV when the root of some dual iteration was not
    # pinned down within the pass limit (the image is still returned)
    status: int = 0


class WProx:
    """Weighted proximal mapping of constrained TV on a fixed image shape."""

    def __init__(self, shape, precision: str = "f32", stream: torch.cuda.Stream | None = None):
        self._lib = L.load()
        self.shape = tuple(int(s) for s in shape)
        self.rdtype = torch.float32 if precision == "f32" else torch.float64
        h = ct.c_void_p()
        s = self._lib.bq_prox_create(*self.shape, L.BQ_F32 if precision == "f32" else L.BQ_F64,
                                     _stream_handle(stream), ct.byref(h))
        if s != L.BQ_OK:
            raise BQError(s, self._lib.bq_prox_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bq_prox_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __call__(self, v: torch.Tensor, tau: float, u: torch.Tensor | None, lam: float,
                 tv: str = "iso", cset: str = "nonneg", n_iter: int = 50,
                 P: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """u: None (metric tau I), an image (rank one), or the r columns of
        the metric factor as an (r,) + image-shape tensor."""
        for t in (v, u, P):
            if t is not None and (t.dtype != self.rdtype or t.device.type != "cuda"):
                raise ValueError(f"expected {self.rdtype} cuda tensors")
        if tuple(v.shape) != self.shape:
            raise ValueError("v has the wrong shape")
        if u is None:
            r = 0
        elif tuple(u.shape) == self.shape:
            r = 1
        elif u.dim() == 4 and tuple(u.shape[1:]) == self.shape:
            r = int(u.shape[0])
        else:
            raise ValueError("u must be an image or an (r,) + image-shape stack")
        if P is not None and (tuple(P.shape) != (3,) + self.shape or not P.is_contiguous()):
            raise ValueError("P must be a contiguous tensor of shape (3,) + image shape")
        if out is not None and (out.dtype != self.rdtype or out.device.type != "cuda"
                                or tuple(out.shape) != self.shape or not out.is_contiguous()):
            raise ValueError("out must be a contiguous cuda image of the workspace's type")
        v = v.contiguous()
        u = None if u is None or r == 0 else u.contiguous()
        x = torch.empty_like(v) if out is None else out
        st = L.ProxStats()
        s = self._lib.bq_wprox(self._h, _ptr(v), float(tau), _ptr(u), r, float(lam),
                               L.BQ_TV_ISO if tv == "iso" else L.BQ_TV_ANISO,
                               L.BQ_SET_NONNEG if cset == "nonneg" else L.BQ_SET_NONE,
                               int(n_iter), _ptr(x), _ptr(P), ct.byref(st))
        if s < 0:
            raise BQError(s, self._lib.bq_prox_last_error(self._h).decode())
        return x, ProxInfo(st.newton_total, st.newton_max, st.beta_last, st.phi_last, int(s))


def wprox_noalloc(v: torch.Tensor, tau: float, u: torch.Tensor | None, lam: float, tv: str = "iso",
                  cset: str = "nonneg", n_iter: int = 50, P: torch.Tensor | None = None,
                  out: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None):
    """bq_wprox_noalloc: the weighted prox without a workspace object (the
    library allocates nothing; its scratch is a static device array).  out
    must be given by callers that may not allocate either; u as for WProx."""
    lib = L.load()
    if v.dtype not in (torch.float32, torch.float64) or v.device.type != "cuda" or v.dim() != 3:
        raise ValueError("v must be a 3-D float32/float64 cuda tensor")
    shape = tuple(v.shape)
    for t in (u, P, out):
        if t is not None and (t.dtype != v.dtype or t.device != v.device or not t.is_contiguous()):
            raise ValueError("u, P, out must be contiguous tensors of v's type and device")
    if u is None:
        r = 0
    elif tuple(u.shape) == shape:
        r = 1
    elif u.dim() == 4 and tuple(u.shape[1:]) == shape:
        r = int(u.shape[0])
    else:
        raise ValueError("u must be an image or an (r,) + image-shape stack")
    if P is not None and tuple(P.shape) != (3,) + shape:
        raise ValueError("P must have shape (3,) + image shape")
    if out is not None and tuple(out.shape) != shape:
        raise ValueError("out has the wrong shape")
    v = v.contiguous()
    x = torch.empty_like(v) if out is None else out
    st = L.ProxStats()
    s = lib.bq_wprox_noalloc(*shape, L.BQ_F32 if v.dtype == torch.float32 else L.BQ_F64, _ptr(v), float(tau),
                             _ptr(u if r else None), r, float(lam),
                             L.BQ_TV_ISO if tv == "iso" else L.BQ_TV_ANISO,
                             L.BQ_SET_NONNEG if cset == "nonneg" else L.BQ_SET_NONE, int(n_iter), _ptr(x),
                             _ptr(P), ct.byref(st), _stream_handle(stream))
    if s < 0:
        raise BQError(s, lib.bq_prox_last_error(None).decode())
    return x, ProxInfo(st.newton_total, st.newton_max, st.beta_last, st.phi_last, int(s)), s


@dataclass
class QNInfo:
    k: int
    subset: int
    loss: float
    tau: float
    u_kept: bool
    metric_rank: int
    tau_sum: float
    prox_passes: int


class QNIteration:
    """Outer iteration of the mini-batch quasi-Newton proximal method
    (Algorithm 4.1, strategies I/II of Section 4.3, SR1 metrics of
    Algorithm 4.2) over an LSContext and a WProx of the same precision."""

    def __init__(self, ls: LSContext, px: WProx, subsets, a: float, lam: float, alpha: float,
                 gamma: float = 0.8, tau_max: float = 1e8, tv: str = "iso", cset: str = "nonneg",
                 prox_iters: int = 50, warm_start: bool = False, first_order: bool = False):
        self._lib = L.load()
        self._ls, self._px = ls, px   # kept alive while this object exists
        subsets = [list(map(int, s)) for s in subsets]
        self.S = len(subsets)
        flat = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.int32) for s in subsets]))
        lens = np.ascontiguousarray(np.array([len(s) for s in subsets], dtype=np.int32))
        prm = L.QnParams(self.S, float(a), float(lam), float(alpha), float(gamma), float(tau_max),
                         L.BQ_TV_ISO if tv == "iso" else L.BQ_TV_ANISO,
                         L.BQ_SET_NONNEG if cset == "nonneg" else L.BQ_SET_NONE, int(prox_iters),
                         int(bool(warm_start)), int(bool(first_order)))
        h = ct.c_void_p()
        s = self._lib.bq_qn_create(ls._h, px._h, ct.byref(prm), flat.ctypes.data_as(ct.POINTER(ct.c_int)),
                                   lens.ctypes.data_as(ct.POINTER(ct.c_int)), ct.byref(h))
        if s != L.BQ_OK:
            raise BQError(s, self._lib.bq_qn_last_error(None).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.bq_qn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, x: torch.Tensor, y: torch.Tensor, pick: int = -1) -> QNInfo:
        """x (N^3 real, updated in place: x_{k-1} -> x_k); y: measurements
        of all L illuminations, (L, N, N) complex; pick: -1 for strategy I,
        else the strategy-II draw in 0..S-1."""
        N = self._ls.N
        if x.dtype != self._ls.rdtype or tuple(x.shape) != (N, N, N) or not x.is_contiguous():
            raise ValueError("x must be a contiguous N^3 tensor of the context's real type")
        D = self._ls.ndet
        if y.dtype != self._ls.cdtype or tuple(y.shape) != (self._ls.L, D, D):
            raise ValueError("y must be (L, D, D) of the context's complex type (D: detector pixels per side)")
        y = y.contiguous()
        info = L.QnInfo()
        s = self._lib.bq_qn_step(self._h, _ptr(x), _ptr(y), int(pick), ct.byref(info))
        if s < 0:
            raise BQError(s, self._lib.bq_qn_last_error(self._h).decode())
        return QNInfo(info.k, info.subset, info.loss, info.tau, bool(info.u_kept), info.metric_rank,
                      info.tau_sum, info.prox_passes)
