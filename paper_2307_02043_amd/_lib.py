"""ctypes declarations of the bq C ABI (include/bq.h).

Loading fails loudly when libbq.so has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes as ct
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbq.so")

BQ_OK, BQ_EINVAL, BQ_ENOMEM, BQ_EDEVICE, BQ_EUNSUPPORTED = 0, -1, -2, -3, -4
BQ_NOTCONV, BQ_BREAKDOWN, BQ_NONFINITE = 1, 2, 3
BQ_F32, BQ_F64 = 0, 1
BQ_MODEL_LS, BQ_MODEL_BORN = 0, 1
BQ_FLAG_PLAIN = 1
BQ_FLAG_FUSED_XY = 2
BQ_FLAG_GRAPH = 4
BQ_TV_ISO, BQ_TV_ANISO = 0, 1
BQ_SET_NONE, BQ_SET_NONNEG = 0, 1
PASS_NAMES = ("zf", "xf", "yc", "xi", "zi", "xy", "vec")
BQ_TIMING_ALL = (1 << len(PASS_NAMES)) - 1
BQ_PROX_MAX_RANK = 8
BQ_WPROX_NOALLOC_SCRATCH = 96 << 20

EXPORTED = ("bq_create", "bq_destroy", "bq_last_error", "bq_forward", "bq_fields",
            "bq_grad", "bq_grad_ws", "bq_loss", "bq_green_apply", "bq_timing", "bq_timing_get", "bq_autotune", "bq_set_plan", "bq_set_batch_limit",
            "bq_set_breakdown_floor", "bq_get_info", "bq_audit_raw_ranges", "bq_prox_create", "bq_prox_destroy",
            "bq_prox_last_error", "bq_wprox", "bq_wprox_noalloc", "bq_qn_create", "bq_qn_destroy", "bq_qn_last_error",
            "bq_qn_step")


class Geom(ct.Structure):
    _fields_ = [("N", ct.c_int), ("h_um", ct.c_double), ("lambda0_um", ct.c_double),
                ("n_b", ct.c_double), ("precision", ct.c_int), ("model", ct.c_int),
                ("tol", ct.c_double), ("max_iter", ct.c_int), ("flags", ct.c_uint),
                ("det_dist_um", ct.c_double), ("cam_n", ct.c_int), ("cam_pitch_um", ct.c_double)]


class Illum(ct.Structure):
    _fields_ = [("dx", ct.c_double), ("dy", ct.c_double), ("dz", ct.c_double)]


class TuneResult(ct.Structure):
    _fields_ = [("x_tile_rows", ct.c_int), ("zf_threads", ct.c_int), ("ms_default", ct.c_double),
                ("ms_tuned", ct.c_double)]


class CtxInfo(ct.Structure):
    _fields_ = [("batch_capacity", ct.c_int), ("x_tile_rows", ct.c_int), ("zf_threads", ct.c_int),
                ("graphs_cached", ct.c_int), ("graph_captures", ct.c_longlong),
                ("breakdown_floor", ct.c_double)]


class SolveStats(ct.Structure):
    _fields_ = [("iters_fwd", ct.c_int), ("iters_adj", ct.c_int),
                ("status_fwd", ct.c_int), ("status_adj", ct.c_int),
                ("relres_fwd", ct.c_double), ("relres_adj", ct.c_double),
                ("green_apps", ct.c_int), ("pad_", ct.c_int)]


class ProxStats(ct.Structure):
    _fields_ = [("newton_total", ct.c_int), ("newton_max", ct.c_int),
                ("beta_last", ct.c_double), ("phi_last", ct.c_double)]


class QnParams(ct.Structure):
    _fields_ = [("S", ct.c_int), ("a", ct.c_double), ("lam", ct.c_double), ("alpha", ct.c_double),
                ("gamma", ct.c_double), ("tau_max", ct.c_double), ("tv", ct.c_int), ("cset", ct.c_int),
                ("prox_iters", ct.c_int), ("warm_start", ct.c_int), ("first_order", ct.c_int)]


class QnInfo(ct.Structure):
    _fields_ = [("k", ct.c_int), ("subset", ct.c_int), ("loss", ct.c_double), ("tau", ct.c_double),
                ("u_kept", ct.c_int), ("metric_rank", ct.c_int), ("tau_sum", ct.c_double),
                ("prox_passes", ct.c_int)]


_lib = None


def load() -> ct.CDLL:
    """Load libbq.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: the library then binds to the HIP runtime torch has
    # loaded, so that the process has one runtime whatever the import order
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ct.CDLL(LIB_PATH)
    P, I, D = ct.c_void_p, ct.c_int, ct.c_double
    sig = {
        "bq_create": ([ct.POINTER(Geom), ct.POINTER(Illum), I, P, ct.POINTER(P)], I),
        "bq_destroy": ([P], I),
        "bq_last_error": ([P], ct.c_char_p),
        "bq_forward": ([P, P, ct.POINTER(I), I, P, ct.POINTER(SolveStats)], I),
        "bq_fields": ([P, P, ct.POINTER(I), I, P, ct.POINTER(SolveStats)], I),
        "bq_grad": ([P, P, P, ct.POINTER(I), I, D, P, ct.POINTER(D), ct.POINTER(SolveStats)], I),
        "bq_grad_ws": ([P, P, P, ct.POINTER(I), I, D, P, ct.POINTER(D), ct.POINTER(SolveStats), P, P, I], I),
        "bq_loss": ([P, P, P, ct.POINTER(I), I, D, ct.POINTER(D), ct.POINTER(SolveStats)], I),
        "bq_green_apply": ([P, P, P, I, I], I),
        "bq_timing": ([P, I], I),
        "bq_timing_get": ([P, I, ct.POINTER(D), ct.POINTER(ct.c_longlong)], I),
        "bq_autotune": ([P, I, ct.POINTER(TuneResult)], I),
        "bq_set_plan": ([P, I, I], I),
        "bq_set_batch_limit": ([P, I], I),
        "bq_set_breakdown_floor": ([P, D], I),
        "bq_get_info": ([P, ct.POINTER(CtxInfo)], I),
        "bq_audit_raw_ranges": ([ct.c_char_p, I, ct.POINTER(ct.c_longlong)], I),
        "bq_prox_create": ([I, I, I, I, P, ct.POINTER(P)], I),
        "bq_prox_destroy": ([P], I),
        "bq_prox_last_error": ([P], ct.c_char_p),
        "bq_wprox": ([P, P, D, P, I, D, I, I, I, P, P, ct.POINTER(ProxStats)], I),
        "bq_wprox_noalloc": ([I, I, I, I, P, D, P, I, D, I, I, I, P, P, ct.POINTER(ProxStats), P], I),
        "bq_qn_create": ([P, P, ct.POINTER(QnParams), ct.POINTER(I), ct.POINTER(I), ct.POINTER(P)], I),
        "bq_qn_destroy": ([P], I),
        "bq_qn_last_error": ([P], ct.c_char_p),
        "bq_qn_step": ([P, P, P, I, ct.POINTER(QnInfo)], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib
