#!/usr/bin/env python
"""Benchmark of the mini-batch Lippmann-Schwinger gradient on one MI355X.

One step = one call of the library's batched mini-batch gradient
(forward solves, detector residual, adjoint solves, gradient reduction) over
one mini-batch of synthetic data, inputs already resident in HBM.

Default workload: 128^3 grid (256^3 padded), mini-batch of 16 out of 120
illuminations, complex64 fields with FP64 reductions, BiCGSTAB tol 1e-5.
The same inputs are also run through the plain path (FP64, one illumination
at a time, host round trip per iteration) and through the CPU oracle on a
bounded sample, and the JSON line reports the dominant kernel against the
HBM roofline.

Measurements: the phantom, illuminations and mini-batch come from the
seeded synthetic generators; the measured fields y are produced by the
library's own FP32 forward model on the phantom (tol 1e-6) plus 30 dB
noise.  They only set up a realistic residual for timing; no parity claim
rests on them.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LS gradient illum-solves/sec at 128^3 (batched FP32 vs plain FP64), % HBM peak"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes of one pass for one system and one application of G,
# in units of V = N^3 complex elements (x the complex element size).  The
# z passes depend on the prologue/epilogue; the figures are those of the
# solver matvecs, which are the bulk of the launches.  The transfer function
# is counted as one octant per system application (its symmetry leaves one
# independent octant of the padded grid); the batched launches read the full
# eight parity classes once per launch, which at a batch of 16 is 0.5 V per
# system.
PASS_UNITS = {
    "zf": 3.5,   # read v (1) + x (real, 0.5); write 2 parity classes (2)
    "xf": 6.0,   # read 2, write 4
    "yc": 9.0,   # read 4, write 4, transfer function 1
    "xi": 6.0,   # read 4, write 2
    "zi": 5.0,   # read 2 + v/s (1) + rhat or s (1); write 1
    "xy": 5.0,   # fused plane pass: read 2, write 2, transfer function 1
}
# Whole-call model: 28.5 V per application of G (the five passes above) and
# 13 V of vector work per BiCGSTAB iteration: s = r - alpha v (3), the x and r
# update (7), and the direction update p = r + beta (p - omega v) fused into
# the first z pass (3 V beyond a plain z pass: r, p, v read, p written).
G_UNITS = 28.5
ITER_VEC_UNITS = 13.0
# Non-packed FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x
# 2.4 GHz.  The code is built with packed FP32 disabled, so the 157.3
# TFLOP/s packed figure is not reachable by it.
FP32_VALU_PEAK_TFLOPS = 78.6
FP64_VALU_PEAK_TFLOPS = 78.6
# wave64 VALU instructions per second: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
VALU_ISSUE_PEAK_G = 256 * 4 * 2.4 / 4


def yc_flops_per_line(N):
    """Radix-2 flop convention (5 M log2 M per complex M-point FFT) for one
    padded y line of the convolution pass: forward FFT, transfer-function
    product (6 flops per point), inverse FFT, with M = 2N."""
    M = 2 * N
    return 2 * 5 * M * np.log2(M) + 6 * M


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_calibration(dev, mib):
    """A plain copy of a known size: one read and one write of `mib` MiB, run
    as an elementwise negation so that it is an ordinary kernel dispatch
    (not a DMA copy) whose HBM counters can be read like the solver's."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 x neg of {n * 4} bytes")
    del src, dst


TRAFFIC_FILES = (os.path.join(ROOT, "profiles", "ls_grad_128cubed_b16_f32_hbm_traffic.txt"),
                 os.path.join(ROOT, "profiles", "ls_grad_256cubed_b32_f32_hbm_traffic.txt"),
                 os.path.join(ROOT, "profiles", "ls_grad_96cubed_b8_f32_hbm_traffic.txt"))


# sources that define the z/y register kernels, their launch and their
# build flags (the kernels the traffic counters are reported for)
TRAFFIC_SOURCES = ("paper_2307_02043_amd/csrc/green_reg.hip", "paper_2307_02043_amd/csrc/bq_common.h",
                   "paper_2307_02043_amd/csrc/bq_state.h", "paper_2307_02043_amd/csrc/bq_kernels.h",
                   "paper_2307_02043_amd/build_lib.py")


def source_digest():
    """SHA-256 over the sources of the measured kernels, to tell whether
    they are still those the traffic counters were taken on."""
    import hashlib
    hs = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            hs.update(f.encode() + b"\0" + fh.read())
    return hs.hexdigest()


def measured_traffic(kernel, systems):
    """HBM bytes per launch of `kernel` with `systems` systems from the
    committed counter summaries (FETCH_SIZE and WRITE_SIZE per dispatch,
    each scaled by the ratio of the known size of a plain copy to what the
    same counter read for it), or None when no summary covers that kernel
    and batch or the sources have changed since."""
    for path in TRAFFIC_FILES:
        if not os.path.exists(path):
            continue
        kv = {}
        with open(path) as fh:
            for line in fh:
                if line.startswith("#") or not line.strip():
                    continue
                k, _, v = line.strip().partition(" ")
                kv.setdefault(k, v.strip())
        if (kv.get("csrc_sha256") != source_digest() or kv.get("kernel") != kernel
                or kv.get("systems_per_dispatch") != str(systems)):
            continue
        try:
            cb = float(kv["copy_bytes"])
            ff = cb / (float(kv["copy_fetch_kib"]) * 1024.0)
            fw = cb / (float(kv["copy_write_kib"]) * 1024.0)
            fetch = float(kv["fetch_kib_per_dispatch"]) * 1024.0 * ff
            write = float(kv["write_kib_per_dispatch"]) * 1024.0 * fw
        except (KeyError, ValueError, ZeroDivisionError):  # an incomplete summary reports no traffic
            return None
        return {"file": os.path.relpath(path, ROOT), "full_dispatch_bytes": round(fetch + write),
                "fetch_bytes": round(fetch), "write_bytes": round(write), "fetch_scale": round(ff, 4),
                "write_scale": round(fw, 4), "systems_per_dispatch": int(kv["systems_per_dispatch"]),
                "dispatches": int(kv.get("dispatches", 0))}
    return None


def measured_sq(kernel, systems):
    """SQ counters of a full dispatch of `kernel` (chip totals) from the
    summary that covers it, or None (no such section, or the sources have
    changed since)."""
    name = "bq::" + kernel.replace(",", ", ") + ":"
    for path in TRAFFIC_FILES:
        if not os.path.exists(path) or measured_traffic(kernel, systems) is None:
            continue
        with open(path) as fh:
            for line in fh:
                if line.startswith(name):
                    try:
                        return {k: float(v) for k, v in (it.split() for it in line[len(name):].split(","))}
                    except ValueError:  # not a counter line of the expected form
                        return None
    return None


def attach_traffic(roofline, systems):
    """The counter traffic of the dominant kernel, scaled to the timed
    launches like `achieved` (counters were taken on launches with every
    system active; system applications per launch)."""
    tr = measured_traffic(roofline["kernel"], systems)
    if tr is None:
        return
    apps, launches = roofline["system_applications"], roofline["launches"]
    per_app = tr["full_dispatch_bytes"] / tr["systems_per_dispatch"]
    per_launch = per_app * apps / launches
    roofline["traffic"] = round(per_launch)
    tr["measured_gbs"] = round(per_launch / (roofline["avg_launch_ms"] * 1e-3) / 1e9, 1)
    tr["vs_algorithmic"] = round(per_app / roofline["bytes_per_system_application"], 4)
    roofline["traffic_detail"] = tr
    sq = measured_sq(roofline["kernel"], systems)
    if sq and "SQ_INSTS_VALU" in sq:
        # wave64 VALU instructions of the counted dispatch, scaled to the timed
        # launches, against the issue rate of the SIMDs (one wave instruction
        # per 4 cycles on each of 1024 SIMDs at 2.4 GHz)
        per_launch_insts = sq["SQ_INSTS_VALU"] / tr["systems_per_dispatch"] * apps / launches
        rate = per_launch_insts / (roofline["avg_launch_ms"] * 1e-3) / 1e9
        roofline["valu_issue"] = {"instr_per_launch": round(per_launch_insts),
                                  "achieved": round(rate, 1), "peak": VALU_ISSUE_PEAK_G,
                                  "unit": "G wave-instructions/s", "frac": round(rate / VALU_ISSUE_PEAK_G, 4)}


def kernel_name(pas, N, prec):
    """The kernel that runs pass `pas` of G at grid N in precision prec
    (register kernels of padded lines up to 128, for the complex64 z and y
    passes at 96 and the complex64 y pass at 256, parity-split lines for
    the other 256 passes, LDS Stockham kernels for the other grids and
    passes)."""
    T = "float" if prec == "f32" else "double"
    if pas in ("xf", "xi", "xy"):
        return f"k_{pas}<{T},{N}>"
    if N in (16, 32, 64, 128):
        suf = "_p"
    elif N == 256:
        suf = "_p" if (pas == "yc" and prec == "f32") else "_r"
    elif N == 96 and prec == "f32":
        suf = "_p"
    else:
        suf = ""
    return f"k_{pas}{suf}<{T},{N}>"


def measure_gradient(w, dev, steps, warmup, autotune=True, prec=None, ctx_kw=None, label=None, event_free=False):
    """Time `steps` calls of the batched mini-batch gradient of workload w
    (after `warmup` untimed calls that also time every pass of G), inputs
    resident on the device.  Measurements from the library's own forward
    model (FP32, tol 1e-6; the Born model for a Born workload) plus noise.
    With event_free, the same number of steps is then timed again with no
    events at all (`no_events`).  Returns the figures of the timed steps and
    the context's last gradient (for cross-precision checks)."""
    import torch

    import synthetic as syn
    from paper_2307_02043_amd import LSContext
    from paper_2307_02043_amd import _lib as L

    prec = prec or w.precision
    N, B = w.N, w.B
    V = N ** 3
    xt = syn.scattering_potential(syn.make_phantom(w))
    dirs = syn.workload_directions(w)
    idx = syn.batch_indices(w)
    scale = 1.0 / B
    t = time.perf_counter()
    fwd = LSContext(N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", w.model, tol=1e-6, max_iter=w.max_iter)
    yc, _ = fwd.forward(torch.from_numpy(xt).to(dev, torch.float32), idx)
    fwd.close()
    y = syn.add_noise(yc.cpu().numpy(), w.snr_db, np.random.default_rng(w.seed("noise")))
    rd, cd = (torch.float32, torch.complex64) if prec == "f32" else (torch.float64, torch.complex128)
    t = time.perf_counter()
    ctx = LSContext(N, w.h_um, w.lambda0_um, w.n_b, dirs, prec, w.model, tol=w.tol, max_iter=w.max_iter,
                    **(ctx_kw or {}))
    setup_s = time.perf_counter() - t
    tune = None
    if autotune and w.model == "ls":
        t = time.perf_counter()
        tune = ctx.autotune(B)
        tune["s"] = round(time.perf_counter() - t, 2)
    lib = L.load()
    xe = torch.from_numpy(w.x_eval_scale * xt).to(dev, rd)
    yt = torch.from_numpy(y).to(dev, cd)

    def read_timers():
        ms_, n_ = {}, {}
        for pid, name in enumerate(L.PASS_NAMES):
            ms = L.ct.c_double()
            n = L.ct.c_longlong()
            lib.bq_timing_get(ctx._h, pid, L.ct.byref(ms), L.ct.byref(n))
            if n.value:
                ms_[name], n_[name] = ms.value, n.value
        return ms_, n_

    # Warmup steps time every pass (two HIP events per launch): per-pass
    # breakdown and the choice of the dominant pass.  The timed steps then
    # record events around the dominant pass only, which keeps the event
    # overhead out of the step time (all passes if there is no warmup).
    lib.bq_timing(ctx._h, L.BQ_TIMING_ALL)
    for i in range(warmup):
        _, loss, info = ctx.grad(xe, yt, idx, scale)
        log(f"{label or w.name} warmup {i}: loss {loss:.6e} iters fwd {info.iters_fwd} adj {info.iters_adj}")
    torch.cuda.synchronize()
    lib.bq_timing(ctx._h, 0)
    warm_ms, warm_n = read_timers()
    if warm_ms:
        dom = max((k for k in warm_ms if k in PASS_UNITS), key=lambda k: warm_ms[k])
        mask = 1 << L.PASS_NAMES.index(dom)
    else:
        dom, mask = None, L.BQ_TIMING_ALL
    lib.bq_timing(ctx._h, mask)
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        g, loss, info = ctx.grad(xe, yt, idx, scale)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lib.bq_timing(ctx._h, 0)
    log(f"{label or w.name} {prec}: {steps} steps in {elapsed:.3f} s")
    pass_ms, pass_n = read_timers()
    if dom is None:
        dom = max((k for k in pass_ms if k in PASS_UNITS), key=lambda k: pass_ms[k])
        warm_ms, breakdown_steps = pass_ms, steps
    else:
        breakdown_steps = warmup
    no_events = None
    if event_free:
        # the same number of steps with no events at all: for short steps the
        # two events around each launch of the dominant pass are a visible
        # share of the step
        t1 = time.perf_counter()
        for i in range(steps):
            ctx.grad(xe, yt, idx, scale)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t1
        no_events = {"value": round(B * steps / el1, 4), "ms_per_step": round(el1 / steps * 1e3, 3)}
    apps = sum(sum(inf.green_apps) for inf in infos)
    iters = sum(sum(inf.iters_fwd) + sum(inf.iters_adj) for inf in infos)
    csz = 8 if prec == "f32" else 16
    alg_bytes = apps * PASS_UNITS[dom] * V * csz
    achieved = alg_bytes / (pass_ms[dom] * 1e-3) / 1e9
    kname = kernel_name(dom, N, prec)
    avg_ms = pass_ms[dom] / pass_n[dom]
    roofline = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None,
                "bytes_per_system_application": PASS_UNITS[dom] * V * csz,
                "system_applications": apps, "launches": pass_n[dom],
                "avg_launch_ms": round(avg_ms, 4)}
    if dom == "yc":
        # the same launches against the vector-ALU roof (4 classes x N^2 lines per system)
        flops = apps * 4 * N * N * yc_flops_per_line(N)
        tf = flops / (pass_ms[dom] * 1e-3) / 1e12
        peak = FP32_VALU_PEAK_TFLOPS if prec == "f32" else FP64_VALU_PEAK_TFLOPS
        roofline["alu_view"] = {"achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
                                "frac": round(tf / peak, 4), "flops_per_line": yc_flops_per_line(N)}
    whole_bytes = (apps * G_UNITS + iters * ITER_VEC_UNITS) * V * csz
    whole = whole_bytes / elapsed / 1e9
    last = infos[-1]
    res = {
        "value": round(B * steps / elapsed, 4), "unit": "illum-solves/s",
        "ms_per_step": round(elapsed / steps * 1e3, 3), "steps": steps, "warmup": warmup,
        "roofline": roofline,
        "whole_call": {"scope": "whole gradient call, model bytes", "achieved": round(whole, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(whole / HBM_PEAK_GBS, 4),
                       "bytes_per_step": whole_bytes / steps},
        "solver": {"status": max(inf.status for inf in infos), "bicgstab_iters_per_step": iters / steps,
                   "green_apps_per_step": apps / steps, "bicgstab_iters_per_s": round(iters / elapsed, 1),
                   "iters_fwd": list(last.iters_fwd), "iters_adj": list(last.iters_adj),
                   "setup_s": round(setup_s, 2)},
        "passes_ms_per_step": {k: round(v / breakdown_steps, 3) for k, v in warm_ms.items()},
        "autotune": tune,
    }
    if no_events:
        res["no_events"] = no_events
    ctx.close()
    return res, g, (xt, y, dirs, idx)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4_ls128_f32")
    ap.add_argument("--plain-steps", type=int, default=5,
                    help="timed steps of the plain FP64 path, after one warmup step (0: skip)")
    ap.add_argument("--cpu-iters", type=int, default=10,
                    help="BiCGSTAB iterations of the oracle sample with all cores (0: skip)")
    ap.add_argument("--cpu-iters-1t", type=int, default=2,
                    help="BiCGSTAB iterations of the single-thread oracle sample (0: skip)")
    ap.add_argument("--configs", default="c1_ls32_f64,c2_born64_f32,c3_ls96_f32,c5_ls256_f32,c6_ls128_strong,"
                                         "c7_ls256_strong",
                    help="other workloads whose gradient is timed alongside ('' to skip)")
    ap.add_argument("--prox-workload", default="c5_ls256_f32",
                    help="workload whose weighted prox is timed alongside ('' to skip)")
    ap.add_argument("--prox-small", default="c1_ls32_f64,c2_born64_f32",
                    help="small workloads whose prox latency is timed ('' to skip)")
    ap.add_argument("--qn-iters", type=int, default=9,
                    help="outer iterations of the quasi-Newton method timed alongside (0: skip)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="choose the launch shapes of the FFT passes by timing before the timed "
                         "steps (bq_autotune; 0: default shapes)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of this many MiB (reference for the "
                         "HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only; --gpus must be 1 "
              "(the gradient would shard by illuminations with one all-reduce "
              "of the N^3 gradient, which is not built here).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synthetic as syn
    from paper_2307_02043_amd import LSContext

    w = syn.WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calibration > 0:
        copy_calibration(dev, args.copy_calibration)
    N, B = w.N, w.B
    V = N ** 3
    log(f"workload {w.name}: N={N} B={B} of L={w.L}")

    # ---- batched FP32 path (the headline) -----------------------------------
    head, g, (xt, y, dirs, idx) = measure_gradient(w, dev, args.steps, args.warmup, bool(args.autotune))
    scale = 1.0 / B
    roofline = head["roofline"]
    attach_traffic(roofline, B)
    value = head["value"]
    iters = head["solver"]["bicgstab_iters_per_step"] * args.steps

    # ---- plain FP64 path ----------------------------------------------------
    plain = None
    if args.plain_steps > 0:
        ctx64 = LSContext(N, w.h_um, w.lambda0_um, w.n_b, dirs, "f64", "ls", tol=w.tol,
                          max_iter=w.max_iter, plain=True)
        x64 = torch.from_numpy(w.x_eval_scale * xt).to(dev)
        y64 = torch.from_numpy(y).to(dev)
        ctx64.grad(x64, y64, idx, scale)  # warmup
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        pinfos = []
        for i in range(args.plain_steps):
            g64, loss64, pinfo = ctx64.grad(x64, y64, idx, scale)
            pinfos.append(pinfo)
        torch.cuda.synchronize()
        pel = time.perf_counter() - p0
        piters = sum(sum(p.iters_fwd) + sum(p.iters_adj) for p in pinfos)
        gerr = float(torch.linalg.norm(g.double() - g64) / torch.linalg.norm(g64))
        plain = {"value": round(B * args.plain_steps / pel, 3), "unit": "illum-solves/s",
                 "ms_per_step": round(pel / args.plain_steps * 1e3, 2), "steps": args.plain_steps,
                 "warmup": 1, "bicgstab_iters_per_s": round(piters / pel, 1),
                 "iters_per_step": piters / args.plain_steps,
                 "f32_vs_f64_grad_rel_diff": gerr}
        log(f"plain f64: {pel / args.plain_steps * 1e3:.2f} ms per step, grad rel diff f32 vs f64 {gerr:.2e}")
        ctx64.close()

    # ---- CPU oracle baseline --------------------------------------------------
    cpu = None
    if args.cpu_iters > 0:
        cpu = cpu_baseline(w, xt, dirs, idx, iters / (args.steps * B), args.cpu_iters, args.cpu_iters_1t)

    # ---- the other workloads ------------------------------------------------
    per_workload = {}
    for name in [c for c in args.configs.split(",") if c]:
        cw = syn.WORKLOADS[name]
        steps = 3 if cw.N >= 256 else 5 if cw.N >= 128 else 20
        r, _, _ = measure_gradient(cw, dev, steps, 1, bool(args.autotune), event_free=True)
        attach_traffic(r["roofline"], cw.B)
        r["workload"] = (f"{cw.name}: {'first-Born' if cw.model == 'born' else 'Lippmann-Schwinger'} "
                         f"mini-batch gradient, {cw.N}^3, batch {cw.B} of {cw.L}, "
                         f"{'complex64' if cw.precision == 'f32' else 'complex128'}, tol {cw.tol:g}, "
                         f"x = {cw.x_eval_scale:g} x_true")
        per_workload[name] = r
    if "c3_ls96_f32" in per_workload:
        # the 96^3 configuration names a persistent batched solver in a HIP graph
        per_workload["c3_ls96_f32"]["graph_replay"] = bench_graph_replay(syn.WORKLOADS["c3_ls96_f32"], dev)

    # ---- propagated detector plane (angular spectrum), same workload ---------
    det = bench_detprop(w, dev, xt, dirs, idx, scale, args.steps, head["ms_per_step"]) \
        if args.steps > 0 else None

    # ---- outer iteration of the method on the same workload -----------------
    qn = None
    if args.qn_iters > 0:
        qn = bench_qn(w, dev, xt, dirs, args.qn_iters, head["ms_per_step"], plan=head["autotune"])

    # ---- weighted TV prox (second kernel of the method) ---------------------
    prox = None
    if args.prox_workload:
        prox = bench_prox(syn.WORKLOADS[args.prox_workload], dev)
    prox_small = {}
    for name in [c for c in args.prox_small.split(",") if c]:
        prox_small[name] = bench_prox_latency(syn.WORKLOADS[name], dev)

    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "illum-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"{w.name}: Lippmann-Schwinger mini-batch gradient, {N}^3 grid "
                                f"({2 * N}^3 padded), batch {B} of {w.L} illuminations, complex64 "
                                f"fields, FP64 reductions, BiCGSTAB tol {w.tol:g}"),
                   "grid": N, "batch": B, "illuminations": w.L, "tol": w.tol},
        "roofline": roofline,
        "whole_call": head["whole_call"],
        "cpu_baseline": cpu,
        "plain_f64": plain,
        "speedup_vs_plain_f64": (round(value / plain["value"], 2) if plain else None),
        "solver": head["solver"],
        "passes_ms_per_step": head["passes_ms_per_step"],
        "autotune": head["autotune"],
        "configs": per_workload,
        "prox": prox,
        "prox_latency": prox_small,
        "qn": qn,
        "detector_propagation": det,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline(w, xt, dirs, idx, mean_iters, iters_all, iters_1t):
    """The oracle (never tuned) on the host cores: FP64 BiCGSTAB iterations
    of one illumination of the workload, with scipy.fft on all cores (at
    most 16) and, sharing its transfer function, on one thread; each
    extrapolated to an illumination's forward and adjoint solves at the
    GPU-observed iteration count plus the 3 extra applications of G."""
    from oracle import lsmodel
    cores = min(os.cpu_count() or 1, 16)
    geom = lsmodel.Geometry(N=w.N, h=w.h_um, lambda0=w.lambda0_um, n_b=w.n_b)
    t = time.perf_counter()
    model = lsmodel.LSModel(geom, workers=cores)
    log(f"oracle transfer function ({time.perf_counter() - t:.1f} s)")
    xe64 = w.x_eval_scale * xt
    uin = lsmodel.incident_field(geom, dirs[idx[0]])
    extra = 3  # initial residuals of both solves + adjoint right-hand side

    def timed(m, n):
        t0 = time.perf_counter()
        m.solve_forward(xe64, uin, 0.0, n)  # tol 0: runs the cap
        t_iter = (time.perf_counter() - t0) / n
        return t_iter, 1.0 / (t_iter * mean_iters + extra * t_iter / 2)

    t_iter, val = timed(model, iters_all)
    out = {"value": round(val, 5), "unit": "illum-solves/s", "cores": cores, "kind": "oracle",
           "sample": (f"one illumination of this workload: the oracle's FP64 BiCGSTAB run for "
                      f"{iters_all} iterations ({t_iter:.2f} s each, scipy.fft with {cores} workers), "
                      f"extrapolated to the GPU-observed {mean_iters:.1f} iterations per illumination "
                      f"(forward + adjoint) plus 3 extra applications of G")}
    log(f"oracle: {t_iter:.2f} s per BiCGSTAB iteration on {cores} cores")
    if iters_1t > 0:
        one = lsmodel.LSModel(geom, ghat_P=model.ghat, workers=1)
        t1, val1 = timed(one, iters_1t)
        out["single_thread"] = {"value": round(val1, 5), "unit": "illum-solves/s", "cores": 1,
                                "s_per_bicgstab_iter": round(t1, 3),
                                "sample": f"{iters_1t} iterations of the same solve, scipy.fft on one thread"}
        log(f"oracle: {t1:.2f} s per BiCGSTAB iteration on one thread")
    return out


def bench_detprop(w, dev, xt, dirs, idx, scale, steps, base_ms, d_um=1.0, cam_n=512):
    """The batched FP32 gradient of the workload with the detector plane
    d_um beyond the exit plane (angular-spectrum propagation before the
    residual and its adjoint before the adjoint right-hand side), and the
    same with a cam_n x cam_n camera sampling that plane over the window
    (pitch N h / cam_n, as a 512^2 camera over the paper's field of view)."""
    import torch

    from paper_2307_02043_amd import LSContext

    out = {"det_dist_um": d_um, "exit_plane_ms_per_step": round(base_ms, 3)}
    pitch = w.N * w.h_um / cam_n
    for key, cam in (("ms_per_step", {}), ("camera", {"cam_n": cam_n, "cam_pitch_um": pitch})):
        ctx = LSContext(w.N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", "ls", tol=1e-6, max_iter=w.max_iter,
                        det_dist_um=d_um, **cam)
        xtt = torch.from_numpy(xt).to(dev, torch.float32)
        y = ctx.forward(xtt, idx)[0]
        ctx.close()
        ctx = LSContext(w.N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", "ls", tol=w.tol, max_iter=w.max_iter,
                        det_dist_um=d_um, **cam)
        x = (w.x_eval_scale * xtt).contiguous()
        ctx.grad(x, y, idx, scale)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            ctx.grad(x, y, idx, scale)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) / steps * 1e3
        ctx.close()
        if cam:
            out["camera"] = {"pixels": cam_n, "pitch_um": round(pitch, 6), "ms_per_step": round(ms, 3)}
            log(f"camera {cam_n}^2 (pitch {pitch:.4f} um) on that plane: {ms:.2f} ms per gradient step")
        else:
            out["ms_per_step"] = round(ms, 3)
            log(f"detector plane {d_um} um beyond the exit plane: {ms:.2f} ms per gradient step")
    return out


def bench_graph_replay(w, dev, steps=20):
    """The workload's batched gradient with the BiCGSTAB iteration replayed
    as a captured HIP graph (BQ_FLAG_GRAPH) against the same context
    launching its kernels one by one, both without per-pass events (a
    timed pass turns replay off).  Same inputs as the configs section."""
    import torch

    import synthetic as syn
    from paper_2307_02043_amd import LSContext

    xt = syn.scattering_potential(syn.make_phantom(w))
    dirs = syn.workload_directions(w)
    idx = syn.batch_indices(w)
    fwd = LSContext(w.N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", w.model, tol=1e-6, max_iter=w.max_iter)
    yc, _ = fwd.forward(torch.from_numpy(xt).to(dev, torch.float32), idx)
    fwd.close()
    y = syn.add_noise(yc.cpu().numpy(), w.snr_db, np.random.default_rng(w.seed("noise")))
    rd, cd = (torch.float32, torch.complex64) if w.precision == "f32" else (torch.float64, torch.complex128)
    xe = torch.from_numpy(w.x_eval_scale * xt).to(dev, rd)
    yt = torch.from_numpy(y).to(dev, cd)
    out = {}
    for key, graphs in (("eager_ms_per_step", False), ("graph_ms_per_step", True)):
        ctx = LSContext(w.N, w.h_um, w.lambda0_um, w.n_b, dirs, w.precision, w.model, tol=w.tol,
                        max_iter=w.max_iter, graphs=graphs)
        ctx.autotune(w.B)
        for _ in range(2):
            g, loss, info = ctx.grad(xe, yt, idx, 1.0 / w.B)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            g, loss, info = ctx.grad(xe, yt, idx, 1.0 / w.B)
        torch.cuda.synchronize()
        out[key] = round((time.perf_counter() - t) / steps * 1e3, 3)
        if graphs:
            out["graph_captures"] = ctx.info()["graph_captures"]
            out["same_loss_bits"] = bool(loss == out["loss"])
        else:
            out["loss"] = loss
        ctx.close()
    log(f"{w.name} graph replay: {out['graph_ms_per_step']:.3f} ms per step against "
        f"{out['eager_ms_per_step']:.3f} ms launching each kernel")
    return out


def bench_qn(w, dev, xt, dirs, iters, grad_ms, S=4, plan=None):
    """Outer iterations of Algorithm 4.1 (strategy I) on the workload's grid:
    S subsets of B illuminations (the first S B directions), x_0 = 0.5
    x_true, step 1/20, 50 dual iterations per WPM, FP32; four variants:
    SR1 metrics of Algorithm 4.2 (gamma 0.8, tau_max 1e8) with cold solves,
    the same with warm-started solves, and the first-order (alpha I)
    variant with warm-started solves, and SR1 with tau_max below the
    curvature scale (rank-one corrections kept, WPM metrics of rank up to
    S).  Measurements from the library's FP32
    forward model (tol 1e-6) without noise.  The LS context takes `plan`,
    the launch shapes tuned for the gradient workload, when given."""
    import torch

    from paper_2307_02043_amd import LSContext, QNIteration, WProx

    N, B = w.N, w.B
    subsets = [list(range(s * B, (s + 1) * B)) for s in range(S)]
    ls = LSContext(N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", "ls", tol=1e-6, max_iter=w.max_iter)
    xtt = torch.from_numpy(xt).to(dev, torch.float32)
    y = torch.zeros((w.L, N, N), dtype=torch.complex64, device=dev)
    for sub in subsets:
        y[sub] = ls.forward(xtt, sub)[0]
    ls.close()
    ls = LSContext(N, w.h_um, w.lambda0_um, w.n_b, dirs, "f32", "ls", tol=w.tol, max_iter=w.max_iter)
    if plan:  # the launch shapes tuned for the gradient workload (same grid, batch and precision)
        ls.set_plan(plan["x_tile_rows"], plan["zf_threads"])
    x = (0.5 * xtt).contiguous()
    g0, _, _ = ls.grad(x, y[subsets[0]], subsets[0], S / w.L)
    alpha = float(g0.abs().max()) / float(xtt.max())
    lam = 1.0 / N ** 3
    px = WProx((N, N, N), "f32")
    variants = {}
    # sr1_clipped: tau_max = 2 alpha, below the curvature ratio <m,m>/(gamma <s,m>) of this
    # problem, so Algorithm 4.2 keeps rank-one corrections and the WPM runs metrics of rank
    # up to S (with tau_max = 1e8 and gamma < 1 it keeps none)
    for name, warm, fo, tmax in (("sr1", False, False, 1e8), ("sr1_warm", True, False, 1e8),
                                 ("first_order_warm", True, True, 1e8), ("sr1_clipped", True, False, 2 * alpha)):
        qn = QNIteration(ls, px, subsets, 1.0 / 20, lam, alpha, 0.8, tmax, prox_iters=50, warm_start=warm,
                         first_order=fo)
        xk = x.clone()
        torch.cuda.synchronize()
        times, infos = [], []
        for _ in range(iters):
            t = time.perf_counter()
            infos.append(qn.step(xk, y))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t)
        qn.close()
        # the gradient alone at the last iterate (cold solves, first subset):
        # what the outer iteration's gradient costs there, against the
        # benchmark's gradient at 0.5 x_true
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, ginfo = ls.grad(xk, y[subsets[0]], subsets[0], S / w.L)
        torch.cuda.synchronize()
        grad_at_iterate_ms = (time.perf_counter() - t) * 1e3
        later = [t for t, inf in zip(times, infos) if inf.k > S]
        variants[name] = {"tau_max": tmax, "ms_per_iter": round(float(np.mean(times)) * 1e3, 2),
                          "ms_per_iter_after_S": round(float(np.mean(later)) * 1e3, 2) if later else None,
                          "loss_first_last": [infos[0].loss, infos[-1].loss],
                          "u_kept": sum(int(i.u_kept) for i in infos),
                          "metric_rank_max": max(int(i.metric_rank) for i in infos),
                          "gradient_ms_at_last_iterate": round(grad_at_iterate_ms, 2),
                          "bicgstab_iters_at_last_iterate": int(sum(ginfo.iters_fwd) + sum(ginfo.iters_adj))}
        log(f"qn {name}: {iters} outer iterations, {np.mean(times) * 1e3:.1f} ms each")
    # the rank-S WPM alone (same shape, metric rank, weight and iterations)
    U = 0.1 * torch.randn((S, N, N, N), dtype=torch.float32, device=dev)
    px(x, 1.0, U, lam, "iso", "nonneg", 50)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, pinfo = px(x, 1.0, U, lam, "iso", "nonneg", 50)
    torch.cuda.synchronize()
    prox_ms = (time.perf_counter() - t) * 1e3
    px.close()
    ls.close()
    log(f"qn: rank-{S} WPM alone {prox_ms:.1f} ms")
    return {"workload": (f"{w.name} outer iteration: {N}^3, S = {S} subsets of {B} illuminations, "
                         f"strategy I, 50 dual iterations per WPM, FP32"),
            "iterations": iters,
            "variants": variants,
            "gradient_ms_same_batch": round(grad_ms, 2),
            "rank_S_wprox_ms": round(prox_ms, 2),
            "rank_S_wprox_root_evaluations_max": int(pinfo.newton_max),
            "rank_S_wprox_status": int(pinfo.status)}


def bench_prox(w, dev, reps=2):
    """One weighted prox of a workload (its TV kind, metric tau I + u u^T,
    lambda and iteration count), FP32, inputs resident on the device.

    Algorithmic HBM bytes per dual iteration, in V = N^3 FP32 images: the
    divergence pass reads R (3), v, u and writes a (6); each root-finding
    pass reads a, u (2); the dual update reads a, u, R (3), P (3) and writes
    P, R (6) (14).  Total 20 + 2 n_pass per iteration.

    The same image, weight and iteration count under the metric tau I (no
    u) are timed as well: one fused kernel per dual iteration reading v,
    R (3), P (3) and writing P, R (6), 13 per iteration, plus 14 per call
    (starting point 3, its copy 6, output 5).
    """
    import torch

    import synthetic as syn
    from paper_2307_02043_amd import WProx

    v, tau, u = syn.prox_inputs(w)
    V = v.size
    vt = torch.from_numpy(v).to(dev, torch.float32)
    ut = torch.from_numpy(u).to(dev, torch.float32)
    px = WProx(v.shape, "f32")
    x, info = px(vt, tau, ut, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)  # warmup
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        x, info = px(vt, tau, ut, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / reps
    K = w.prox_iters
    extra_passes = info.newton_total - (K + 1)   # evaluations beyond the fused one
    units = 20.0 * K + 2.0 * extra_passes + 6.0 + 1.0  # + final divergence and output
    achieved = units * V * 4 / el / 1e9
    x, _ = px(vt, tau, None, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)  # metric tau I: warmup
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        x, _ = px(vt, tau, None, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)
    torch.cuda.synchronize()
    el0 = (time.perf_counter() - t) / reps
    units0 = 13.0 * K + 14.0
    achieved0 = units0 * V * 4 / el0 / 1e9
    px.close()
    log(f"prox {w.name}: {el * 1e3:.2f} ms per call, {info.newton_total} root evaluations; "
        f"metric tau I {el0 * 1e3:.2f} ms")
    return {"workload": (f"{w.name} prox: {w.N}^3 {w.prox_tv}-TV, nonnegativity, metric tau I + u u^T, "
                         f"lambda {w.prox_lambda:g}, {K} dual iterations, FP32"),
            "ms_per_call": round(el * 1e3, 3), "dual_iters_per_s": round(K / el, 1),
            "root_evaluations": info.newton_total, "max_evaluations_per_iter": info.newton_max,
            "roofline": {"bound": "hbm", "scope": "whole call", "achieved": round(achieved, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "bytes": units * V * 4},
            "tau_metric": {"ms_per_call": round(el0 * 1e3, 3), "dual_iters_per_s": round(K / el0, 1),
                           "roofline": {"bound": "hbm", "scope": "whole call", "achieved": round(achieved0, 1),
                                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                        "frac": round(achieved0 / HBM_PEAK_GBS, 4), "bytes": units0 * V * 4}}}


def bench_prox_latency(w, dev, reps=5):
    """Latency of one weighted prox of a small workload (its TV kind,
    precision, metric tau I + u u^T, lambda, iteration count): images that
    stay in the last-level cache, where the launch sequence, not HBM,
    sets the time."""
    import torch

    import synthetic as syn
    from paper_2307_02043_amd import WProx

    v, tau, u = syn.prox_inputs(w)
    dt = torch.float32 if w.precision == "f32" else torch.float64
    vt = torch.from_numpy(v).to(dev, dt)
    ut = torch.from_numpy(u).to(dev, dt)
    px = WProx(v.shape, w.precision)
    x, info = px(vt, tau, ut, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)  # warmup
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        x, info = px(vt, tau, ut, w.prox_lambda, w.prox_tv, "nonneg", w.prox_iters)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / reps
    px.close()
    log(f"prox latency {w.name}: {el * 1e3:.2f} ms per call of {w.prox_iters} dual iterations")
    return {"workload": (f"{w.name} prox: {w.N}^3 {w.prox_tv}-TV, nonnegativity, metric tau I + u u^T, "
                         f"lambda {w.prox_lambda:g}, {w.prox_iters} dual iterations, "
                         f"{'FP32' if w.precision == 'f32' else 'FP64'}"),
            "ms_per_call": round(el * 1e3, 3), "us_per_dual_iter": round(el / w.prox_iters * 1e6, 2),
            "root_evaluations": info.newton_total}


if __name__ == "__main__":
    main()
