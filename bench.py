#!/usr/bin/env python3
"""Benchmark of the SG-WLS hot path on one MI355X.

Workload: one 1080x1920 RGB float32 image (synthetic: 200 random rectangles,
a sinusoidal gradient and Gaussian noise, seed 1000), luma guidance, r = 1,
T = 3 iterations (6 passes), stride 1, lambda = 4, omega^exp with
sigma_s = 1, sigma_r = 0.1.  One step = one full filter call (all 2T passes,
all channels) with the inputs resident in HBM.

Prints ONE JSON line:
  value      MPixel/s = M*N / (time of one filter call)
  roofline   the dominant kernel's algorithmic bytes per launch / its mean
             duration (HIP events around launches of that kernel alone), vs
             the 8 TB/s HBM peak
  cpu_baseline  the FP64 oracle on the host cores, same workload
  fwd_bwd    one forward call that saves the pass inputs (and every pass's
             separator solutions) plus the backward call (gradients for f, g
             and lambda) for a fixed output gradient, as MPixel/s and
             algorithmic bytes / time vs 8 TB/s; also the same pair without
             saved separators
  fp64_pivot the same forward call with float64 pivots and recurrences
  fp32_delta the same forward call in the cancellation-free float32 mode
             (one serial solve per strip, pivots carried as their excess)
  batched    64 grey images with sides in [256, 2048], r in {1, 2}, lambda in
             [0.5, 32], T = 3, in one batched call (hipGraph replay on a side
             stream, autotuned variant), against a loop of single-image calls
  cold       single calls after a 512 MiB scratch write (Infinity Cache evicted)
  fused_passes  the same call with fused passes (one launch per pass, or two)
             against the default three launches per pass
  stride3    the same workload with stride 3 (centres 2r+1 apart, no overlap)
  stride_sweep  1024x1024 RGB, T = 4: filter time at (r, stride) = (1, 1),
             (1, 3), (2, 1), (2, 5), (4, 1), (4, 4), (4, 9), each autotuned
  ctx        1024x1024 RGB, r = 1, T = 4 (the paper's timing image size)
  wls2d      the 2D WLS model SG-WLS approximates (Eqs. 1-4) on the same
             input, solved by GPU conjugate gradients: time and the SG-WLS gap
  interpolation  guided sparse interpolation (Eq. 21): 8x depth upsampling of
             a 1080x1920 depth map (r = 4, stride 4, lambda 400) and scribble
             colourisation at 1024x1024 (r = 4, stride 2, lambda 900)
  traffic    (in roofline) HBM bytes per k_expand_d launch from the committed
             rocprofv3 counter summary, null when it was taken on other sources
  radius     the same image at r = 2 and r = 3 (T = 3, lambda = 16): FP32 and
             FP64-pivot time, algorithmic bytes / time vs 8 TB/s, and the
             VALU-busy fraction of each stage from the committed counter
             summary (null when it was taken on other sources); these radii
             carry several times the arithmetic per byte of r = 1
  configs    the other workloads: grey 256x256 (r = 1, T = 1, lambda 1), RGB
             768x1024 (r = 1, T = 3, lambda 4) forward, and 16 RGB 512x512
             images (r = 1, T = 3, learnable lambda = 8, MSE loss) forward +
             backward through the autograd function; MPixel/s and algorithmic
             bytes / time vs 8 TB/s each
The default precision is automatic (float32 where the host bound on
lambda * omega allows it; FP64 pivots for calls that save pass inputs for a
lambda gradient): fwd_bwd is that default, fwd_bwd_fp32 the same step in
explicit float32.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3)
    ap.add_argument("--stride", type=int, default=1)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="only the stride / radius sweep: 1024x1024 RGB, T=4, r = 1..4, "
                         "stride 1..2r+1; one JSON line")
    ap.add_argument("--fused", action="store_true",
                    help="only the fused-pass comparison on the 1080p RGB workload (tuned "
                         "variants): one JSON line")
    ap.add_argument("--counters", choices=("fwd", "fwdbwd", "radius"), default=None,
                    help="for rocprofv3 --pmc runs: the tuned forward (or forward + backward) "
                         "steps only, then three copies of 64 MiB (the counter calibration), "
                         "one short JSON line; 'radius': three tuned forward calls at each of "
                         "r = 1, 2, 3 on the 1080p RGB image (for the VALU-busy counter)")
    return ap.parse_args()


def sources_digest():
    """SHA-256 over the sources the single-image kernels are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_01674_amd", "csrc")
    for name in ("sgwls_device.hpp", "sgwls_internal.hpp", "sgwls_pass_r1.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_expand_d_rgb1080p_r1_T3_counters.md")


def frame_variants(tuned):
    """The tuned kernel variant of each channel-block width: every pass of a
    stride-1 filter call is a column pass of a frame (the image or its
    transpose) and runs the column-direction variant."""
    return {f"c{cb}": v for (d, cb), v in sorted(tuned.items()) if d == 0}


def counted_traffic(tuned):
    """HBM bytes per k_expand_d launch (mean of the column and row frame) from
    the committed counter summary, or None when it is missing, was taken on
    other kernel sources, or lacks the tuned variants."""
    try:
        with open(COUNTERS_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    tag = "traffic-json:"
    if tag not in text:
        return None
    data = json.loads(text.split(tag, 1)[1].split("-->", 1)[0])
    if data.get("source_sha256") != sources_digest():
        return None
    per = data.get("bytes_per_launch", {})
    # Every pass of the filter is a column pass of a frame (the image or its
    # transpose), both run with the column-direction variant.
    v = per.get(str(tuned.get((0, 3))))
    if not v or "col" not in v or "row" not in v:
        return None
    return round((v["col"] + v["row"]) / 2)


VALU_FILE = os.path.join(ROOT, "profiles", "valu_rgb1080p_r1_r2_r3_T3.md")


def radius_digest():
    """SHA-256 over the sources the kernels at r = 1, 2, 3 are built from."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_01674_amd", "csrc")
    for name in ("sgwls_device.hpp", "sgwls_internal.hpp", "sgwls_pass_r1.hip",
                 "sgwls_pass_r2.hip", "sgwls_pass_r3.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counted_valu(r):
    """Per-stage VALU-busy fraction at radius r from the committed counter
    summary (with the variants it was counted at), or None when the summary
    is missing or was taken on other kernel sources."""
    try:
        with open(VALU_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    tag = "valu-json:"
    if tag not in text:
        return None
    data = json.loads(text.split(tag, 1)[1].split("-->", 1)[0])
    if data.get("source_sha256") != radius_digest():
        return None
    return data.get("rows", {}).get(str(r))


def radius_rows(torch, ops, nat, synth, dev, args, counters=False):
    """The metric image at r = 2 and r = 3 (T = 3, lambda = 16; the FP32
    path's cost does not depend on lambda): per call FP32 and FP64-pivot time
    and the algorithmic bytes / time.  With counters, only three tuned forward
    calls at each of r = 1, 2, 3 (the dispatches a VALU-busy pass reads)."""
    rows = []
    for r in ((1, 2, 3) if counters else (2, 3)):
        w = synth.rgb1080p(r=r, lam=16.0)
        C, M, N = w.f.shape
        p = ops.Params(**w.params, prec="fp32")
        f = torch.from_numpy(w.f).to(dev)
        g = torch.from_numpy(w.g).to(dev)
        u = torch.empty_like(f)
        ws = torch.empty(ops.workspace_bytes(C, M, N, p), dtype=torch.uint8, device=dev)
        tuned = ops.autotune(f, g, p, reps=10)
        variants = frame_variants(tuned)

        def step():
            ops.sgwls_filter(f, g, p, out=u, workspace=ws)

        if counters:
            for _ in range(3):
                step()
            torch.cuda.synchronize()
            rows.append({"r": r, "variants": variants})
            continue
        for _ in range(args.warmup):
            step()
        ms = time_events(torch, step, max(5, args.steps // 2))
        p64 = p.with_(prec="fp64_pivot")
        ws64 = torch.empty(ops.workspace_bytes(C, M, N, p64), dtype=torch.uint8, device=dev)

        def step64():
            ops.sgwls_filter(f, g, p64, out=u, workspace=ws64)

        for _ in range(args.warmup):
            step64()
        ms64 = time_events(torch, step64, max(5, args.steps // 5))
        alg = (8 * C + 4) * M * N * 2 * p.iters
        _, st, _ = stage_times(torch, nat, f, g, p, ws, max(10, args.steps // 5))
        rows.append({"workload": w.name, "r": r, "iters": p.iters, "lambda": p.lam, "prec": "fp32",
                     "default_precision": ops.resolve_precision(ops.Params(**w.params)),
                     "ms_per_step": round(ms, 5), "value": round(M * N / (ms * 1e-3) / 1e6, 2),
                     "unit": "MPixel/s", "alg_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "fp64_pivot_ms": round(ms64, 5), "variants": variants,
                     "kernels_ms_per_launch": {f"{'col' if d == 0 else 'row'}:{n}": round(t, 5)
                                               for (d, n), t in st.items()},
                     "valu_busy": counted_valu(r)})
    return rows


def stage_times(torch, nat, f, g, p, ws, steps):
    """Per-kernel timing: each stage of each pass launched alone on the current
    stream, between HIP events, exactly as the filter launches it.  When the
    filter runs every pass as a column pass (of the image, then of its
    transpose, storing transposed), so does this timing.  Returns whether it
    does, the mean ms per launch of each (frame, stage) and each stage's ms
    per filter call."""
    import ctypes
    C, M, N = f.shape
    cp = p.c()
    stream = ctypes.c_void_p(torch.cuda.current_stream(f.device).cuda_stream)
    y = torch.empty_like(f)

    def stages_call(mask, direction, xx, gg, yy, MM, NN):
        return nat.lib.sgwls_pass_stages(mask, direction, ctypes.c_void_p(xx.data_ptr()),
                                         ctypes.c_void_p(gg.data_ptr()), ctypes.c_void_p(yy.data_ptr()),
                                         C, MM, NN, ctypes.byref(cp), None,
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream)

    transposed = stages_call(7 | 8, 0, f, g, y, M, N) == 0
    if transposed:
        fT = f.transpose(1, 2).contiguous()
        gT = g.t().contiguous()
        frames = [(0, f, g, M, N, 8), (0, fT, gT, N, M, 8)]
    else:
        frames = [(0, f, g, M, N, 0), (1, f, g, M, N, 0)]
    stage_names = {1: "k_reduce", 2: "k_interface", 4: "k_expand"}
    per_filter_ms = {}
    stage_ms = {}
    for direction, (dflag, xx, gg, MM, NN, extra) in enumerate(frames):
        yy = torch.empty_like(xx)

        def run(mask):
            nat.check(stages_call(mask | extra, dflag, xx, gg, yy, MM, NN), "sgwls_pass_stages")
        run(7)
        for mask, name in stage_names.items():
            for _ in range(3):
                run(mask)
            t = time_events(torch, lambda: run(mask), max(10, steps))
            stage_ms[(direction, name)] = t
            per_filter_ms[name] = per_filter_ms.get(name, 0.0) + t * p.iters
    return transposed, stage_ms, per_filter_ms


def time_workload(torch, ops, w, dev, steps, warmup):
    """Mean ms of one filter call on workload w (autotuned, inputs resident)."""
    C, M, N = w.f.shape
    p = ops.Params(**w.params)
    f = torch.from_numpy(w.f).to(dev)
    g = torch.from_numpy(w.g).to(dev)
    u = torch.empty_like(f)
    ws = torch.empty(ops.workspace_bytes(C, M, N, p), dtype=torch.uint8, device=dev)
    ops.autotune(f, g, p, reps=10)

    def step():
        ops.sgwls_filter(f, g, p, out=u, workspace=ws)

    for _ in range(warmup):
        step()
    ms = time_events(torch, step, steps)
    return {"workload": w.name, "M": M, "N": N, "C": C, "r": p.r, "iters": p.iters,
            "stride": p.stride, "ms_per_step": round(ms, 5),
            "value": round(M * N / (ms * 1e-3) / 1e6, 2), "unit": "MPixel/s"}


def time_interpolation(torch, ops, w, dev, steps, warmup):
    """Mean ms of one guided sparse interpolation (Eq. 21) on workload w."""
    C, M, N = w.f.shape
    p = ops.Params(**w.params)
    f = torch.from_numpy(w.f).to(dev)
    h = torch.from_numpy(w.h).to(dev)
    g = torch.from_numpy(w.g).to(dev)
    u = torch.empty_like(f)
    ws = torch.empty(ops.interpolate_workspace_bytes(C, M, N, p), dtype=torch.uint8, device=dev)

    def step():
        ops.sgwls_interpolate(f, h, g, p, out=u, workspace=ws)

    for _ in range(warmup):
        step()
    ms = time_events(torch, step, steps)
    return {"workload": w.name, "M": M, "N": N, "C": C, "r": p.r, "iters": p.iters,
            "stride": p.stride, "lambda": p.lam, "known": round(float(w.h.mean()), 4),
            "ms_per_step": round(ms, 5), "value": round(M * N / (ms * 1e-3) / 1e6, 2),
            "unit": "MPixel/s"}


COMPACT_SWEEP = ((1, 1), (1, 3), (2, 1), (2, 5), (4, 1), (4, 4), (4, 9))


def stride_sweep(torch, ops, synth, dev, args, compact=False):
    """Filter time over radius and stride on the paper's timing shape (a 1 MP
    RGB image, T = 4): the same sweep as the paper's timing figure (compact:
    the (r, stride) pairs of COMPACT_SWEEP only).  Every point autotuned."""
    rows = []
    pairs = COMPACT_SWEEP if compact else [(r, s) for r in (1, 2, 3, 4) for s in range(1, 2 * r + 2)]
    for r, stride in pairs:
        w = synth.single(f"rgb1024_r{r}_T4_s{stride}", 1024, 1024, 3, 200, 0.03, 1000, 4.0, r,
                         4, stride, sinus=True)
        t = time_workload(torch, ops, w, dev, max(5, args.steps // 5), 2)
        rows.append({"r": r, "stride": stride, "ms_per_step": t["ms_per_step"],
                     "value": t["value"]})
        print(f"[sweep] r={r} stride={stride} {t['ms_per_step']:.4f} ms", file=sys.stderr,
              flush=True)
    return {"workload": "1024x1024 RGB, T=4, lambda 4, exp weights", "unit": "MPixel/s",
            "rows": rows}


def time_wls2d(torch, ops, f, g, p, u_sg, steps):
    """The 2D WLS model (Eqs. 1-4) on the same input, by the GPU conjugate-
    gradient solver to a relative residual of 1e-6: its time and the SG-WLS
    approximation gap (normwise max and mean over the output)."""
    out = torch.empty_like(f)
    ws = torch.empty(ops.wls2d_workspace_bytes(*f.shape, p), dtype=torch.uint8, device=f.device)
    _, its, res = ops.wls2d(f, g, p, tol=1e-6, out=out, workspace=ws)
    ms = time_events(torch, lambda: ops.wls2d(f, g, p, tol=1e-6, out=out, workspace=ws), steps)
    scale = float(out.abs().max())
    return {"solver": "Jacobi-preconditioned CG, float32 vectors, float64 dot products",
            "iterations": its, "rel_residual": res, "ms_per_call": round(ms, 4),
            "sgwls_gap_max": round(float((u_sg - out).abs().max()) / scale, 5),
            "sgwls_gap_mean": round(float((u_sg - out).abs().mean()) / scale, 6)}


def counter_run(torch, step, args, ms_note):
    """Forward steps followed by a plain device copy of known size: a counter
    pass divides each kernel's FETCH_SIZE / WRITE_SIZE by what the copy's
    dispatches read for their 64 MiB, which gives HBM bytes."""
    for _ in range(args.warmup + args.steps):
        step()
    torch.cuda.synchronize()
    src = torch.ones(64 * 1024 * 1024 // 4, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)          # 64 MiB read + 64 MiB written per copy
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": True, "filter_calls": args.warmup + args.steps,
                      "calibration_copy_bytes": 64 * 1024 * 1024, **ms_note}), flush=True)


def fused_rows(torch, ops, f, g, p, ws, reps):
    """The filter call with its passes fused (SGWLS_ONE_LAUNCH = 1: one launch
    per pass; 2: elimination + separator systems in one launch, re-solve in a
    second) against the default three launches, at the tuned variants."""
    old = os.environ.get("SGWLS_ONE_LAUNCH")
    out = {}
    try:
        for mode, key in (("0", "three_launch_ms"), ("2", "two_launch_ms"), ("1", "one_launch_ms")):
            os.environ["SGWLS_ONE_LAUNCH"] = mode
            fn = lambda: ops.sgwls_filter(f, g, p, workspace=ws)
            fn()
            out[key] = round(time_events(torch, fn, reps), 5)
            ops.filter_status(ws)
    finally:
        if old is None:
            os.environ.pop("SGWLS_ONE_LAUNCH", None)
        else:
            os.environ["SGWLS_ONE_LAUNCH"] = old
    return out


def time_events(torch, fn, reps):
    """Mean milliseconds of fn() over reps calls, HIP events on the current stream."""
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def bench_batched(torch, ops, synth, args):
    """The 64-image uneven batch: one batched call (graph replay on a side
    stream) against a loop of single-image filter calls on the same images."""
    ws_ = synth.batch_uneven()
    fs = [torch.from_numpy(w.f).cuda() for w in ws_]
    gs = [torch.from_numpy(w.g).cuda() for w in ws_]
    ps = [ops.Params(**w.params) for w in ws_]
    outs = [torch.empty_like(x) for x in fs]
    px = sum(w.f.shape[-2] * w.f.shape[-1] for w in ws_)
    ws = torch.empty(ops.batched_workspace_bytes(fs, gs, ps), dtype=torch.uint8, device="cuda")
    variant = ops.autotune_batched(fs, gs, ps, reps=2, workspace=ws)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()

    def step():
        ops.sgwls_filter_batched(fs, gs, ps, outs=outs, workspace=ws, stream=side)

    with torch.cuda.stream(side):
        for _ in range(2):
            step()
        side.synchronize()
        reps = max(3, args.steps // 10)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(side)
        for _ in range(reps):
            step()
        stop.record(side)
        side.synchronize()
    ms = start.elapsed_time(stop) / reps
    wss = [torch.empty(ops.workspace_bytes(1, x.shape[-2], x.shape[-1], p), dtype=torch.uint8,
                       device="cuda") for x, p in zip(fs, ps)]

    def loop():
        for x, gg, p, o, w in zip(fs, gs, ps, outs, wss):
            ops.sgwls_filter(x, gg, p, out=o, workspace=w)

    loop()
    ms_loop = time_events(torch, loop, max(3, args.steps // 10))
    alg = 12 * px * 2 * ps[0].iters            # grey: (8C + 4) bytes per pixel and pass
    return {"workload": "64 grey images, sides U[256, 2048], r in {1, 2}, lambda 2^U[-1, 5], T=3",
            "MPixel": round(px / 1e6, 2), "variant": variant,
            "value": round(px / (ms * 1e-3) / 1e6, 2), "unit": "MPixel/s", "ms_per_step": round(ms, 4),
            "alg_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "per_image_loop_ms": round(ms_loop, 4), "speedup_vs_loop": round(ms_loop / ms, 3)}


def config_rows(torch, ops, synth, dev, args):
    """The other workloads: grey 256^2 (r=1, T=1) and RGB 768x1024 (r=1, T=3)
    forward, and the 16 x 3 x 512^2 differentiation batch forward + backward
    through the autograd function (learnable lambda, MSE loss to the seeded
    noise-free targets), in the default precision and in float32."""
    rows = []
    for w in (synth.grey256(), synth.rgb768x1024()):
        t = time_workload(torch, ops, w, dev, args.steps, args.warmup)
        C, M, N = w.f.shape
        alg = (8 * C + 4) * M * N * 2 * w.params["iters"]
        t["precision"] = ops.resolve_precision(ops.Params(**w.params))
        t["hbm_frac"] = round(alg / (t["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        rows.append(t)
    B, C, M, N = 16, 3, 512, 512
    fs, gs, ts = synth.rgb_batch_with_target(B=B, M=M, N=N)
    f = torch.from_numpy(fs).to(dev)
    g = torch.from_numpy(gs).to(dev)
    tgt = torch.from_numpy(ts).to(dev)
    alg = ((8 * C + 4) + (12 * C + 8)) * M * N * B * 2 * 3
    for prec in ("auto", "fp32"):
        p = ops.Params(lam=8.0, r=1, iters=3, sigma_r=0.1, prec=prec)
        ft = f.clone().requires_grad_(True)
        gt = g.clone().requires_grad_(True)
        lam = torch.tensor([8.0], device=dev, requires_grad=True)

        def step():
            ft.grad = gt.grad = lam.grad = None
            u = ops.sgwls(ft, gt, lam, p)
            ((u - tgt) ** 2).mean().backward()

        for _ in range(max(2, args.warmup // 2)):
            step()
        ms = time_events(torch, step, max(3, args.steps // 4))
        rows.append({"workload": "diff16x3x512x512_r1_T3_lam8", "B": B, "C": C, "M": M, "N": N,
                     "r": 1, "iters": 3, "prec": prec,
                     "precision": ops.resolve_precision(p.with_(lam=8.0), True) if prec == "auto" else prec,
                     "step": "forward + MSE loss + backward (grad f, g, lambda) via ops.sgwls",
                     "ms_per_step": round(ms, 4), "value": round(B * M * N / (ms * 1e-3) / 1e6, 2),
                     "unit": "MPixel/s", "alg_GBps": round(alg / (ms * 1e-3) / 1e9, 1),
                     "hbm_frac": round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    return rows


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1705_01674_amd import _native as nat
    from paper_1705_01674_amd import ops, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.sweep:
        print(json.dumps({"sweep": stride_sweep(torch, ops, synth, dev, args)}), flush=True)
        return
    if args.counters == "radius":
        rows = radius_rows(torch, ops, nat, synth, dev, args, counters=True)
        print(json.dumps({"counters_run": True, "radius": rows}), flush=True)
        return
    w = synth.rgb1080p(stride=args.stride)
    C, M, N = w.f.shape
    p = ops.Params(**w.params)
    f = torch.from_numpy(w.f).to(dev)
    g = torch.from_numpy(w.g).to(dev)
    u = torch.empty_like(f)
    ws = torch.empty(ops.workspace_bytes(C, M, N, p), dtype=torch.uint8, device=dev)

    # kernel variants chosen by the autotuner for this shape
    tuned = ops.autotune(f, g, p, reps=20)

    def step():
        ops.sgwls_filter(f, g, p, out=u, workspace=ws)

    if args.counters == "fwd":
        counter_run(torch, step, args, {"variants": frame_variants(tuned)})
        return
    if args.fused:
        print(json.dumps({"fused_passes": fused_rows(torch, ops, f, g, p, ws, args.steps)}),
              flush=True)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = time_events(torch, step, args.steps)
    mpix = M * N / (ms * 1e-3) / 1e6

    transposed, stage_ms, per_filter_ms = stage_times(torch, nat, f, g, p, ws, args.steps)
    # Cold calls: a 512 MiB scratch write before each call evicts the 256 MB
    # Infinity Cache, so the first pass reads its inputs from HBM.
    scratch = torch.empty(128 * 1024 * 1024, dtype=torch.float32, device=dev)
    cold = []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(max(5, args.steps // 5)):
        scratch.fill_(1.0)
        ev0.record()
        step()
        ev1.record()
        torch.cuda.synchronize()
        cold.append(ev0.elapsed_time(ev1))
    ms_cold = sorted(cold)[len(cold) // 2]
    del scratch

    dom = max(per_filter_ms, key=per_filter_ms.get)
    dom_launch_ms = per_filter_ms[dom] / (2 * p.iters)   # mean over column and row launches
    px = M * N
    alg_bytes = {"k_expand": (8 * C + 4) * px, "k_reduce": (4 * C + 4) * px}
    alg = alg_bytes.get(dom)
    achieved = alg / (dom_launch_ms * 1e-3) / 1e9 if alg else None

    # Forward + backward: the forward call saves every pass input, the
    # backward call consumes them with a fixed output gradient (that of an MSE
    # loss to a seeded target, computed once outside the timed region).
    saved = torch.empty((2 * p.iters, C, M, N), dtype=torch.float32, device=dev)
    ws_b = torch.empty(ops.backward_workspace_bytes(C, M, N, p), dtype=torch.uint8, device=dev)
    ws_s = torch.empty(ops.workspace_bytes(C, M, N, p, True), dtype=torch.uint8, device=dev)
    # the forward also keeps every pass's separator solutions, so that each
    # backward pass solves only the adjoint's separator systems
    seps = torch.empty(ops.separator_bytes_nchw(1, C, M, N, p), dtype=torch.uint8, device=dev)
    ops.sgwls_filter(f, g, p, saved=saved, out=u, workspace=ws_s)
    tgt = torch.from_numpy(synth.image(M, N, C, 200, 0.0, 1000, sinus=True)).to(dev)
    ubar = (2.0 / u.numel()) * (u - tgt)
    grad_f = torch.empty_like(f)
    grad_g = torch.empty_like(g)
    grad_l = torch.empty(1, dtype=torch.float64, device=dev)

    def step_fb():
        ops.sgwls_filter(f, g, p, saved=saved, out=u, workspace=ws_s, seps=seps)
        ops.sgwls_backward(g, saved, ubar, p, grad_f=grad_f, grad_g=grad_g, grad_lambda=grad_l,
                           workspace=ws_b, seps=seps, f=f)

    def step_fb_plain():
        ops.sgwls_filter(f, g, p, saved=saved, out=u, workspace=ws_s)
        ops.sgwls_backward(g, saved, ubar, p, grad_f=grad_f, grad_g=grad_g, grad_lambda=grad_l,
                           workspace=ws_b)

    if args.counters == "fwdbwd":
        counter_run(torch, step_fb, args, {})
        return
    for _ in range(args.warmup):
        step_fb()
    torch.cuda.synchronize()
    ms_fb = time_events(torch, step_fb, args.steps)
    for _ in range(args.warmup):
        step_fb_plain()
    ms_fb_plain = time_events(torch, step_fb_plain, args.steps)
    fb_bytes = ((8 * C + 4) + (12 * C + 8)) * M * N * 2 * p.iters
    step_fb()
    torch.cuda.synchronize()
    gpu_grads = (grad_f.cpu().numpy().astype(np.float64), grad_g.cpu().numpy().astype(np.float64),
                 float(grad_l.item()))

    # The same step in explicit float32 (no lambda-gradient precision rule).
    p32 = p.with_(prec="fp32")
    ws_s32 = torch.empty(ops.workspace_bytes(C, M, N, p32, True), dtype=torch.uint8, device=dev)
    ws_b32 = torch.empty(ops.backward_workspace_bytes(C, M, N, p32), dtype=torch.uint8, device=dev)
    grad_f32, grad_g32 = torch.empty_like(f), torch.empty_like(g)
    grad_l32 = torch.empty(1, dtype=torch.float64, device=dev)
    u32 = torch.empty_like(f)
    seps32 = torch.empty(ops.separator_bytes_nchw(1, C, M, N, p32), dtype=torch.uint8, device=dev)

    def step_fb32():
        ops.sgwls_filter(f, g, p32, saved=saved, out=u32, workspace=ws_s32, seps=seps32)
        ops.sgwls_backward(g, saved, ubar, p32, grad_f=grad_f32, grad_g=grad_g32,
                           grad_lambda=grad_l32, workspace=ws_b32, seps=seps32, f=f)

    for _ in range(args.warmup):
        step_fb32()
    ms_fb32 = time_events(torch, step_fb32, args.steps)
    step_fb32()
    torch.cuda.synchronize()
    gpu_grads32 = (grad_f32.cpu().numpy().astype(np.float64),
                   grad_g32.cpu().numpy().astype(np.float64), float(grad_l32.item()))

    # Float64 pivots and recurrences on the same workload.
    p64 = p.with_(prec="fp64_pivot")
    ws64 = torch.empty(ops.workspace_bytes(C, M, N, p64), dtype=torch.uint8, device=dev)
    u64 = torch.empty_like(f)

    def step64():
        ops.sgwls_filter(f, g, p64, out=u64, workspace=ws64)

    for _ in range(args.warmup):
        step64()
    ms64 = time_events(torch, step64, max(5, args.steps // 2))

    # The cancellation-free float32 mode (serial strips, excess pivots).
    pd = p.with_(prec="fp32_delta")
    wsd = torch.empty(ops.workspace_bytes(C, M, N, pd), dtype=torch.uint8, device=dev)
    ud = torch.empty_like(f)

    def stepd():
        ops.sgwls_filter(f, g, pd, out=ud, workspace=wsd)

    stepd()
    msd = time_events(torch, stepd, max(3, args.steps // 10))

    batched = None if args.no_batched else bench_batched(torch, ops, synth, args)
    step()
    wls = time_wls2d(torch, ops, f, g, p, u.clone(), max(3, args.steps // 10))
    # The other reading of "tau = 3" (stride 3 = 2r+1, no overlap) and the
    # 1024x1024 RGB T=4 context row.
    alt_steps = max(5, args.steps // 2)
    stride3 = time_workload(torch, ops, synth.rgb1080p(stride=3), dev, alt_steps, args.warmup)
    ctx = time_workload(torch, ops, synth.rgb1024_ctx(), dev, alt_steps, args.warmup)
    radius = radius_rows(torch, ops, nat, synth, dev, args)
    # Guided sparse interpolation, Eq. (21): 8x depth upsampling at 1080p and
    # scribble colourisation (two chrominance planes) at 1024x1024.
    interp = [time_interpolation(torch, ops, synth.depth_upsample(1080, 1920, 8), dev, alt_steps,
                                 args.warmup),
              time_interpolation(torch, ops, synth.colorize_scribbles(1024, 1024, 120), dev,
                                 alt_steps, args.warmup)]

    configs = config_rows(torch, ops, synth, dev, args)
    fused = fused_rows(torch, ops, f, g, p, ws, args.steps)
    sweep = stride_sweep(torch, ops, synth, dev, args, compact=True)

    # Accuracy of this very output against the oracle, and the CPU baseline.
    step()
    torch.cuda.synchronize()
    gpu_out = u.cpu().numpy().astype(np.float64)
    cpu = None
    max_rel = None
    max_rel64 = None
    max_reld = None
    grad_err = None
    grad_err32 = None
    if not args.no_cpu_baseline:
        import oracle
        P = oracle.OracleParams(**w.params)
        f64, g64 = w.f.astype(np.float64), w.g.astype(np.float64)
        times = []
        ref = None
        for _ in range(args.cpu_reps):
            t0 = time.perf_counter()
            ref = oracle.filter(f64, g64, P)
            times.append(time.perf_counter() - t0)
        tmed = sorted(times)[len(times) // 2]
        cores = oracle.num_threads()
        # the same filter on one core (one run)
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.filter(f64, g64, P)
        t1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        cpu = {"value": round(px / tmed / 1e6, 4), "unit": "MPixel/s",
               "cores": cores, "kind": "oracle",
               "sample": f"the full workload (one {M}x{N}x{C} filter, T={p.iters}), "
                         f"median of {args.cpu_reps} runs, {tmed:.2f} s each",
               "single_core": {"value": round(px / t1 / 1e6, 4), "cores": 1,
                               "sample": f"one run, {t1:.2f} s"}}
        max_rel = float(np.abs(gpu_out - ref).max() / np.abs(ref).max())
        max_rel64 = float(np.abs(u64.cpu().numpy().astype(np.float64) - ref).max() / np.abs(ref).max())
        max_reld = float(np.abs(ud.cpu().numpy().astype(np.float64) - ref).max() / np.abs(ref).max())
        _, ref_saved = oracle.filter(f64, g64, P, save=True)
        rf, rg, rl = oracle.filter_backward(g64, ref_saved, ubar.cpu().numpy().astype(np.float64), P)
        def gerr(gr):
            return {"grad_f": float(np.abs(gr[0] - rf).max() / np.abs(rf).max()),
                    "grad_g": float(np.abs(gr[1] - rg).max() / np.abs(rg).max()),
                    "grad_lambda": abs(gr[2] - rl) / abs(rl)}
        grad_err = gerr(gpu_grads)
        grad_err32 = gerr(gpu_grads32)

    line = {
        "metric": "MPixel/s per SG-WLS filter (1080p RGB, r=1, tau=3) fwd",
        "value": round(mpix, 2),
        "unit": "MPixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "M": M, "N": N, "C": C, "r": p.r, "iters": p.iters,
                   "stride": p.stride, "lambda": p.lam, "weight": p.kind,
                   "sigma_s": float(p.r), "sigma_r": p.sigma_r,
                   "variants": frame_variants(tuned)},
        "roofline": {"bound": "hbm", "kernel": dom,
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": counted_traffic(tuned) if dom == "k_expand" else None},
        "kernels_ms_per_launch": {f"{'col' if d == 0 else 'row'}:{n}": round(t, 5)
                                  for (d, n), t in stage_ms.items()},
        "row_pass_as_transposed_column_pass": transposed,
        "filter_alg_GBps": round((8 * C + 4) * px * 2 * p.iters / (ms * 1e-3) / 1e9, 1),
        "filter_hbm_frac": round((8 * C + 4) * px * 2 * p.iters / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "precision": ops.resolve_precision(p),
        "max_rel_err_vs_oracle": max_rel,
        "fwd_bwd": {"metric": "MPixel/s per SG-WLS filter (1080p RGB, r=1, tau=3) fwd+bwd",
                    "precision": {"forward": ops.resolve_precision(p, True),
                                  "backward": ops.resolve_precision(p, True)},
                    "value": round(M * N / (ms_fb * 1e-3) / 1e6, 2), "ms_per_step": round(ms_fb, 5),
                    "alg_bytes": fb_bytes,
                    "alg_GBps": round(fb_bytes / (ms_fb * 1e-3) / 1e9, 1),
                    "hbm_frac": round(fb_bytes / (ms_fb * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "saved_separators": True,
                    "without_saved_separators": {
                        "ms_per_step": round(ms_fb_plain, 5),
                        "value": round(M * N / (ms_fb_plain * 1e-3) / 1e6, 2)},
                    "max_rel_err_vs_oracle": grad_err},
        "fwd_bwd_fp32": {"value": round(M * N / (ms_fb32 * 1e-3) / 1e6, 2),
                         "ms_per_step": round(ms_fb32, 5),
                         "alg_GBps": round(fb_bytes / (ms_fb32 * 1e-3) / 1e9, 1),
                         "hbm_frac": round(fb_bytes / (ms_fb32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "max_rel_err_vs_oracle": grad_err32},
        "fp64_pivot": {"ms_per_step": round(ms64, 5), "value": round(M * N / (ms64 * 1e-3) / 1e6, 2),
                       "max_rel_err_vs_oracle": max_rel64},
        "fp32_delta": {"ms_per_step": round(msd, 5), "value": round(M * N / (msd * 1e-3) / 1e6, 2),
                       "max_rel_err_vs_oracle": max_reld,
                       "note": "serial strip solves with excess pivots (r = 1 precision mode)"},
        "cold": {"ms_per_step": round(ms_cold, 5), "value": round(M * N / (ms_cold * 1e-3) / 1e6, 2),
                 "note": "median of single calls, each after a 512 MiB scratch write"},
        "fused_passes": fused,
        "stride_sweep": sweep,
        "stride3": stride3,
        "ctx": ctx,
        "radius": radius,
        "interpolation": interp,
        "wls2d": wls,
        "batched": batched,
        "configs": configs,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
