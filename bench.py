"""Benchmark of the structure-flow filter on one MI355X.

A step is one frame through the whole hot path: sf_push_frame (pyramid, the fused level
step of every level - prediction, image and depth models, least-squares update, smoothing,
inverse-depth update - and the coarse-to-fine reconstruction) followed by sf_get_flow of the
finest-level structure flow in rad/s.  Inputs are seeded synthetic ray-cast frames already
resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s at 512x512 (Hz) + HBM GB/s % peak; batched & learned vs plain at EPE"
# The paper's own runtime tables (GTX-780; mapping onto the Spherepix grid plus the filter,
# transfers excluded; Hz is a mean of per-frame rates): context for the sweep, not a target.
PAPER_TABLES = {
    "runtime_pyramid_1": {"512^2, 1 level, smoothing 2": {"1": 1133.9, "2": 998.1, "4": 755.6}},
    "runtime_pyramid_2": {"512^2, 2 levels, smoothing [2, 4]": {"1": 747.4, "2": 720.5,
                                                                 "4": 674.3, "8": 594.7}},
    "runtime_pyramid_2_1024": {"1024^2, 2 levels, smoothing [2, 4]": {"1": 213.889,
                                                                      "2": 207.480,
                                                                      "4": 194.258,
                                                                      "8": 172.149}},
}
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3          # published MI355X vector FP32 (packed FMA)
FP32_UNPACKED_TFLOPS = 78.6       # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


# ---- algorithmic models of the fused level-step kernel (per pixel of a level) ----------
def step_bytes_per_px(top: bool, esize: int) -> int:
    """Each input and state value read once, each new state value written once:
    measurements Y, rho (2); frame-k state w(3) [+ dw(3)] + rho + Yhat; new state
    (dw(3) or w(3)) + rho + Yhat."""
    reads = 2 + (5 if top else 8)
    writes = 5
    return (reads + writes) * esize


def step_flops_per_px(top: bool, N: int, Ns: int) -> int:
    """Floating-point operations of the method per pixel (one count per add/mul, FMA = 2):
    per half-step 11 for the flow component and <eta, w>, 7 per sourced field, 4 for the
    image; image model 50 (separable taps), depth model 6, least-squares update 90,
    5x5 smoothing 27 per pass, inverse-depth update 5."""
    half = 11 + (4 * 7 if top else 7 * 7 + 4)
    return 2 * N * half + 50 + 6 + 90 + 27 * Ns + 5


def level_table(rows, cols, levels, max_flow, smooth):
    out = []
    r, c = rows, cols
    for h in range(levels):
        N = max(1, math.ceil(max_flow / 2 ** h))
        out.append(dict(rows=r, cols=c, N=N, Ns=smooth[h], top=h == levels - 1))
        r, c = (r + 1) // 2, (c + 1) // 2
    return out


def render_frames(seq, device):
    import torch
    Ys, Rs = [], []
    for k in range(seq.n_frames):
        f = seq.frame(k, device)
        Ys.append(f.Y.to(torch.float32).contiguous())
        Rs.append(f.rho.to(torch.float32).contiguous())
    return Ys, Rs


def tune_levels(rows, cols, levels, max_flow, smooth):
    """The autotuner's description of one stream's levels."""
    lv = []
    for h in range(levels):
        lv.append(dict(rows=rows, cols=cols, max_flow_px=max_flow, smooth=smooth[h], h=h))
        rows, cols = (rows + 1) // 2, (cols + 1) // 2
    return lv


def run_gpu(wl_name, steps, warmup, storage=0, autotune=False):
    import numpy as np
    import torch
    from paper_2406_18031_amd import sflow
    from synth.workloads import workload

    wl = workload(wl_name)
    seq = wl["build"]("cuda")
    cam = seq.camera
    Ys, Rs = render_frames(seq, "cuda")
    if storage == 1:
        Ys = [y.half() for y in Ys]
        Rs = [r.half() for r in Rs]
    F = len(Ys)
    f = sflow.Filter(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"], wl["smooth"],
                     cam.fx, cam.fy, cam.cx, cam.cy, storage=storage)
    out = torch.empty((3, seq.rows, seq.cols), dtype=torch.float32, device="cuda")
    setting = None
    if autotune:   # launch shape from the autotuner, then the stream restarts from frame 0
        from paper_2406_18031_amd import tune
        setting = tune.tune(f.ctx, lambda k: f.push(Ys[k % F], Rs[k % F], seq.dt),
                            tune_levels(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"],
                                        wl["smooth"]))
        sflow.sf_set_camera(f.ctx, cam.fx, cam.fy, cam.cx, cam.cy)

    def step(k):
        f.push(Ys[k % F], Rs[k % F], seq.dt)
        sflow.sf_get_flow(f.ctx, sflow.SF_FLOW_W_RAD_S, out)

    def restart():   # the next push is a first frame (the launch shape is kept)
        sflow.sf_set_camera(f.ctx, cam.fx, cam.fy, cam.cx, cam.cy)

    # every pass starts from a restarted state and runs warmup + steps frames, so that no pass
    # carries the state further than the throughput pass (see finite_after)
    restart()
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    finite = bool(torch.isfinite(out).all())
    graph = graph_pass(f.ctx, step, steps, warmup, restart)
    overlap = overlap_pass(f.ctx, step, steps, warmup, restart)

    # kernel durations from HIP events on the context stream, over a second pass of the
    # same frames (events add host work, so the throughput pass above runs without them)
    restart()
    for k in range(warmup):
        step(k)
    sflow.sf_set_timing(f.ctx, True)
    sflow.sf_kernel_times(f.ctx, reset=True)
    for k in range(warmup, warmup + steps):
        step(k)
    ms, n = sflow.sf_kernel_times(f.ctx, reset=True)
    sflow.sf_set_timing(f.ctx, False)
    final = f.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
    f.close()
    return dict(seq=seq, wl=wl, elapsed=elapsed, kernel_ms=ms, kernel_n=n, final=final,
                tuned=setting, graph=graph, overlap=overlap,
                finite_after={"frames": warmup + steps, "timed_pass": finite,
                              "timing_pass": bool(np.isfinite(final).all())})


def run_batched(n_streams, steps, warmup, storage=0, frames=40):
    """n_streams independent camera streams of mixed sizes advanced together: one pyramid
    launch and one reconstruction launch per two depths, the level-step launches and one
    output call per frame for all streams.  A step is one frame of every stream plus every
    stream's output."""
    import torch
    from paper_2406_18031_amd import sflow
    from synth.workloads import stream_mix

    mix = stream_mix(n_streams, n_frames=frames, device="cuda")
    specs, Ys, Rs = [], [], []
    for m in mix:
        seq = m["build"]()
        c = seq.camera
        specs.append(dict(rows=seq.rows, cols=seq.cols, levels=m["levels"],
                          max_flow_px=m["max_flow_px"], smooth=m["smooth"],
                          camera=(c.fx, c.fy, c.cx, c.cy)))
        y, r = render_frames(seq, "cuda")
        if storage == 1:
            y = [v.half() for v in y]
            r = [v.half() for v in r]
        Ys.append(y)
        Rs.append(r)
        dt = seq.dt
    b = sflow.Batch(specs, storage=storage)
    outs = [torch.empty((3, sp["rows"], sp["cols"]), dtype=torch.float32, device="cuda")
            for sp in specs]
    dts = [dt] * len(specs)

    def step(k):
        b.push([y[k % frames] for y in Ys], [r[k % frames] for r in Rs], dts)
        sflow.sf_get_flows(b.ctx, sflow.SF_FLOW_W_RAD_S, outs)

    # launch shape from the autotuner (pass length; tiles of the largest stream's levels)
    from paper_2406_18031_amd import tune
    big = max(specs, key=lambda sp: sp["rows"] * sp["cols"])
    lv = []
    r_, c_ = big["rows"], big["cols"]
    for h in range(big["levels"]):
        lv.append(dict(rows=r_, cols=c_, max_flow_px=big["max_flow_px"], smooth=big["smooth"][h],
                       h=h))
        r_, c_ = (r_ + 1) // 2, (c_ + 1) // 2
    setting = tune.tune(b.ctx, lambda k: b.push([y[k % frames] for y in Ys],
                                                [r[k % frames] for r in Rs], dts), lv)

    def restart():   # every stream's next push is a first frame (the launch shape is kept)
        sflow.sf_set_cameras(b.ctx, [sp["camera"] for sp in specs])

    def finite():
        return all(bool(torch.isfinite(o).all()) for o in outs)

    warm = max(2, min(warmup, frames // 8))
    elapsed, steps, fin_timed = segmented(step, restart, finite, steps, frames, warm)
    graph = graph_pass(b.ctx, step, frames - warm, warm, restart)
    restart()
    for k in range(warm):
        step(k)
    sflow.sf_set_timing(b.ctx, True)
    sflow.sf_kernel_times(b.ctx, reset=True)
    for k in range(warm, frames):
        step(k)
    ms, n = sflow.sf_kernel_times(b.ctx, reset=True)
    fin_timing = finite()
    b.close()
    kt = frames - warm   # frames of the kernel-timing pass
    px = sum(sp["rows"] * sp["cols"] for sp in specs)
    step_bytes = step_flops = 0
    for sp in specs:
        for L in level_table(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"]):
            npx = L["rows"] * L["cols"]
            step_bytes += npx * step_bytes_per_px(L["top"], 2 if storage == 1 else 4)
            step_flops += npx * step_flops_per_px(L["top"], L["N"], L["Ns"])
    step_s = ms[1] / kt * 1e-3          # level-step time per frame (all passes)
    sizes = {}
    for sp in specs:
        sizes[sp["rows"]] = sizes.get(sp["rows"], 0) + 1
    return {
        "streams": len(specs), "sizes": {f"{k}x{k}": v for k, v in sorted(sizes.items())},
        "storage": "fp16" if storage == 1 else "fp32",
        "aggregate_frames_per_s": len(specs) * steps / elapsed,
        "batch_steps_per_s": steps / elapsed,
        "mpix_per_s": px * steps / elapsed / 2 ** 20,
        "kernel_us_per_frame": {k: v / kt * 1e3 for k, v in
                                zip(("pyramid", "level_step", "reconstruct"), ms)},
        "level_step_tflops": step_flops / step_s / 1e12,
        "level_step_hbm_gbs": step_bytes / step_s / 1e9,
        "tuned": {"pass_steps": setting["pass_steps"], "tiles": setting["tiles"]},
        "frame_graph": graph,
        "timing": f"{steps} frames in segments of frames {warm}-{frames - 1} after a restart "
                  f"({frames} rendered frames per stream, cycled)",
        "finite_after": {"frames": frames, "timed_pass": fin_timed, "timing_pass": fin_timing},
    }


def segmented(step, restart, finite, n_timed, cycle, warm):
    """Throughput of a form whose inputs repeat every `cycle` frames, timed in segments: each
    segment restarts the state, runs `warm` untimed frames and times frames warm..cycle-1, so
    that no timed frame follows a jump back to the cycle's first frame and no state is older
    than one cycle (the method's state grows without bound after O(100-1000) frames of cycled
    inputs, in the FP64 oracle too).  Returns (elapsed seconds, timed frames, state finite at
    the end of every segment)."""
    import torch
    el, done, fin = 0.0, 0, True
    while done < n_timed:
        restart()
        for k in range(warm):
            step(k)
        m = min(cycle - warm, n_timed - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warm, warm + m):
            step(k)
        torch.cuda.synchronize()
        el += time.perf_counter() - t0
        done += m
        fin = fin and finite()
    return el, done, fin


def overlap_pass(ctx, step, steps, warmup, restart):
    """The same loop with the frames declared as produced on a stream of their own
    (sf_set_input_stream; they are resident in HBM already, so that stream holds no work): each
    frame's pyramid then runs on the library's pyramid stream beside the previous frame's level
    step.  Throughput over the same frames from a restarted state."""
    import torch
    from paper_2406_18031_amd import sflow
    restart()
    s_in = torch.cuda.Stream()
    sflow.sf_set_input_stream(ctx, s_in)
    for k in range(warmup):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(warmup, warmup + steps):
        step(k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sflow.sf_set_input_stream(ctx, None)
    return {"steps_per_s": steps / el, "ms_per_step": el / steps * 1e3}


def graph_pass(ctx, step, steps, warmup, restart):
    """The same loop with the frame's launches replayed from a HIP graph (sf_set_graph):
    throughput, and the host time per step with and without the graph (submissions timed in
    chunks with the device idle before each; the long loop's wall time up to its last
    submission is kept as well); each loop from a restarted state."""
    import torch
    from paper_2406_18031_amd import sflow
    out = {}
    for on in (False, True):
        restart()
        sflow.sf_set_graph(ctx, on)
        for k in range(warmup):
            step(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup, warmup + steps):
            step(k)
        t1 = time.perf_counter()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = "graph" if on else "eager"
        out[f"steps_per_s_{key}"] = steps / (t2 - t0)
        # host time of a submission, in chunks of 32 steps with the device idle before each:
        # over a long loop the runtime blocks a launch once a few hundred launches with these
        # kernels' 2.6-3.6 KB argument blocks are queued (each block holds a slot of a fixed
        # pool until its kernel ends), so that loop's host time follows the device
        sflow.sf_set_graph(ctx, False)
        restart()
        sflow.sf_set_graph(ctx, on)
        for k in range(4):   # the first frame, then both parities' graphs are captured
            step(k)
        host, m = 0.0, 0
        while m < min(steps, 256):
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for k in range(4 + m, 4 + m + 32):
                step(k)
            host += time.perf_counter() - c0
            m += 32
        torch.cuda.synchronize()
        out[f"host_us_per_step_{key}"] = host / m * 1e6
        out[f"host_us_per_step_{key}_long_loop"] = (t1 - t0) / steps * 1e6
    sflow.sf_set_graph(ctx, False)
    return out


def run_inertial(steps, warmup):
    """The prediction with the inertial source terms (sf_push_frame_ex) on the boxes512
    workload, fed the rates the camera's inertial unit would report (synth: angular velocity and
    its rate of change at mid-interval, zero inertial acceleration).  Throughput as the headline's loop; accuracy:
    endpoint error against the true flow over frames 10-99, plain and inertial, on boxes512
    (20 % of the image motion from rotation) and on a rotation-dominated variant (80 %)."""
    import torch
    from paper_2406_18031_amd import sflow
    from synth.scenes import box_sequence
    from synth.workloads import workload

    wl = workload("boxes512")
    out = {}
    for name, seq in (("boxes512", wl["build"]("cuda")),
                      ("boxes512_rotation80", box_sequence(512, 512, 100, seed=2, max_flow_px=8.0,
                                                           rot_share=0.8, device="cuda"))):
        cam = seq.camera
        fr = [seq.frame(k, "cuda") for k in range(seq.n_frames)]
        Ys = [f.Y.to(torch.float32).contiguous() for f in fr]
        Rs = [f.rho.to(torch.float32).contiguous() for f in fr]
        Ws = [(f.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous() for f in fr]
        imu = [seq.imu(k) for k in range(seq.n_frames)]
        del fr
        dmu = _pinhole_dmu_t(seq, "cuda")
        F = len(Ys)
        row = {}
        for use in (False, True):
            f = sflow.Filter(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"], wl["smooth"],
                             cam.fx, cam.fy, cam.cx, cam.cy)
            err = []
            for k in range(F):
                if use:
                    f.push(Ys[k], Rs[k], seq.dt, omega=imu[k][0], omega_dot=imu[k][1],
                           acc=imu[k][2])
                else:
                    f.push(Ys[k], Rs[k], seq.dt)
                if k >= 10:
                    err.append(float(((f.flow(sflow.SF_FLOW_W_FRAME) - Ws[k]).norm(dim=0)
                                      / dmu).mean()))
            key = "inertial" if use else "plain"
            row[f"gt_epe_px_{key}"] = sum(err) / len(err)
            if use and name == "boxes512":
                out_t = torch.empty((3, seq.rows, seq.cols), dtype=torch.float32, device="cuda")

                def step(k):
                    m = imu[k % F]
                    f.push(Ys[k % F], Rs[k % F], seq.dt, omega=m[0], omega_dot=m[1], acc=m[2])
                    sflow.sf_get_flow(f.ctx, sflow.SF_FLOW_W_RAD_S, out_t)

                def restart():
                    sflow.sf_set_camera(f.ctx, cam.fx, cam.fy, cam.cx, cam.cy)

                def finite():
                    return bool(torch.isfinite(out_t).all())

                el, nt, fin = segmented(step, restart, finite, steps, F, 10)
                out["frames_per_s"] = nt / el
                out["timing"] = (f"{nt} frames in segments of frames 10-{F - 1} after a restart")
                out["finite_after"] = {"frames": F, "timed_pass": fin}
            f.close()
        row["gt_epe_inertial_over_plain"] = row["gt_epe_px_inertial"] / row["gt_epe_px_plain"]
        out[name] = row
    out["workload"] = ("boxes512 (and its rotation-dominated variant) with the renderer's "
                       "angular velocity at mid-interval; accuracy over frames 10-99")
    return out


def run_grid_stereo(steps, warmup, frames=40, warm=10):
    """Two forms beyond the pinhole depth-sensor filter, on 512x512 box scenes (3 levels,
    max flow 8 px):
    - grid: a 90-degree equiangular grid of 512x512 directions fed by a 640x640 pinhole camera;
      each step maps the camera's frame onto the grid (sf_map_frame) and pushes it;
    - stereo: the inverse depth taken from a rectified stereo pair (baseline 0.1 m) each frame
      (sf_stereo_depth) instead of a depth sensor; throughput, and the true-flow endpoint
      error over frames warm..frames-1 against the same filter fed the scene's depth (1 %
      noise)."""
    import torch
    from paper_2406_18031_amd import sflow
    from synth.scenes import box_sequence, equiangular_rays
    out = {}
    # grid + mapping
    GF = 100
    src = box_sequence(640, 640, GF, seed=2, max_flow_px=10.0, device="cuda")
    c = src.camera
    Ys, Rs = render_frames(src, "cuda")
    eta = equiangular_rays(512, 512, 90.0)
    g = sflow.Filter(512, 512, 3, 8.0, [2, 4, 4], 256.0, 256.0, 255.5, 255.5, eta=eta)
    g.set_source_camera(c.fx, c.fy, c.cx, c.cy, 640, 640)
    Yg = torch.empty((512, 512), dtype=torch.float32, device="cuda")
    Rg = torch.empty_like(Yg)
    o = torch.empty((3, 512, 512), dtype=torch.float32, device="cuda")

    def gstep(k):
        g.map(Ys[k % GF], Rs[k % GF], Yg, Rg)
        g.push(Yg, Rg, src.dt)
        sflow.sf_get_flow(g.ctx, sflow.SF_FLOW_W_RAD_S, o)

    def grestart():
        sflow.sf_set_camera(g.ctx, 256.0, 256.0, 255.5, 255.5, eta)
        g.set_source_camera(c.fx, c.fy, c.cx, c.cy, 640, 640)

    el, nt, fin = segmented(gstep, grestart, lambda: bool(torch.isfinite(o).all()), steps, GF, 10)
    out["grid_equiangular_512"] = {
        "frames_per_s": nt / el,
        "timing": f"{nt} frames in segments of frames 10-{GF - 1} after a restart",
        "finite_after": {"frames": GF, "timed_pass": fin},
        "workload": "512x512 equiangular grid of 90 degrees, frames mapped from a 640x640 "
                    "pinhole camera each step (map + push + read)"}
    g.close()
    # stereo
    b = 0.1
    seq = box_sequence(512, 512, frames, seed=2, max_flow_px=8.0, device="cuda")
    c = seq.camera
    fr = [seq.frame(k, "cuda") for k in range(frames)]
    YL = [f.Y.to(torch.float32).contiguous() for f in fr]
    YR = [seq.right_image(k, b, "cuda").to(torch.float32).contiguous() for k in range(frames)]
    RD = [f.rho.to(torch.float32).contiguous() for f in fr]
    W = [(f.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous() for f in fr]
    del fr
    dmu = _pinhole_dmu_t(seq, "cuda")
    cam = (c.fx, c.fy, c.cx, c.cy)
    dmax = 16
    row = {}
    for mode in ("stereo", "depth"):
        f = sflow.Filter(512, 512, 3, 8.0, [2, 4, 4], *cam)
        f.set_stereo(b, dmax)
        rho = torch.empty((512, 512), dtype=torch.float32, device="cuda")
        err = []
        for k in range(frames):
            if mode == "stereo":
                f.stereo_depth(YL[k], YR[k], rho)
                f.push(YL[k], rho, seq.dt)
            else:
                f.push(YL[k], RD[k], seq.dt)
            if k >= warm:
                err.append(float(((f.flow(sflow.SF_FLOW_W_FRAME) - W[k]).norm(dim=0) / dmu).mean()))
        row[f"gt_epe_px_{mode}"] = sum(err) / len(err)
        if mode == "stereo":
            def sstep(k):
                f.stereo_depth(YL[k % frames], YR[k % frames], rho)
                f.push(YL[k % frames], rho, seq.dt)
                sflow.sf_get_flow(f.ctx, sflow.SF_FLOW_W_RAD_S, o)
            for k in range(warmup):
                sstep(k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(warmup, warmup + steps):
                sstep(k)
            torch.cuda.synchronize()
            row["frames_per_s"] = steps / (time.perf_counter() - t0)
            row["finite_after"] = {"frames": frames + warmup + steps,
                                   "timed_pass": bool(torch.isfinite(o).all())}
        f.close()
    row["workload"] = (f"boxes512 scene seen by a rectified stereo pair (baseline {b} m, "
                       f"disparities up to {dmax} px); accuracy over frames {warm}-{frames - 1}")
    out["stereo_boxes512"] = row
    return out


def _pinhole_dmu_t(seq, device):
    """Tangent-plane pixel spacing of the finest pinhole grid (closed form), torch float32."""
    import torch
    c = seq.camera
    j = torch.arange(seq.cols, dtype=torch.float64, device=device)[None, :]
    i = torch.arange(seq.rows, dtype=torch.float64, device=device)[:, None]
    x = (j - c.cx) / c.fx
    y = (i - c.cy) / c.fy
    xn = x + torch.where(j < seq.cols - 1, 1.0, -1.0) / c.fx
    d = torch.sqrt(1 + y * y) / torch.sqrt(x * x + y * y + 1) / (c.fx * torch.sqrt(xn * xn + y * y + 1))
    return d.to(torch.float32)


def run_learned(n_streams, steps, warmup, frames=40, eval_frames=100, warm=10):
    """The learned update on n_streams 512 x 512 box sequences (3 levels, max flow 8 px;
    held-out seeds 20000 + i, not trained on), with the committed trained parameters and the
    fallback threshold chosen on validation seeds.  Throughput: plain and learned side by side
    on the same frames (every stream's output read each frame).  Accuracy: endpoint error
    against the true flow (px/frame) over frames warm..eval_frames-1, plain and learned on the
    same frames, and the learned form's fallback rate."""
    import torch
    from paper_2406_18031_amd import learned, sflow
    from synth.scenes import box_sequence

    params, threshold = learned.load_trained()
    seqs, specs, Ys, Rs = [], [], [], []
    for i in range(n_streams):
        seq = box_sequence(512, 512, max(eval_frames, frames), seed=20000 + i, dt=1.0 / 300.0,
                           max_flow_px=8.0, device="cuda")
        c = seq.camera
        seqs.append(seq)
        specs.append(dict(rows=512, cols=512, levels=3, max_flow_px=8.0, smooth=[2, 4, 4],
                          camera=(c.fx, c.fy, c.cx, c.cy)))
        y, r = [], []
        for k in range(frames):
            f = seq.frame(k, "cuda")
            y.append(f.Y.to(torch.float32).contiguous())
            r.append(f.rho.to(torch.float32).contiguous())
        Ys.append(y)
        Rs.append(r)
    dt = seqs[0].dt
    dts = [dt] * n_streams
    out = {}
    for name, upd in (("plain", sflow.SF_UPDATE_PLAIN), ("learned", sflow.SF_UPDATE_LEARNED)):
        b = sflow.Batch(specs, update=upd)
        if upd == sflow.SF_UPDATE_LEARNED:
            b.set_learned(params, threshold)
        outs = [torch.empty((3, 512, 512), dtype=torch.float32, device="cuda")
                for _ in range(n_streams)]

        def step(k):   # a frame of every stream and every stream's output (the learned
            # correction is applied to the output)
            b.push([y[k % frames] for y in Ys], [r[k % frames] for r in Rs], dts)
            sflow.sf_get_flows(b.ctx, sflow.SF_FLOW_W_RAD_S, outs)

        def restart(b=b):
            sflow.sf_set_cameras(b.ctx, [sp["camera"] for sp in specs])

        def finite(outs=outs):
            return all(bool(torch.isfinite(o).all()) for o in outs)

        w0 = max(2, min(warmup, frames // 8))
        el, nt, fin = segmented(step, restart, finite, steps, frames, w0)
        out[name] = {"aggregate_frames_per_s": n_streams * nt / el,
                     "ms_per_batch_frame": el / nt * 1e3,
                     "timing": f"{nt} frames in segments of frames {w0}-{frames - 1} after a "
                               f"restart ({frames} rendered frames per stream, cycled)",
                     "finite_after": {"frames": frames, "timed_pass": fin}}
        b.close()
    # accuracy against the true flow, both forms on the same rendered frames
    bp = sflow.Batch(specs)
    bl = sflow.Batch(specs, update=sflow.SF_UPDATE_LEARNED)
    bl.set_learned(params, threshold)
    dmu = [_pinhole_dmu_t(s, "cuda") for s in seqs]
    err = {"plain": [], "learned": []}
    for k in range(eval_frames):
        fr = [s.frame(k, "cuda") for s in seqs]
        ys = [f.Y.to(torch.float32).contiguous() for f in fr]
        rs = [f.rho.to(torch.float32).contiguous() for f in fr]
        if k == warm:
            bl.learned_stats(reset=True)
        for name, b in (("plain", bp), ("learned", bl)):
            b.push(ys, rs, dts)
            if k >= warm:
                e = torch.stack([((b.flow(i, sflow.SF_FLOW_W_FRAME)
                                   - (f.w_gt * s.dt).permute(2, 0, 1).to(torch.float32))
                                  .norm(dim=0) / dmu[i]).mean()
                                 for i, (f, s) in enumerate(zip(fr, seqs))])
                err[name].append(float(e.mean()))
    fb, px = bl.learned_stats()
    bp.close()
    bl.close()
    out["plain"]["gt_epe_px"] = float(sum(err["plain"]) / len(err["plain"]))
    out["learned"]["gt_epe_px"] = float(sum(err["learned"]) / len(err["learned"]))
    out["learned"]["fallback_rate"] = fb / max(1, px)
    out["learned"]["threshold"] = threshold
    out["gt_epe_learned_over_plain"] = out["learned"]["gt_epe_px"] / out["plain"]["gt_epe_px"]
    out["streams"] = n_streams
    out["workload"] = (f"512x512 box sequences, 3 levels, max flow 8 px, held-out seeds "
                       f"20000-{20000 + n_streams - 1}; trained parameters "
                       f"(paper_2406_18031_amd/weights/learned_boxes512.npz); accuracy over "
                       f"frames {warm}-{eval_frames - 1}")
    return out


def run_sweep(steps, warmup, frames=100):
    """The paper's runtime tables' shapes (512^2 one level; 512^2 and 1024^2 two levels;
    maximum flow 1/2/4/8 px; smoothing 2 / [2, 4]) on seeded box scenes: frames/s of the push
    plus output read, and the level step's HIP-event duration per frame."""
    import torch
    from paper_2406_18031_amd import sflow
    from synth.workloads import PAPER_SWEEP, sweep_sequence

    rows = []
    for t in PAPER_SWEEP:
        for mf in t["flows"]:
            seq = sweep_sequence(t["size"], mf, frames, "cuda")
            Ys, Rs = render_frames(seq, "cuda")
            c = seq.camera
            f = sflow.Filter(t["size"], t["size"], t["levels"], mf, t["smooth"], c.fx, c.fy,
                             c.cx, c.cy)
            out = torch.empty((3, t["size"], t["size"]), dtype=torch.float32, device="cuda")

            def step(k):
                f.push(Ys[k % frames], Rs[k % frames], seq.dt)
                sflow.sf_get_flow(f.ctx, sflow.SF_FLOW_W_RAD_S, out)

            def restart():
                sflow.sf_set_camera(f.ctx, c.fx, c.fy, c.cx, c.cy)

            w0 = 10
            el, nt, fin = segmented(step, restart, lambda: bool(torch.isfinite(out).all()),
                                    steps, frames, w0)
            restart()
            for k in range(w0):
                step(k)
            sflow.sf_set_timing(f.ctx, True)
            sflow.sf_kernel_times(f.ctx, reset=True)
            for k in range(w0, frames):
                step(k)
            ms, n = sflow.sf_kernel_times(f.ctx, reset=True)
            f.close()
            levels = level_table(t["size"], t["size"], t["levels"], mf, t["smooth"])
            rows.append({
                "table": t["table"], "size": t["size"], "levels": t["levels"],
                "smooth": t["smooth"], "max_flow_px": mf,
                "N": [L["N"] for L in levels],
                "frames_per_s": nt / el, "ms_per_frame": el / nt * 1e3,
                "mpix_per_s": t["size"] ** 2 * nt / el / 2 ** 20,
                "level_step_us_per_frame": ms[1] / (frames - w0) * 1e3,
                "finite_after": {"frames": frames, "timed_pass": fin},
            })
            print(f"[sweep] {t['table']} {t['size']}^2 H={t['levels']} flow {mf:g}: "
                  f"{rows[-1]['frames_per_s']:.0f} frames/s", flush=True)
    return rows


def cpu_baseline(wl_name, budget_s=20.0):
    """The oracle on the host's cores over a bounded sample of the same workload."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import Filter as Oracle
    from synth.scenes import render_sequence
    from synth.workloads import workload

    wl = workload(wl_name)
    seq = wl["build"]()
    c = seq.camera
    with threadpool_limits(limits=1):
        o = Oracle(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"], wl["smooth"],
                   c.fx, c.fy, c.cx, c.cy)
        Y, R, _ = render_sequence(seq, range(min(20, seq.n_frames)))
        o.push(Y[0].astype(np.float32), R[0].astype(np.float32), seq.dt)   # first frame: init
        t0 = time.perf_counter()
        k = 1
        while k < len(Y):
            o.push(Y[k].astype(np.float32), R[k].astype(np.float32), seq.dt)
            k += 1
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    frames = k - 1
    return {"value": frames / el, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"frames 2..{k} of the {wl_name} workload ({frames} full frames, "
                      f"{el:.1f} s, NumPy FP64, one thread)"}


def _finest_dmu(seq):
    """Tangent-plane pixel spacing of the finest grid (closed form for a pinhole)."""
    import numpy as np
    c = seq.camera
    j = np.arange(seq.cols, dtype=np.float64)[None, :]
    i = np.arange(seq.rows, dtype=np.float64)[:, None]
    x = (j - c.cx) / c.fx
    y = (i - c.cy) / c.fy
    xn = x + np.where(j < seq.cols - 1, 1.0, -1.0) / c.fx
    return np.sqrt(1 + y * y) / np.sqrt(x * x + y * y + 1) / (c.fx * np.sqrt(xn * xn + y * y + 1))


COUNTERS = os.path.join(ROOT, "profiles", "k_step_boxes512_counters.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2406_18031_amd", "csrc", "sflow_kernels.hip")


TRACE = os.path.join(ROOT, "profiles", "k_step_boxes512_trace.md")


def traced_kernel_us():
    """Average duration (us) of the level-step kernel in the committed rocprofv3 kernel trace of
    the boxes512 workload, or None when the kernel source changed since it was taken."""
    import hashlib
    import re
    if not os.path.exists(TRACE):
        return None
    txt = open(TRACE).read()
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if sha not in txt:
        return None
    m = re.search(r"^\| k_step<float[^|]*\| *\d+ *\| *(\d+) *\|", txt, re.M)
    return float(m.group(1)) * 1e-3 if m else None


def measured_counters():
    """Values per level-step launch from the committed rocprofv3 counter summary: HBM bytes
    (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on a plain copy of known size) and
    VALU instructions (SQ_INSTS_VALU), or None when the kernel source changed since the counters
    were taken."""
    import hashlib
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if line.startswith("- ") and " = " in line:
                k, v = line[2:].split(" = ", 1)
                vals[k.strip()] = v.strip().strip("`")
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in vals:
        return None
    return {"traffic": float(vals["traffic_bytes_per_launch"]),
            "valu": float(vals["valu_instructions_per_launch"])
            if "valu_instructions_per_launch" in vals else None}


def copy_probe(mib: int, reps: int = 10, quiet: bool = False):
    """The library's plain streaming copy (sf_copy_probe) of `mib` MiB, timed with HIP events
    on its stream: the achievable HBM bandwidth (bytes read + written per second), and a
    copy of known size for scaling the HBM byte counters."""
    import torch
    from paper_2406_18031_amd import sflow
    n = mib * 2 ** 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.current_stream()
    for _ in range(2):
        sflow.sf_copy_probe(a, b, n, s.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        sflow.sf_copy_probe(a, b, n, s.cuda_stream)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert torch.equal(a[:1024], b[:1024]) and torch.equal(a[-1024:], b[-1024:])
    res = {"copy_bytes_read": n, "copy_bytes_written": n, "launches": reps + 2,
           "us_per_copy": ms * 1e3, "gbs": 2 * n / (ms * 1e-3) / 1e9}
    del a, b
    torch.cuda.empty_cache()
    if not quiet:
        print(json.dumps(res), flush=True)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the 512x512 frame takes about 43 us: 1000 timed frames after 200 untimed ones, so that the
    # clocks and caches have settled before the timed region (100 frames after 10 measured a few
    # per cent low in alternating runs)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="boxes512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16 and batched forms")
    ap.add_argument("--streams", type=int, default=64)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the paper's runtime-table shapes and print them as one "
                         "JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the filter runs on a single device and this build "
              f"has no multi-GPU path (asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.sweep:
        rows = run_sweep(args.steps, args.warmup)
        print(json.dumps({"sweep": rows, "paper": PAPER_TABLES}), flush=True)
        return

    r = run_gpu(args.workload, args.steps, args.warmup, storage=0)
    seq, wl = r["seq"], r["wl"]
    fps = args.steps / r["elapsed"]
    levels = level_table(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"], wl["smooth"])
    step_bytes = sum(L["rows"] * L["cols"] * step_bytes_per_px(L["top"], 4) for L in levels)
    step_flops = sum(L["rows"] * L["cols"] * step_flops_per_px(L["top"], L["N"], L["Ns"])
                     for L in levels)
    step_ms = r["kernel_ms"][1] / max(1, r["kernel_n"][1])
    counters = measured_counters() if args.workload == "boxes512" else None
    achieved_tflops = step_flops / (step_ms * 1e-3) / 1e12
    achieved_gbs = step_bytes / (step_ms * 1e-3) / 1e9
    traced = traced_kernel_us() if args.workload == "boxes512" else None
    copy = copy_probe(4096, quiet=True)      # 4 GiB: far beyond the 256 MB last-level cache

    print(f"[bench] {args.workload}: {fps:.1f} frames/s, level-step kernel {step_ms * 1e3:.2f} us"
          f" ({achieved_gbs:.0f} GB/s algorithmic, {achieved_tflops:.2f} TFLOP/s)", flush=True)

    res = {
        "metric": METRIC,
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {seq.rows}x{seq.cols}, {wl['levels']} levels, max flow "
                        f"{wl['max_flow_px']} px (N={'/'.join(str(L['N']) for L in levels)}), "
                        f"smoothing {'/'.join(str(s) for s in wl['smooth'])}, {seq.n_frames} "
                        f"seeded ray-cast frames at {1 / seq.dt:.0f} Hz, 1% depth noise",
            "storage": "fp32", "update": "plain",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / FP32_PEAK_TFLOPS,
            "traffic": counters["traffic"] if counters else None,
            "kernel": "k_step (fused level step, all levels in one launch)",
            "kernel_us": step_ms * 1e3,
            "algorithmic_flops": step_flops,
            "algorithmic_bytes": step_bytes,
            # the same kernel's average duration in the committed rocprofv3 kernel trace of this
            # workload (null when the kernel source changed since), and the fraction it gives
            "kernel_us_rocprof": traced,
            "frac_rocprof": (step_flops / (traced * 1e-6) / 1e12 / FP32_PEAK_TFLOPS
                             if traced else None),
            "hbm_achieved_gbs": achieved_gbs,
            "hbm_frac": achieved_gbs / HBM_PEAK_GBS,
            # a plain streaming copy of 4 GiB (sf_copy_probe), the bandwidth reachable in practice
            "hbm_copy_gbs": copy["gbs"],
            "hbm_frac_of_copy": achieved_gbs / copy["gbs"],
            "frac_of_unpacked_fp32": achieved_tflops / FP32_UNPACKED_TFLOPS,
            # VALU wave64 instructions retired per SIMD per 4 cycles over the launch
            # (SQ_INSTS_VALU of the committed counters against 256 CUs x 4 SIMDs x 2.4 GHz x
            # the live kernel time / 4), the instructions the FLOP model does not count (halo
            # recomputation, lane shifts, selects) included.  A rate against a nominal one
            # instruction per 4 cycles, not a utilisation: some instructions issue faster, and
            # a long batched launch of this kernel measured 1.13 on it
            "valu_rate_nominal": (counters["valu"] * 4 / (256 * 4 * 2.4e9 * step_ms * 1e-3)
                                  if counters and counters["valu"] else None),
        },
        # HIP events around every launch of a second pass over the same frames: each pair adds
        # about a microsecond, so for the short pyramid and reconstruction launches these are
        # upper bounds (their rocprofv3 durations are the figures to use)
        "kernel_us_per_frame_event_upper_bound": {
            k: v / max(1, n) * 1e3 * n / args.steps for k, v, n in
            zip(("pyramid", "level_step", "reconstruct"), r["kernel_ms"], r["kernel_n"])},
        "paper_context": {"hz": 594.7, "workload": "512x512, 2 levels, max flow 8 px, GTX-780",
                          "source": "Table runtime_pyramid_2"},
        # the method's state grows without bound after O(1000) frames of these cycled inputs
        # (the FP64 oracle too); every pass restarts it and reports that it stayed finite
        "finite_after": r["finite_after"],
        "frame_graph": r["graph"],
        # the same frames declared as produced on a stream of their own (sf_set_input_stream):
        # the pyramid runs beside the previous frame's level step
        "input_stream": r["overlap"],
    }
    print(f"[bench] {args.workload} with an input stream: "
          f"{r['overlap']['steps_per_s']:.1f} frames/s", flush=True)
    forms = {}
    if not args.no_forms:
        import numpy as np
        r16 = run_gpu(args.workload, args.steps, args.warmup, storage=1)
        ms16 = r16["kernel_ms"][1] / max(1, r16["kernel_n"][1])
        dmu = _finest_dmu(seq)
        d = np.sqrt(np.sum((r16["final"] - r["final"]) ** 2, axis=0)) / dmu
        forms["fp16_storage"] = {
            "frames_per_s": args.steps / r16["elapsed"],
            "level_step_us": ms16 * 1e3,
            "level_step_hbm_gbs": sum(L["rows"] * L["cols"] * step_bytes_per_px(L["top"], 2)
                                      for L in levels) / (ms16 * 1e-3) / 1e9,
            "epe_vs_fp32_storage_px": {"mean": float(d.mean()), "max": float(d.max()),
                                       "after_frames": args.warmup + args.steps},
            "finite_after": r16["finite_after"],
        }
        print(f"[bench] fp16 storage: {forms['fp16_storage']['frames_per_s']:.1f} frames/s",
              flush=True)
        for st in (0, 1):
            rb = run_batched(args.streams, max(5, args.steps // 5), max(2, args.warmup // 10),
                             storage=st)
            forms[f"batched_{rb['storage']}"] = rb
            print(f"[bench] batched {rb['storage']}: {rb['aggregate_frames_per_s']:.1f} "
                  f"stream-frames/s ({rb['mpix_per_s']:.0f} Mpix/s)", flush=True)
        rd = run_gpu("driving2048x1024", max(10, args.steps // 2), max(2, args.warmup // 2),
                     storage=1, autotune=True)
        ld = level_table(rd["seq"].rows, rd["seq"].cols, rd["wl"]["levels"], rd["wl"]["max_flow_px"],
                         rd["wl"]["smooth"])
        msd = rd["kernel_ms"][1] / max(1, rd["kernel_n"][1])   # per level-step launch
        launches = rd["kernel_n"][1] / max(1, max(10, args.steps // 2))
        forms["large_2048x1024_fp16"] = {
            "frames_per_s": max(10, args.steps // 2) / rd["elapsed"],
            "level_step_us_per_frame": msd * launches * 1e3,
            "level_step_launches_per_frame": launches,
            "finite_after": rd["finite_after"],
            "level_step_hbm_gbs": sum(L["rows"] * L["cols"] * step_bytes_per_px(L["top"], 2)
                                      for L in ld) / (msd * launches * 1e-3) / 1e9,
            "workload": "2048x1024, 4 levels, max flow 16 px (N=16/8/4/2), driving scene, "
                        "FP16 storage",
            "tuned": {"pass_steps": rd["tuned"]["pass_steps"], "tiles": rd["tuned"]["tiles"]},
        }
        print(f"[bench] large 2048x1024 fp16: {forms['large_2048x1024_fp16']['frames_per_s']:.1f} "
              f"frames/s", flush=True)
        ri = run_inertial(args.steps, args.warmup)
        forms["inertial_boxes512"] = ri
        print(f"[bench] inertial terms: {ri['frames_per_s']:.1f} frames/s; true-flow EPE "
              f"boxes512 {ri['boxes512']['gt_epe_px_inertial']:.4f} px (plain "
              f"{ri['boxes512']['gt_epe_px_plain']:.4f}), 80 % rotation "
              f"{ri['boxes512_rotation80']['gt_epe_px_inertial']:.4f} px (plain "
              f"{ri['boxes512_rotation80']['gt_epe_px_plain']:.4f})", flush=True)
        rg = run_grid_stereo(args.steps, args.warmup)
        forms.update(rg)
        st = rg["stereo_boxes512"]
        print(f"[bench] grid 512x512 with mapping: "
              f"{rg['grid_equiangular_512']['frames_per_s']:.1f} frames/s; stereo: "
              f"{st['frames_per_s']:.1f} frames/s, true-flow EPE {st['gt_epe_px_stereo']:.4f} px "
              f"(depth sensor {st['gt_epe_px_depth']:.4f})", flush=True)
        rl = run_learned(16, max(5, args.steps // 5), max(2, args.warmup // 10))
        forms["learned_16x512"] = rl
        print(f"[bench] learned 16x512: {rl['learned']['aggregate_frames_per_s']:.1f} "
              f"stream-frames/s (plain {rl['plain']['aggregate_frames_per_s']:.1f}); true-flow "
              f"EPE {rl['learned']['gt_epe_px']:.4f} px (plain {rl['plain']['gt_epe_px']:.4f}), "
              f"fallback rate {rl['learned']['fallback_rate']:.3f}", flush=True)
        res["forms"] = forms
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
