"""GPU parity of the prediction with the inertial source terms (sf_push_frame_ex,
sf_push_frames_ex; eq:hflow_conservation without eq:assumption) against the FP64 oracle, and
what the terms gain against the true flow of a rotating camera.

Bars as in test_gpu_parity: every output kind per frame, mean and 99th percentile of the
endpoint error at most 1e-3 px (FP32 storage) or 2e-2 px (FP16), the largest pixel at most
10x that."""
import numpy as np
import pytest

from gpu_helpers import compare_outputs, log, make_pair, rounded, to_dev

pytestmark = pytest.mark.gpu

OMEGA = np.array([1.0, -0.7, 1.5])       # rad/s
DOMEGA = np.array([-30.0, 12.0, 20.0])   # rad/s^2
ACC = np.array([20.0, 5.0, -10.0])       # m/s^2


def _frames(rng, R, C, n, nan_frac=0.05):
    out = []
    base = rng.random((R + 8, C + 8))
    for k in range(n):
        Y = 0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:R, :C] + 0.2 * rng.random((R, C))
        rho = 0.2 + 0.3 * rng.random((R, C))
        rho[rng.random((R, C)) < nan_frac] = np.nan
        out.append((Y, rho))
    return out


def test_ragged_three_levels_with_inertial_terms():
    """150x131, three levels with ragged tiles, missing depth, a dt change, rates (angular
    velocity and acceleration) that change from frame to frame; FP32 storage (the per-pixel
    noise of these frames is no input for the FP16 bar, see the rendered scene below)."""
    storage = 0
    rng = np.random.default_rng(41)
    R, C = 150, 131
    cam = (120.0, 110.0, 64.2, 73.9)
    o, g = make_pair(R, C, 3, 6.0, [2, 3, 1], cam, storage=storage)
    dtype = "float16" if storage == 1 else "float32"
    dts = [0.01, 0.01, 0.01, 0.02, 0.02]
    for k, (Y, rho) in enumerate(_frames(rng, R, C, len(dts))):
        om = OMEGA * (1.0 + 0.3 * k)
        dom = DOMEGA * (1.0 - 0.1 * k)
        acc = ACC * (1.0 - 0.2 * k)
        log(f"  frame {k} {R}x{C} H=3 storage={storage} omega={om} omega_dot={dom} acc={acc}")
        g.push(to_dev(Y, dtype), to_dev(rho, dtype), dts[k], omega=om, acc=acc, omega_dot=dom)
        o.push(rounded(Y, storage), rounded(rho, storage), dts[k], omega=om, acc=acc,
               omega_dot=dom)
        compare_outputs(g, o, storage, f"frame {k}")
    g.close()


@pytest.mark.parametrize("storage", [0, 1])
def test_rotating_box_scene_with_inertial_terms(storage):
    """A rendered 150x131 box scene whose image motion is mostly camera rotation, three levels
    with ragged tiles, the rates the camera's inertial unit would report (synth), FP32 and FP16
    storage: every output kind of every frame against the oracle."""
    import torch
    from synth.scenes import box_sequence
    seq = box_sequence(150, 131, 6, seed=7, max_flow_px=6.0, rot_share=0.8, device="cuda")
    c = seq.camera
    o, g = make_pair(150, 131, 3, 6.0, [2, 4, 4], (c.fx, c.fy, c.cx, c.cy), storage=storage)
    dtype = torch.float16 if storage == 1 else torch.float32
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        Y, rho = fr.Y.to(dtype).contiguous(), fr.rho.to(dtype).contiguous()
        om, dom, acc = seq.imu(k)
        log(f"  frame {k} rotating boxes 150x131 storage={storage} omega={om}")
        g.push(Y, rho, seq.dt, omega=om, acc=acc, omega_dot=dom)
        o.push(Y.cpu().double().numpy(), rho.cpu().double().numpy(), seq.dt, omega=om, acc=acc,
               omega_dot=dom)
        compare_outputs(g, o, storage, f"frame {k}")
    g.close()


def test_zero_rates_equal_the_plain_push():
    """Zero rates through the inertial kernel give the plain push's flow (the terms add zeros);
    NULL rates are the plain push itself."""
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(43)
    R, C = 70, 90
    cam = (80.0, 80.0, 44.5, 34.5)
    a = sflow.Filter(R, C, 2, 3.0, [2, 2], *cam)
    b = sflow.Filter(R, C, 2, 3.0, [2, 2], *cam)
    c = sflow.Filter(R, C, 2, 3.0, [2, 2], *cam)
    for k, (Y, rho) in enumerate(_frames(rng, R, C, 4)):
        y, r = to_dev(Y), to_dev(rho)
        a.push(y, r, 0.01)
        b.push(y, r, 0.01, omega=np.zeros(3), acc=np.zeros(3), omega_dot=np.zeros(3))
        sflow.sf_push_frame_ex(c.ctx, y, r, 0.01, None, None, None)
        fa = a.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
        np.testing.assert_array_equal(fa, b.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy())
        np.testing.assert_array_equal(fa, c.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy())
    for f in (a, b, c):
        f.close()


def test_batch_rates_per_stream():
    """A batch whose streams get different rates: each stream bitwise equal to the same
    stream run alone with its own rates."""
    import torch
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(44)
    specs = [dict(rows=60, cols=80, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(70.0, 70.0, 39.5, 29.5)),
             dict(rows=45, cols=45, levels=3, max_flow_px=4.0, smooth=[1, 2, 2],
                  camera=(50.0, 52.0, 22.0, 22.0))]
    batch = sflow.Batch(specs)
    alone = [sflow.Filter(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                          *sp["camera"]) for sp in specs]
    frames = [_frames(rng, sp["rows"], sp["cols"], 4) for sp in specs]
    oms = [OMEGA, -0.5 * OMEGA[::-1]]
    doms = [np.zeros(3), DOMEGA]
    accs = [ACC, np.zeros(3)]
    for k in range(4):
        ys = [to_dev(frames[s][k][0]) for s in range(2)]
        rs = [to_dev(frames[s][k][1]) for s in range(2)]
        batch.push(ys, rs, [0.01, 0.01], omegas=np.stack(oms), accs=np.stack(accs),
                   omega_dots=np.stack(doms))
        for s in range(2):
            alone[s].push(ys[s], rs[s], 0.01, omega=oms[s], acc=accs[s], omega_dot=doms[s])
            got = batch.flow(s, sflow.SF_FLOW_W_FRAME)
            want = alone[s].flow(sflow.SF_FLOW_W_FRAME)
            assert torch.equal(got, want), (k, s)
    batch.close()
    for f in alone:
        f.close()


def test_rates_are_validated():
    from paper_2406_18031_amd import sflow
    f = sflow.Filter(16, 16, 1, 1.0, [1], 16.0, 16.0, 7.5, 7.5)
    y = to_dev(np.zeros((16, 16)))
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_push_frame_ex(f.ctx, y, y, 0.01, [0.0, np.nan, 0.0], None, None)
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_push_frame_ex(f.ctx, y, y, 0.01, None, [0.0, 0.0, np.inf], None)
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_push_frame_ex(f.ctx, y, y, 0.01, None, None, [np.inf, 0.0, 0.0])
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    f.close()


def _boxes512(n):
    import torch
    from synth.workloads import workload
    wl = workload("boxes512")
    seq = wl["build"]("cuda")
    frames = []
    for k in range(n):
        fr = seq.frame(k, "cuda")
        frames.append((fr.Y.to(torch.float32).contiguous(), fr.rho.to(torch.float32).contiguous(),
                       (fr.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous()))
    return wl, seq, frames


def test_boxes512_with_the_renderers_rates_against_the_oracle():
    """The 512x512 three-level workload (sinusoidal angular velocity) with the rates the camera's
    inertial unit would report (synth: angular velocity at mid-interval, zero acceleration),
    every pixel of every output kind over six frames against the oracle."""
    wl, seq, frames = _boxes512(6)
    c = seq.camera
    o, g = make_pair(seq.rows, seq.cols, wl["levels"], wl["max_flow_px"], wl["smooth"],
                     (c.fx, c.fy, c.cx, c.cy))
    for k, (Y, rho, _) in enumerate(frames):
        om, dom, acc = seq.imu(k)
        log(f"  frame {k} boxes512 omega {om}")
        g.push(Y, rho, seq.dt, omega=om, acc=acc, omega_dot=dom)
        o.push(Y.cpu().numpy().astype(np.float64), rho.cpu().numpy().astype(np.float64), seq.dt,
               omega=om, acc=acc, omega_dot=dom)
        compare_outputs(g, o, 0, f"frame {k}")
    g.close()


def test_inertial_terms_lower_the_true_error_under_rotation():
    """A 512x512 three-level box scene whose image motion is mostly camera rotation (80 %;
    the bench's boxes512 has 20 %), 40 frames, with the rates (angular velocity and its rate of
    change) the camera's inertial unit would report: the mean endpoint error against the true
    flow over frames 10-39 is lower with the inertial terms than with the paper's prediction
    without them."""
    import torch
    from paper_2406_18031_amd import sflow
    from synth.scenes import box_sequence
    seq = box_sequence(512, 512, 40, seed=31, max_flow_px=8.0, rot_share=0.8, device="cuda")
    c = seq.camera
    frames = []
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        frames.append((fr.Y.to(torch.float32).contiguous(), fr.rho.to(torch.float32).contiguous(),
                       (fr.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous()))
    x = (torch.arange(seq.cols, device="cuda", dtype=torch.float64)[None, :] - c.cx) / c.fx
    y = (torch.arange(seq.rows, device="cuda", dtype=torch.float64)[:, None] - c.cy) / c.fy
    xn = x + torch.where(torch.arange(seq.cols, device="cuda")[None, :] < seq.cols - 1, 1.0,
                         -1.0) / c.fx
    # tangent-plane spacing of the pinhole grid in closed form
    dmu = torch.sqrt(1 + y * y) / torch.sqrt(x * x + y * y + 1) / (c.fx * torch.sqrt(xn * xn + y * y + 1))
    res = {}
    for use in (False, True):
        f = sflow.Filter(512, 512, 3, 8.0, [2, 4, 4], c.fx, c.fy, c.cx, c.cy)
        e = []
        for k, (Y, rho, w) in enumerate(frames):
            if use:
                om, dom, acc = seq.imu(k)
                f.push(Y, rho, seq.dt, omega=om, acc=acc, omega_dot=dom)
            else:
                f.push(Y, rho, seq.dt)
            if k >= 10:
                e.append(float(((f.flow(sflow.SF_FLOW_W_FRAME).double() - w.double())
                                .norm(dim=0) / dmu).mean()))
        f.close()
        res[use] = float(np.mean(e))
    log(f"  true-flow EPE over frames 10-39: plain {res[False]:.4f} px, inertial {res[True]:.4f} px")
    assert res[True] < res[False], res
