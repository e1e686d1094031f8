"""Inverse depth from a rectified stereo pair on the GPU (sf_set_stereo, sf_stereo_depth)
against the oracle (oracle/stereo.py), and the filter running on the stereo pair alone."""
import numpy as np
import pytest

from gpu_helpers import compare_outputs, log, to_dev

pytestmark = pytest.mark.gpu


def _box_scene(S, seed=6, n=1):
    from synth.scenes import box_sequence
    return box_sequence(S, S, n, seed=seed, max_flow_px=4.0, device="cuda")


@pytest.mark.parametrize("storage", [0, 1])
def test_stereo_depth_against_the_oracle(storage):
    """A rendered 256x256 box scene (baseline 0.2 m, disparities 0.5-5 px) and a 200x120 crop of
    it (ragged tiles, its own principal point): the integer search must agree exactly (any disagreement moves the result
    by a pixel), the refined disparity kappa rho within 2e-3 px (float32 against float64
    refinement; FP16 storage: the output's rounding), the missing pixels the same up to 1e-3
    of the image (threshold ties)."""
    import torch
    from oracle import stereo
    from paper_2406_18031_amd import sflow
    S, b = 256, 0.2
    seq = _box_scene(S)
    c = seq.camera
    fr = seq.frame(0, "cuda")
    dtype = torch.float16 if storage == 1 else torch.float32
    YL_full = fr.Y.to(dtype)
    YR_full = seq.right_image(0, b, "cuda").to(dtype)
    for (r0, c0, R, C) in ((0, 0, S, S), (40, 50, 120, 200)):
        YL = YL_full[r0:r0 + R, c0:c0 + C].contiguous()
        YR = YR_full[r0:r0 + R, c0:c0 + C].contiguous()
        cam = (c.fx, c.fy, c.cx - c0, c.cy - r0)
        f = sflow.Filter(R, C, 1, 1.0, [1], *cam, storage=storage)
        f.set_stereo(b, 8)
        rho = f.stereo_depth(YL, YR).float().cpu().numpy().astype(np.float64)
        f.close()
        want = stereo.stereo_rho(YL.float().cpu().numpy(), YR.float().cpu().numpy(), *cam, b, 8)
        k = stereo.kappa(R, C, *cam, b)
        both = ~np.isnan(rho) & ~np.isnan(want)
        flips = np.isnan(rho) != np.isnan(want)
        err = np.abs(k[both] * (rho[both] - want[both]))
        tol = 2e-2 if storage == 1 else 2e-3
        log(f"  {R}x{C} storage {storage}: {both.mean():.3f} measured, {flips.mean():.2e} "
            f"flipped, disparity error max {err.max():.2e} px")
        assert flips.mean() <= 1e-3
        assert err.max() <= tol


def test_filter_on_a_stereo_pair_alone():
    """The 256x256 box scene through the filter (three levels) with its inverse depth taken
    from the stereo pair every frame: every output kind against the oracle filter fed the same
    measurements; and its endpoint error against the true flow over frames 5-19 within 1.2x
    that of the filter fed the scene's depth (1 % noise)."""
    import torch
    from oracle import Filter as OFilter
    from paper_2406_18031_amd import sflow
    S, b = 256, 0.2
    seq = _box_scene(S, n=20)
    c = seq.camera
    cam = (c.fx, c.fy, c.cx, c.cy)
    g = sflow.Filter(S, S, 3, 4.0, [2, 4, 4], *cam)
    g.set_stereo(b, 8)
    d = sflow.Filter(S, S, 3, 4.0, [2, 4, 4], *cam)
    o = OFilter(S, S, 3, 4.0, [2, 4, 4], *cam)
    x = (torch.arange(S, device="cuda", dtype=torch.float64)[None, :] - c.cx) / c.fx
    y = (torch.arange(S, device="cuda", dtype=torch.float64)[:, None] - c.cy) / c.fy
    xn = x + torch.where(torch.arange(S, device="cuda")[None, :] < S - 1, 1.0, -1.0) / c.fx
    dmu = torch.sqrt(1 + y * y) / torch.sqrt(x * x + y * y + 1) / (c.fx * torch.sqrt(xn * xn + y * y + 1))
    err = {"stereo": [], "depth": []}
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        Y = fr.Y.to(torch.float32).contiguous()
        YR = seq.right_image(k, b, "cuda").to(torch.float32).contiguous()
        rho = g.stereo_depth(Y, YR)
        g.push(Y, rho, seq.dt)
        d.push(Y, fr.rho.to(torch.float32).contiguous(), seq.dt)
        if k < 4:
            o.push(Y.cpu().double().numpy(), rho.cpu().double().numpy(), seq.dt)
            compare_outputs(g, o, 0, f"frame {k}")
        if k >= 5:
            w = (fr.w_gt * seq.dt).permute(2, 0, 1)
            for name, f in (("stereo", g), ("depth", d)):
                e = (f.flow(sflow.SF_FLOW_W_FRAME).double() - w).norm(dim=0) / dmu
                err[name].append(float(e.mean()))
    g.close()
    d.close()
    es, ed = float(np.mean(err["stereo"])), float(np.mean(err["depth"]))
    log(f"  true-flow EPE: stereo {es:.4f} px, depth sensor {ed:.4f} px")
    assert es <= 1.2 * ed


def test_stereo_needs_parameters_and_a_pinhole():
    from paper_2406_18031_amd import sflow
    from synth.scenes import equiangular_rays
    f = sflow.Filter(16, 16, 1, 1.0, [1], 16.0, 16.0, 7.5, 7.5)
    y = to_dev(np.zeros((16, 16)))
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_stereo_depth(f.ctx, 0, y, y, y)
    assert ei.value.status == sflow.SF_ERR_STATE
    with pytest.raises(sflow.SflowError) as ei:
        f.set_stereo(0.1, 65)
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    f.close()
    g = sflow.Filter(16, 16, 1, 1.0, [1], 16.0, 16.0, 7.5, 7.5, eta=equiangular_rays(16, 16, 90.0))
    g.set_stereo(0.1, 4)
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_stereo_depth(g.ctx, 0, y, y, y)
    assert ei.value.status == sflow.SF_ERR_UNSUPPORTED
    g.close()
