"""Mapping and stereo depth on a batch context: each stream's calls (sf_set_source_camera,
sf_map_frame, sf_set_stereo, sf_stereo_depth, by stream index) give bitwise what the same
calls give on a context of that stream alone, and the batch's flow after pushing the mapped or
stereo frames is bitwise each single context's.  Both streams are pinhole streams: a batch
that mixes a grid stream with pinhole streams runs every stream's level step from geometry
tables (the pinholes' own rays), which agree with a pinhole context alone to rounding, not
bitwise (the grid forms have their own tests)."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_mapping_and_stereo_on_a_batch():
    import torch
    from paper_2406_18031_amd import sflow
    from synth.scenes import box_sequence
    # stream 0: a 96x80 pinhole camera of a narrower view than the 160x140 pinhole camera whose
    # frames are mapped onto it; stream 1: a 120x150 pinhole stream fed by a stereo pair
    # (baseline 0.15 m, 12 px search)
    src = box_sequence(140, 160, 4, seed=31, max_flow_px=4.0, hfov_deg=80.0, device="cuda")
    ster = box_sequence(120, 150, 4, seed=32, max_flow_px=4.0, device="cuda")
    cs, ct = src.camera, ster.camera
    specs = [dict(rows=96, cols=80, levels=2, max_flow_px=3.0, smooth=[2, 4],
                  camera=(60.0, 60.0, 39.5, 47.5)),
             dict(rows=120, cols=150, levels=3, max_flow_px=4.0, smooth=[2, 4, 4],
                  camera=(ct.fx, ct.fy, ct.cx, ct.cy))]
    batch = sflow.Batch(specs)
    single = [sflow.Filter(96, 80, 2, 3.0, [2, 4], 60.0, 60.0, 39.5, 47.5),
              sflow.Filter(120, 150, 3, 4.0, [2, 4, 4], ct.fx, ct.fy, ct.cx, ct.cy)]
    for ctx, s in ((batch.ctx, 0), (single[0].ctx, 0)):
        sflow.sf_set_source_camera(ctx, s, cs.fx, cs.fy, cs.cx, cs.cy, 140, 160)
    for ctx, s in ((batch.ctx, 1), (single[1].ctx, 0)):
        sflow.sf_set_stereo(ctx, s, 0.15, 12)
    f32 = lambda t: t.to(torch.float32).contiguous()
    for k in range(4):
        fs, ft = src.frame(k, "cuda"), ster.frame(k, "cuda")
        Ys, Rs = f32(fs.Y), f32(fs.rho)
        YL, YR = f32(ft.Y), f32(ster.right_image(k, 0.15, "cuda"))
        outs = {}
        for name, ctx, s0, s1 in (("batch", batch.ctx, 0, 1), ("single", None, 0, 0)):
            c0 = batch.ctx if ctx else single[0].ctx
            c1 = batch.ctx if ctx else single[1].ctx
            Yg = torch.empty((96, 80), device="cuda")
            Rg = torch.empty((96, 80), device="cuda")
            sflow.sf_map_frame(c0, s0, Ys, Rs, Yg, Rg)
            rho = torch.empty((120, 150), device="cuda")
            sflow.sf_stereo_depth(c1, s1, YL, YR, rho)
            outs[name] = (Yg, Rg, rho)
        for a, b, what in zip(outs["batch"], outs["single"], ("mapped Y", "mapped rho", "stereo rho")):
            assert torch.equal(a.nan_to_num(-7.0), b.nan_to_num(-7.0)), (k, what)
        Yg, Rg, rho = outs["batch"]
        batch.push([Yg, YL], [Rg, rho], [src.dt, ster.dt])
        single[0].push(Yg, Rg, src.dt)
        single[1].push(YL, rho, ster.dt)
        for s in range(2):
            assert torch.equal(batch.flow(s), single[s].flow()), (k, s)
        log(f"  frame {k}: mapping, stereo and flow bitwise")
    batch.close()
    for f in single:
        f.close()
