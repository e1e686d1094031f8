"""General grids of directions (sf_camera.eta; Section "Spherical image data structure") on the
GPU against the FP64 oracle on the same grid.

Bars as in test_gpu_parity: every output kind per frame, mean and 99th percentile of the
endpoint error at most 1e-3 px (FP32 storage) or 2e-2 px (FP16), the largest pixel at most
10x that."""
import numpy as np
import pytest

from gpu_helpers import compare_outputs, log, rounded, to_dev

pytestmark = pytest.mark.gpu


def _frames(rng, R, C, n, nan_frac=0.05):
    out = []
    base = rng.random((R + 8, C + 8))
    for k in range(n):
        Y = 0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:R, :C] + 0.2 * rng.random((R, C))
        rho = 0.2 + 0.3 * rng.random((R, C))
        rho[rng.random((R, C)) < nan_frac] = np.nan
        out.append((Y, rho))
    return out


def _pair(R, C, H, mf, smooth, cam, eta, storage=0):
    from oracle import Filter as OFilter
    from paper_2406_18031_amd import sflow
    o = OFilter(R, C, H, mf, smooth, *cam, eta=eta)
    g = sflow.Filter(R, C, H, mf, smooth, *cam, storage=storage, eta=eta)
    return o, g


@pytest.mark.parametrize("which", ["equiangular", "pinhole_rays"])
def test_ragged_three_levels_on_a_grid(which):
    """150x131, three levels with ragged tiles, missing depth, a dt change: a 110-degree
    equiangular grid, and the pinhole's own rays given as a grid (the table path on a grid
    the closed forms also describe)."""
    from oracle import geometry
    from synth.scenes import equiangular_rays
    rng = np.random.default_rng(71)
    R, C = 150, 131
    cam = (90.0, 90.0, 64.2, 73.9)
    eta = (equiangular_rays(R, C, 110.0) if which == "equiangular"
           else geometry.pinhole_eta(R, C, *cam))
    o, g = _pair(R, C, 3, 6.0, [2, 3, 1], cam, eta)
    dts = [0.01, 0.01, 0.01, 0.02, 0.02]
    for k, (Y, rho) in enumerate(_frames(rng, R, C, len(dts))):
        log(f"  frame {k} {R}x{C} H=3 {which}")
        g.push(to_dev(Y), to_dev(rho), dts[k])
        o.push(rounded(Y, 0), rounded(rho, 0), dts[k])
        compare_outputs(g, o, 0, f"frame {k}")
    g.close()


def _grid_box_sequence(R, C, n, seed, hfov):
    """A rendered box scene seen through an equiangular grid of the same field of view."""
    from synth.scenes import GridCamera, box_sequence, equiangular_rays
    seq = box_sequence(R, C, n, seed=seed, max_flow_px=6.0, device="cuda", hfov_deg=hfov)
    c = seq.camera
    seq.camera = GridCamera(R, C, c.fx, c.fy, c.cx, c.cy, eta=equiangular_rays(R, C, hfov))
    seq._eta = {}
    return seq


@pytest.mark.parametrize("storage", [0, 1])
def test_rendered_scene_on_an_equiangular_grid(storage):
    """A rendered box scene through a 100-degree equiangular grid, FP32 and FP16 storage."""
    import torch
    R, C = 150, 131
    seq = _grid_box_sequence(R, C, 6, 8, 100.0)
    c = seq.camera
    o, g = _pair(R, C, 3, 6.0, [2, 4, 4], (c.fx, c.fy, c.cx, c.cy), seq.camera.eta, storage)
    dtype = torch.float16 if storage == 1 else torch.float32
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        Y, rho = fr.Y.to(dtype).contiguous(), fr.rho.to(dtype).contiguous()
        log(f"  frame {k} equiangular boxes storage={storage}")
        g.push(Y, rho, seq.dt)
        o.push(Y.cpu().double().numpy(), rho.cpu().double().numpy(), seq.dt)
        compare_outputs(g, o, storage, f"frame {k}")
    g.close()


def test_batch_with_grid_and_pinhole_streams():
    """A batch whose first stream has a grid and whose second is a pinhole: both against the
    oracle; the grid stream bitwise equal to itself run alone."""
    import torch
    from oracle import Filter as OFilter
    from paper_2406_18031_amd import sflow
    from synth.scenes import equiangular_rays
    rng = np.random.default_rng(72)
    eta = equiangular_rays(60, 80, 120.0)
    specs = [dict(rows=60, cols=80, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(40.0, 40.0, 39.5, 29.5), eta=eta),
             dict(rows=45, cols=45, levels=3, max_flow_px=4.0, smooth=[1, 2, 2],
                  camera=(50.0, 52.0, 22.0, 22.0))]
    batch = sflow.Batch(specs)
    alone = sflow.Filter(60, 80, 2, 3.0, [2, 2], 40.0, 40.0, 39.5, 29.5, eta=eta)
    oracles = [OFilter(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                       *sp["camera"], eta=sp.get("eta")) for sp in specs]
    frames = [_frames(rng, sp["rows"], sp["cols"], 4) for sp in specs]
    for k in range(4):
        ys = [to_dev(frames[s][k][0]) for s in range(2)]
        rs = [to_dev(frames[s][k][1]) for s in range(2)]
        batch.push(ys, rs, [0.01, 0.01])
        alone.push(ys[0], rs[0], 0.01)
        assert torch.equal(batch.flow(0, sflow.SF_FLOW_W_FRAME), alone.flow(sflow.SF_FLOW_W_FRAME))
        for s in range(2):
            oracles[s].push(rounded(frames[s][k][0], 0), rounded(frames[s][k][1], 0), 0.01)

            class _One:   # the batch's stream s seen through the single-stream interface
                def flow(self, kind, s=s):
                    return batch.flow(s, kind)
            compare_outputs(_One(), oracles[s], 0, f"frame {k} stream {s}")
    batch.close()
    alone.close()


def test_invalid_grids_are_refused():
    from paper_2406_18031_amd import sflow
    from synth.scenes import equiangular_rays
    f = sflow.Filter(16, 16, 1, 1.0, [1], 16.0, 16.0, 7.5, 7.5)
    eta = equiangular_rays(16, 16, 90.0)
    bad = eta * 1.01
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_set_camera(f.ctx, 16.0, 16.0, 7.5, 7.5, bad)
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    dup = eta.copy()
    dup[:, 5] = dup[:, 4]
    with pytest.raises(sflow.SflowError) as ei:
        sflow.sf_set_camera(f.ctx, 16.0, 16.0, 7.5, 7.5, dup)
    assert ei.value.status == sflow.SF_ERR_INVALID_ARG
    sflow.sf_set_camera(f.ctx, 16.0, 16.0, 7.5, 7.5, eta)     # a valid grid is taken
    f.close()
