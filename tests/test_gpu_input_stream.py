"""Frame inputs produced on a stream of the caller's (sf_set_input_stream): the pyramid runs on
the library's own stream beside the previous frame's level step, and the results are bitwise
those of a context that orders everything on its own stream.  The frames are copied into two
alternating buffer sets on the input stream just before each push, with no synchronisation
between frames, so that a push that ordered its reads wrongly, or a buffer rewritten while a
level step still reads it, would show up as a difference."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _frames(rng, R, C, n, nan_frac=0.05):
    import torch
    base = rng.random((R + 16, C + 16))
    Ys, Rs = [], []
    for k in range(n):
        Y = 0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:R, :C] + 0.2 * rng.random((R, C))
        rho = 0.2 + 0.3 * rng.random((R, C))
        rho[rng.random((R, C)) < nan_frac] = np.nan
        Ys.append(Y)
        Rs.append(rho)
    return (torch.tensor(np.stack(Ys), dtype=torch.float32).cuda(),
            torch.tensor(np.stack(Rs), dtype=torch.float32).cuda())


class _Feeder:
    """Two buffer sets per camera stream, filled on the input stream frame after frame."""

    def __init__(self, shapes, dtype):
        import torch
        self.s = torch.cuda.Stream()
        self.buf = [[(torch.empty(sh, dtype=dtype, device="cuda"),
                      torch.empty(sh, dtype=dtype, device="cuda")) for sh in shapes]
                    for _ in range(2)]

    def fill(self, k, Ys, Rs):
        import torch
        sets = self.buf[k % 2]
        with torch.cuda.stream(self.s):
            for (y, r), Y, R in zip(sets, Ys, Rs):
                y.copy_(Y)
                r.copy_(R)
        return [y for y, _ in sets], [r for _, r in sets]


@pytest.mark.parametrize("storage", [0, 1])
def test_single_stream_matches_the_default_mode(storage):
    """192x160, three levels, a dt change, 12 frames; every frame's flow and inverse depth
    kept in its own output and compared after the last frame."""
    import torch
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(71 + storage)
    R, C, n = 192, 160, 12
    cam = (150.0, 150.0, 79.5, 95.5)
    dtype = torch.float16 if storage == 1 else torch.float32
    Ys, Rs = _frames(rng, R, C, n)
    Ys, Rs = Ys.to(dtype), Rs.to(dtype)
    ref = sflow.Filter(R, C, 3, 6.0, [2, 4, 4], *cam, storage=storage)
    ovl = sflow.Filter(R, C, 3, 6.0, [2, 4, 4], *cam, storage=storage)
    feed = _Feeder([(R, C)], dtype)
    ovl.set_input_stream(feed.s)
    torch.cuda.synchronize()
    dts = [0.01] * 6 + [0.02] * 6
    out = {name: torch.empty((n, 3, R, C), device="cuda") for name in ("ref", "ovl")}
    rho = {name: torch.empty((n, 1, R, C), device="cuda") for name in ("ref", "ovl")}
    for k in range(n):
        ref.push(Ys[k], Rs[k], dts[k])
        y, r = feed.fill(k, [Ys[k]], [Rs[k]])
        ovl.push(y[0], r[0], dts[k])
        for name, f in (("ref", ref), ("ovl", ovl)):
            f.flow(sflow.SF_FLOW_W_FRAME, out=out[name][k])
            f.flow(sflow.SF_FLOW_RHO, out=rho[name][k])
    torch.cuda.synchronize()
    for k in range(n):
        assert torch.equal(out["ref"][k], out["ovl"][k]), ("frame", k)
        assert torch.equal(rho["ref"][k].nan_to_num(-1), rho["ovl"][k].nan_to_num(-1)), ("rho", k)
    log(f"  storage {storage}: {n} frames bitwise")
    ref.close()
    ovl.close()


@pytest.mark.parametrize("mode", ["plain", "graph", "timing"])
def test_batch_matches_the_default_mode(mode):
    """Three streams of different sizes and levels; with frame graphs or kernel timing on the
    pyramid stays on the context stream, which then waits for the input stream."""
    import torch
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(73)
    specs = [dict(rows=96, cols=128, levels=3, max_flow_px=4.0, smooth=[2, 4, 4],
                  camera=(110.0, 110.0, 63.5, 47.5)),
             dict(rows=70, cols=60, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(60.0, 62.0, 29.5, 34.5)),
             dict(rows=40, cols=40, levels=1, max_flow_px=2.0, smooth=[2],
                  camera=(40.0, 40.0, 19.5, 19.5))]
    n = 8
    data = [_frames(rng, sp["rows"], sp["cols"], n) for sp in specs]
    ref, ovl = sflow.Batch(specs), sflow.Batch(specs)
    feed = _Feeder([(sp["rows"], sp["cols"]) for sp in specs], torch.float32)
    ovl.set_input_stream(feed.s)
    if mode == "graph":
        sflow.sf_set_graph(ovl.ctx, True)
    if mode == "timing":
        sflow.sf_set_timing(ovl.ctx, True)
    outs = {name: [[torch.empty((3, sp["rows"], sp["cols"]), device="cuda") for sp in specs]
                   for _ in range(n)] for name in ("ref", "ovl")}
    torch.cuda.synchronize()
    for k in range(n):
        ref.push([d[0][k] for d in data], [d[1][k] for d in data], [0.01] * 3)
        ys, rs = feed.fill(k, [d[0][k] for d in data], [d[1][k] for d in data])
        ovl.push(ys, rs, [0.01] * 3)
        for name, b in (("ref", ref), ("ovl", ovl)):
            b.flows(sflow.SF_FLOW_W_FRAME, outs=outs[name][k])
    torch.cuda.synchronize()
    for k in range(n):
        for s in range(3):
            assert torch.equal(outs["ref"][k][s], outs["ovl"][k][s]), (mode, "frame", k, s)
    ref.close()
    ovl.close()


def test_learned_and_switching_streams():
    """The learned update with the input stream set from the third frame and unset again at
    the seventh: every frame bitwise, fallback counts equal."""
    import torch
    from paper_2406_18031_amd import learned, sflow
    rng = np.random.default_rng(74)
    R, C, n = 64, 96, 9
    cam = (90.0, 90.0, 47.5, 31.5)
    p = learned.init_params(3, last_scale=1.0)
    fs = [sflow.Filter(R, C, 2, 3.0, [2, 2], *cam, update=sflow.SF_UPDATE_LEARNED)
          for _ in range(2)]
    ref, ovl = fs
    for f in fs:
        f.set_learned(p, 0.5)
    Ys, Rs = _frames(rng, R, C, n)
    feed = _Feeder([(R, C)], torch.float32)
    outs = {name: torch.empty((n, 3, R, C), device="cuda") for name in ("ref", "ovl")}
    torch.cuda.synchronize()
    for k in range(n):
        if k == 2:
            ovl.set_input_stream(feed.s)
        if k == 6:
            ovl.set_input_stream(None)
        ref.push(Ys[k], Rs[k], 0.01)
        if 2 <= k < 6:
            y, r = feed.fill(k, [Ys[k]], [Rs[k]])
            ovl.push(y[0], r[0], 0.01)
        else:
            ovl.push(Ys[k], Rs[k], 0.01)
        for name, f in (("ref", ref), ("ovl", ovl)):
            f.flow(sflow.SF_FLOW_W_FRAME, out=outs[name][k])
    torch.cuda.synchronize()
    for k in range(n):
        assert torch.equal(outs["ref"][k], outs["ovl"][k]), ("frame", k)
    assert ref.learned_stats() == ovl.learned_stats()
    for f in fs:
        f.close()
