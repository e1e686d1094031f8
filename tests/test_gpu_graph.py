"""Frame graphs (sf_set_graph): a context that replays its captured frame graph gives bitwise
the results of a context that enqueues the same launches one by one, frame after frame, with
the program's own eager work and synchronisations between the replays; also after the layout
changes that make it capture again (tiles, pass length, learned parameters), across a state
restore, with and without inertial rates, for batches and FP16 storage."""
import numpy as np
import pytest

from gpu_helpers import log, to_dev

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


def _busy():
    """Eager work of the program between replays (its own kernels and a synchronisation)."""
    import torch
    a = torch.randn(257, 263, device="cuda")
    float((a * 2.0 + 1.0).sum())
    torch.cuda.synchronize()


def _equal_outputs(a, b, what, kinds=None):
    import torch
    from paper_2406_18031_amd import sflow
    for kind in kinds or (sflow.SF_FLOW_W_FRAME, sflow.SF_FLOW_RHO):
        x, y = a(kind), b(kind)
        assert torch.equal(x, y), (what, kind, float((x - y).abs().max()))


@pytest.mark.parametrize("storage", [0, 1])
def test_single_stream_graph_equals_eager(storage):
    """150x131, three levels, the finest prediction split into passes (pass length 2), a dt
    change, a tile change and a pass-length change mid-sequence (both make it capture again),
    inertial rates on some frames (the second pair of graphs), a state restore."""
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(61 + storage)
    R, C = 150, 131
    cam = (120.0, 110.0, 64.2, 73.9)
    dtype = "float16" if storage == 1 else "float32"
    ctx = [sflow.Filter(R, C, 3, 6.0, [2, 3, 1], *cam, storage=storage) for _ in range(2)]
    eager, graph = ctx
    sflow.sf_set_graph(graph.ctx, True)
    for f in ctx:
        sflow.sf_set_pass_steps(f.ctx, 2)
    frames = _frames(rng, R, C, 12)
    dts = [0.01] * 5 + [0.02] * 7
    om, acc = np.array([1.0, -0.5, 0.8]), np.array([3.0, 0.0, -2.0])
    dom = np.array([10.0, -5.0, 2.0])
    blob = None
    for k, (Y, rho) in enumerate(frames):
        y, r = to_dev(Y, dtype), to_dev(rho, dtype)
        rates = k in (3, 4, 8)
        if k == 6:
            for f in ctx:
                sflow.sf_set_tile(f.ctx, 1, 24, 20)
        if k == 9:
            for f in ctx:
                sflow.sf_set_pass_steps(f.ctx, 8)
        if k == 10:
            for f in ctx:
                f.set_state(*blob)
        log(f"  frame {k} storage {storage} rates {rates}")
        for f in ctx:
            if rates:
                f.push(y, r, dts[k], omega=om, acc=acc, omega_dot=dom)
            else:
                f.push(y, r, dts[k])
        _busy()
        _equal_outputs(lambda kd: eager.flow(kd), lambda kd: graph.flow(kd), ("frame", k))
        if k == 7:
            blob = eager.get_state()
    for f in ctx:
        f.close()


def test_batch_graph_equals_eager():
    """A batch of three streams of different sizes and levels: every stream's output, every
    frame, bitwise."""
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(63)
    specs = [dict(rows=96, cols=128, levels=3, max_flow_px=4.0, smooth=[2, 4, 4],
                  camera=(110.0, 110.0, 63.5, 47.5)),
             dict(rows=70, cols=60, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(60.0, 62.0, 29.5, 34.5)),
             dict(rows=40, cols=40, levels=1, max_flow_px=2.0, smooth=[2],
                  camera=(40.0, 40.0, 19.5, 19.5))]
    eager, graph = sflow.Batch(specs), sflow.Batch(specs)
    sflow.sf_set_graph(graph.ctx, True)
    frames = [_frames(rng, sp["rows"], sp["cols"], 8) for sp in specs]
    for k in range(8):
        ys = [to_dev(frames[s][k][0]) for s in range(3)]
        rs = [to_dev(frames[s][k][1]) for s in range(3)]
        for b in (eager, graph):
            b.push(ys, rs, [0.01] * 3)
        _busy()
        for s in range(3):
            _equal_outputs(lambda kd: eager.flow(s, kd), lambda kd: graph.flow(s, kd),
                           ("frame", k, "stream", s))
    eager.close()
    graph.close()


def test_learned_graph_equals_eager():
    """The learned update's launches (network layers, choice and smoothing) in the graph; a
    new threshold mid-sequence makes it capture again; fallback counts agree."""
    from paper_2406_18031_amd import learned, sflow
    rng = np.random.default_rng(64)
    specs = [dict(rows=64, cols=96, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(90.0, 90.0, 47.5, 31.5)),
             dict(rows=48, cols=48, levels=2, max_flow_px=3.0, smooth=[2, 3],
                  camera=(50.0, 50.0, 23.5, 23.5))]
    p = learned.init_params(3, last_scale=1.0)
    bs = [sflow.Batch(specs, update=sflow.SF_UPDATE_LEARNED) for _ in range(2)]
    eager, graph = bs
    sflow.sf_set_graph(graph.ctx, True)
    for b in bs:
        b.set_learned(p, 0.5)
    frames = [_frames(rng, sp["rows"], sp["cols"], 7) for sp in specs]
    for k in range(7):
        if k == 4:
            for b in bs:
                b.set_learned(p, 0.05)
        ys = [to_dev(frames[s][k][0]) for s in range(2)]
        rs = [to_dev(frames[s][k][1]) for s in range(2)]
        for b in bs:
            b.push(ys, rs, [0.01] * 2)
        _busy()
        for s in range(2):
            _equal_outputs(lambda kd: eager.flow(s, kd), lambda kd: graph.flow(s, kd),
                           ("frame", k, "stream", s))
    assert eager.learned_stats() == graph.learned_stats()
    for b in bs:
        b.close()


def test_disabling_releases_and_returns_to_eager():
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(65)
    R, C = 50, 70
    cam = (60.0, 60.0, 34.5, 24.5)
    eager = sflow.Filter(R, C, 2, 3.0, [2, 2], *cam)
    graph = sflow.Filter(R, C, 2, 3.0, [2, 2], *cam)
    for k, (Y, rho) in enumerate(_frames(rng, R, C, 6)):
        sflow.sf_set_graph(graph.ctx, k < 3 or k == 5)
        y, r = to_dev(Y), to_dev(rho)
        eager.push(y, r, 0.01)
        graph.push(y, r, 0.01)
        _equal_outputs(lambda kd: eager.flow(kd), lambda kd: graph.flow(kd), ("frame", k))
    eager.close()
    graph.close()
