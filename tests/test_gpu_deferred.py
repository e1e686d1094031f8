"""The frame's last reconstruction launch (the one holding the finest level) waits for the next
call that needs the finest flow: sf_get_flow runs it together with the output, a push, a state
read or write, a tiling change or an update-input read runs it on its own.  Every order of calls
gives bitwise the same outputs and state."""
import numpy as np
import pytest

from gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu

R, C, H, MF, SMOOTH = 72, 90, 3, 5.0, [2, 3, 1]
CAM = (80.0, 80.0, 44.5, 35.5)
KINDS = (0, 4, 1, 2)    # rad/s, rad/frame, tangent px, normal px


def _frames(seed, n, rows=R, cols=C, dtype=np.float32):
    rng = np.random.default_rng(seed)
    base = rng.random((rows + 8, cols + 8))
    out = []
    for k in range(n):
        Y = 0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:rows, :cols] + 0.2 * rng.random((rows, cols))
        rho = 0.2 + 0.3 * rng.random((rows, cols))
        rho[rng.random((rows, cols)) < 0.05] = np.nan
        out.append((to_dev(Y, dtype), to_dev(rho, dtype)))
    return out


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(a, b, equal_nan=True)


@pytest.mark.parametrize("storage", [0, 1])
def test_fused_output_equals_separate_output(storage):
    from paper_2406_18031_amd import sflow
    dtype = np.float16 if storage == 1 else np.float32
    log(f"storage {storage}")
    frames = _frames(7, 4, dtype=dtype)
    a = sflow.Filter(R, C, H, MF, SMOOTH, *CAM, storage=storage)
    b = sflow.Filter(R, C, H, MF, SMOOTH, *CAM, storage=storage)
    for k, (Y, rho) in enumerate(frames):
        kind = KINDS[k % len(KINDS)]
        a.push(Y, rho, 0.01)
        b.push(Y, rho, 0.01)
        fused = a.flow(kind)               # reconstruction and output in one launch
        again = a.flow(kind)               # output launch alone
        b.flow(sflow.SF_FLOW_RHO)          # does not need the reconstruction
        b.get_state()                      # runs it alone
        sep = b.flow(kind)
        assert _same(fused, again) and _same(fused, sep), (k, kind)
        for kk in KINDS:
            assert _same(a.flow(kk), b.flow(kk)), (k, kk)
    a.close()
    b.close()


def test_unread_frames_match_read_frames():
    """Pushing without reading (the reconstruction runs at the next push) changes nothing."""
    from paper_2406_18031_amd import sflow
    frames = _frames(8, 5)
    a = sflow.Filter(R, C, H, MF, SMOOTH, *CAM)
    b = sflow.Filter(R, C, H, MF, SMOOTH, *CAM)
    for Y, rho in frames:
        a.push(Y, rho, 0.02)
        a.flow(sflow.SF_FLOW_W_RAD_S)
        b.push(Y, rho, 0.02)
    assert _same(a.flow(), b.flow())
    sa, sb = a.get_state()[0], b.get_state()[0]
    for la, lb in zip(sa, sb):
        for key in la:
            assert np.array_equal(la[key], lb[key], equal_nan=True), key
    a.close()
    b.close()


def test_tiling_change_and_state_write_with_a_pending_reconstruction():
    from paper_2406_18031_amd import sflow
    frames = _frames(9, 4)
    a = sflow.Filter(R, C, H, MF, SMOOTH, *CAM)
    b = sflow.Filter(R, C, H, MF, SMOOTH, *CAM)
    for Y, rho in frames[:3]:
        a.push(Y, rho, 0.01)
        a.flow()
        b.push(Y, rho, 0.01)
    sflow.sf_set_tile(b.ctx, 1, 24, 24)      # relays the levels out: runs the pending launch
    state, dt_prev, nfr = b.get_state()
    c = sflow.Filter(R, C, H, MF, SMOOTH, *CAM)
    c.set_state(state, dt_prev, frames=nfr)
    Y, rho = frames[3]
    for f in (a, b, c):
        f.push(Y, rho, 0.01)
    assert _same(a.flow(), b.flow()) and _same(a.flow(), c.flow())
    for f in (a, b, c):
        f.close()


def test_batch_reads_in_any_order():
    from paper_2406_18031_amd import sflow
    specs = [
        dict(rows=72, cols=90, levels=3, max_flow_px=5.0, smooth=[2, 3, 1], camera=CAM),
        dict(rows=40, cols=33, levels=1, max_flow_px=2.0, smooth=[2], camera=(40.0, 41.0, 16.0, 19.5)),
        dict(rows=130, cols=64, levels=4, max_flow_px=9.0, smooth=[2, 4, 4, 4],
             camera=(70.0, 70.0, 31.5, 64.5)),
        dict(rows=17, cols=23, levels=2, max_flow_px=5.0, smooth=[0, 1], camera=(20.0, 20.0, 11.0, 8.0)),
    ]
    fr = [_frames(20 + s, 3, sp["rows"], sp["cols"]) for s, sp in enumerate(specs)]
    a, b = sflow.Batch(specs), sflow.Batch(specs)
    orders = ([0, 1, 2, 3], [2, 1, 3, 0], [1, 3, 0, 2])
    for k in range(3):
        Ys = [fr[s][k][0] for s in range(len(specs))]
        rhos = [fr[s][k][1] for s in range(len(specs))]
        a.push(Ys, rhos, [0.01] * len(specs))
        b.push(Ys, rhos, [0.01] * len(specs))
        out_a = {s: a.flow(s, sflow.SF_FLOW_W_RAD_S) for s in orders[k]}
        out_b = {s: b.flow(s, sflow.SF_FLOW_W_RAD_S) for s in reversed(orders[k])}
        for s in range(len(specs)):
            assert _same(out_a[s], out_b[s]), (k, s)
    a.close()
    b.close()


def test_learned_correction_in_the_fused_output():
    from paper_2406_18031_amd import learned, sflow
    params = learned.init_params(3, last_scale=1.0)
    frames = _frames(10, 4)
    a = sflow.Filter(R, C, H, MF, SMOOTH, *CAM, update=sflow.SF_UPDATE_LEARNED)
    b = sflow.Filter(R, C, H, MF, SMOOTH, *CAM, update=sflow.SF_UPDATE_LEARNED)
    for f in (a, b):
        f.set_learned(params, float("inf"))
    for k, (Y, rho) in enumerate(frames):
        a.push(Y, rho, 0.01)
        b.push(Y, rho, 0.01)
        fused = a.flow(sflow.SF_FLOW_TANGENT_PX)
        if k > 0:
            b.update_inputs()              # runs the reconstruction alone
        assert _same(fused, b.flow(sflow.SF_FLOW_TANGENT_PX)), k
    fb, px = a.learned_stats()
    assert px > 0 and fb < px
    a.close()
    b.close()


def test_all_streams_in_one_call():
    """sf_get_flows gives bitwise what sf_get_flow_stream gives, stream by stream."""
    import torch
    from paper_2406_18031_amd import sflow
    specs = [
        dict(rows=72, cols=90, levels=3, max_flow_px=5.0, smooth=[2, 3, 1], camera=CAM),
        dict(rows=40, cols=33, levels=1, max_flow_px=2.0, smooth=[2], camera=(40.0, 41.0, 16.0, 19.5)),
        dict(rows=130, cols=64, levels=4, max_flow_px=9.0, smooth=[2, 4, 4, 4],
             camera=(70.0, 70.0, 31.5, 64.5)),
    ]
    fr = [_frames(30 + s, 4, sp["rows"], sp["cols"]) for s, sp in enumerate(specs)]
    a, b = sflow.Batch(specs), sflow.Batch(specs)
    with pytest.raises(sflow.SflowError):
        a.flows()                                   # nothing pushed yet
    for k, kind in enumerate((0, 1, 2, 3)):
        Ys = [fr[s][k][0] for s in range(len(specs))]
        rhos = [fr[s][k][1] for s in range(len(specs))]
        a.push(Ys, rhos, [0.01, 0.02, 0.005])
        b.push(Ys, rhos, [0.01, 0.02, 0.005])
        if k == 2:                                  # a subset: the others stay untouched
            outs = [torch.full((sflow.FLOW_COMPONENTS[kind], sp["rows"], sp["cols"]), 7.0,
                               device="cuda") for sp in specs]
            a.flows(kind, [outs[0], None, outs[2]])
            assert bool((outs[1] == 7.0).all())
            got = [outs[0], a.flow(1, kind), outs[2]]
        else:
            got = a.flows(kind)
        for s in range(len(specs)):
            assert _same(got[s], b.flow(s, kind)), (k, s)
    with pytest.raises(ValueError):
        a.flows(0, [None])
    host = np.zeros(3 * 72 * 90, np.float32)        # a host buffer is refused
    with pytest.raises(sflow.SflowError):
        sflow.sf_get_flows(a.ctx, 0, [host.ctypes.data, None, None])
    with pytest.raises(sflow.SflowError):                # unknown kind
        sflow.sf_get_flows(a.ctx, 9, a.flows(0))
    a.close()
    b.close()
