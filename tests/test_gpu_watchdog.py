"""The state watchdog (sf_check_state): a stored flow value that is not finite sets the stream's
bit, the check reports and clears it, and setting the cameras restarts it.  Non-finite state is
produced from the host's side by a frame with infinite brightness at a few pixels (the image
model's gradient there is inf - inf); every kernel runs to its end as usual."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def _frames(rng, R, C, n):
    import torch
    base = rng.random((R + 8, C + 8))
    Ys, Rs = [], []
    for k in range(n):
        Ys.append(0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:R, :C] + 0.2 * rng.random((R, C)))
        Rs.append(0.2 + 0.3 * rng.random((R, C)))
    return ([torch.tensor(y, dtype=torch.float32).cuda() for y in Ys],
            [torch.tensor(r, dtype=torch.float32).cuda() for r in Rs])


def _poisoned(Y):
    Yb = Y.clone()
    Yb[10:12, 20:23] = float("inf")
    return Yb


@pytest.mark.parametrize("storage", [0, 1])
def test_single_stream(storage):
    """96x128, three levels: clean frames pass the check; a frame with infinite brightness
    makes the next check fail, and the check after it fails again while the state holds the
    non-finite values; after setting the camera the clean frames pass again."""
    import torch
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(81)
    R, C = 96, 128
    cam = (110.0, 110.0, 63.5, 47.5)
    Ys, Rs = _frames(rng, R, C, 8)
    if storage == 1:
        Ys, Rs = [y.half() for y in Ys], [r.half() for r in Rs]
    f = sflow.Filter(R, C, 3, 4.0, [2, 4, 4], *cam, storage=storage)
    for k in range(4):
        f.push(Ys[k], Rs[k], 0.01)
    assert f.check_state()
    assert sflow.sf_check_state(f.ctx) == 0
    f.push(_poisoned(Ys[4]), Rs[4], 0.01)
    f.push(Ys[5], Rs[5], 0.01)
    out = f.flow(sflow.SF_FLOW_W_FRAME)
    torch.cuda.synchronize()
    assert not bool(torch.isfinite(out).all())
    with pytest.raises(sflow.SflowError) as e:
        sflow._check(sflow.lib.sf_check_state(f.ctx, sflow.ctypes.byref(sflow.ctypes.c_uint64())),
                     f.ctx)
    assert e.value.status == sflow.SF_ERR_NUMERIC and "not finite" in str(e.value)
    f.push(Ys[6], Rs[6], 0.01)            # the state is still non-finite: flagged again
    assert sflow.sf_check_state(f.ctx) == 1
    sflow.sf_set_camera(f.ctx, *cam)      # restart
    for k in range(3):
        f.push(Ys[k], Rs[k], 0.01)
    assert f.check_state()
    assert bool(torch.isfinite(f.flow(sflow.SF_FLOW_W_FRAME)).all())
    log(f"  storage {storage}: flagged after the poisoned frame, clean after the restart")
    f.close()


def test_batch_names_the_stream():
    """Three streams of different sizes and levels; only stream 1 receives the poisoned
    frame, so only its bit is set."""
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(82)
    specs = [dict(rows=96, cols=128, levels=3, max_flow_px=4.0, smooth=[2, 4, 4],
                  camera=(110.0, 110.0, 63.5, 47.5)),
             dict(rows=70, cols=60, levels=2, max_flow_px=3.0, smooth=[2, 2],
                  camera=(60.0, 62.0, 29.5, 34.5)),
             dict(rows=40, cols=40, levels=1, max_flow_px=2.0, smooth=[2],
                  camera=(40.0, 40.0, 19.5, 19.5))]
    data = [_frames(rng, sp["rows"], sp["cols"], 5) for sp in specs]
    b = sflow.Batch(specs)
    for k in range(3):
        b.push([d[0][k] for d in data], [d[1][k] for d in data], [0.01] * 3)
    assert b.check_state() == []
    ys = [d[0][3] for d in data]
    ys[1] = _poisoned(ys[1])
    b.push(ys, [d[1][3] for d in data], [0.01] * 3)
    b.push([d[0][4] for d in data], [d[1][4] for d in data], [0.01] * 3)
    assert b.check_state() == [1]
    sflow.sf_set_cameras(b.ctx, [sp["camera"] for sp in specs])
    for k in range(3):
        b.push([d[0][k] for d in data], [d[1][k] for d in data], [0.01] * 3)
    assert b.check_state() == []
    b.close()


def test_learned_update_is_watched():
    """A learned context, whose finest level is stored by the network-and-choice kernel."""
    from paper_2406_18031_amd import learned, sflow
    rng = np.random.default_rng(83)
    R, C = 64, 96
    f = sflow.Filter(R, C, 2, 3.0, [2, 2], 90.0, 90.0, 47.5, 31.5,
                     update=sflow.SF_UPDATE_LEARNED)
    f.set_learned(learned.init_params(3, last_scale=1.0), 0.5)
    Ys, Rs = _frames(rng, R, C, 6)
    for k in range(3):
        f.push(Ys[k], Rs[k], 0.01)
    assert f.check_state()
    f.push(_poisoned(Ys[3]), Rs[3], 0.01)
    f.push(Ys[4], Rs[4], 0.01)
    assert not f.check_state()
    f.close()
