"""Batches of camera streams (one launch per stage for all streams): each stream of a batch
gives bitwise the result of the same stream run alone, and matches the oracle."""
import numpy as np
import pytest

from gpu_helpers import check_bar, epe_px, log, to_dev

pytestmark = pytest.mark.gpu

SPECS = [
    dict(rows=72, cols=90, levels=3, max_flow_px=5.0, smooth=[2, 3, 1],
         camera=(80.0, 80.0, 44.5, 35.5)),
    dict(rows=40, cols=33, levels=1, max_flow_px=2.0, smooth=[2], camera=(40.0, 41.0, 16.0, 19.5),
         read_flags=1 | 2),
    dict(rows=130, cols=64, levels=4, max_flow_px=9.0, smooth=[2, 4, 4, 4],
         camera=(70.0, 70.0, 31.5, 64.5)),
    # no stability clamp: the motion (2.2 px/frame, doubled by the dt change) stays within the
    # bound N >= |flow| of the prediction; beyond it the unclamped scheme diverges
    dict(rows=17, cols=23, levels=2, max_flow_px=5.0, smooth=[0, 1], camera=(20.0, 20.0, 11.0, 8.0),
         read_flags=4),
]


def _frames(rng, sp, n):
    R, C = sp["rows"], sp["cols"]
    base = rng.random((R + 8, C + 8))
    out = []
    for k in range(n):
        Y = 0.6 * np.roll(base, (k, 2 * k), axis=(0, 1))[:R, :C] + 0.2 * rng.random((R, C))
        rho = 0.2 + 0.3 * rng.random((R, C))
        rho[rng.random((R, C)) < 0.05] = np.nan
        out.append((Y.astype(np.float32), rho.astype(np.float32)))
    return out


def test_batch_matches_single_streams_and_oracle():
    from oracle import Filter as Oracle, Readings
    from paper_2406_18031_amd import sflow
    rng = np.random.default_rng(31)
    nfr = 4
    frames = [_frames(rng, sp, nfr) for sp in SPECS]
    dts = [[0.01, 0.01, 0.02, 0.02], [1.0] * 4, [0.005] * 4, [0.1, 0.2, 0.2, 0.1]]
    log("batch of", len(SPECS), "streams")
    batch = sflow.Batch(SPECS)
    singles = [sflow.Filter(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                            *sp["camera"], read_flags=sp.get("read_flags", 0)) for sp in SPECS]
    oracles = []
    for sp in SPECS:
        f = sp.get("read_flags", 0)
        oracles.append(Oracle(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                              *sp["camera"], readings=Readings(bool(f & 1), bool(f & 2), not f & 4)))
    for k in range(nfr):
        dev = [(to_dev(frames[s][k][0]), to_dev(frames[s][k][1])) for s in range(len(SPECS))]
        log("  frame", k)
        batch.push([d[0] for d in dev], [d[1] for d in dev], [dts[s][k] for s in range(len(SPECS))])
        for s in range(len(SPECS)):
            singles[s].push(dev[s][0], dev[s][1], dts[s][k])
            oracles[s].push(frames[s][k][0].astype(np.float64), frames[s][k][1].astype(np.float64),
                            dts[s][k])
        for s in range(len(SPECS)):
            wb = batch.flow(s, sflow.SF_FLOW_W_RAD_S).cpu().numpy()
            ws = singles[s].flow(sflow.SF_FLOW_W_RAD_S).cpu().numpy()
            assert np.array_equal(wb, ws), (k, s)
            e = epe_px(wb.transpose(1, 2, 0) * dts[s][k], oracles[s].flow("w_frame"),
                       oracles[s].grids[0].dmu)
            check_bar(e, 0, ("frame", k, "stream", s))
    batch.close()
    for f in singles:
        f.close()


def test_batch_call_rules():
    from paper_2406_18031_amd import sflow
    cfgs = [sflow.make_config(16, 16, 1, 1.0, [1]), sflow.make_config(20, 16, 2, 2.0, [1, 1])]
    ctx = sflow.sf_create_batch(cfgs)
    assert sflow.sf_stream_count(ctx) == 2
    Y = to_dev(np.zeros((16, 16)))
    with pytest.raises(sflow.SflowError) as e:
        sflow.sf_push_frame(ctx, Y, Y, 1.0)
    assert e.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as e:
        sflow.sf_set_camera(ctx, 10.0, 10.0, 7.5, 7.5)
    assert e.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as e:
        sflow.sf_push_frames(ctx, [Y, Y], [Y, Y], [1.0, 1.0])
    assert e.value.status == sflow.SF_ERR_STATE
    sflow.sf_destroy(ctx)
    mixed = [sflow.make_config(16, 16, 1, 1.0, [1]),
             sflow.make_config(16, 16, 1, 1.0, [1], storage=sflow.SF_FP16)]
    with pytest.raises(sflow.SflowError) as e:
        sflow.sf_create_batch(mixed)
    assert e.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as e:
        sflow.sf_create_batch([sflow.make_config(16, 16, 1, 1.0, [1])] * 65)
    assert e.value.status == sflow.SF_ERR_INVALID_ARG


def test_autotuned_launch_shape_keeps_results():
    """The autotuner only changes tiles and pass lengths, which never change the result: a
    tuned batch gives bitwise the output of an untuned one."""
    from paper_2406_18031_amd import sflow, tune
    rng = np.random.default_rng(41)
    specs = SPECS[:3]
    frames = [_frames(rng, sp, 5) for sp in specs]
    dev = [[(to_dev(Y), to_dev(r)) for Y, r in fr] for fr in frames]
    dts = [0.01] * len(specs)
    plain = sflow.Batch(specs)
    tuned = sflow.Batch(specs)

    def push(b, k):
        b.push([d[k % 5][0] for d in dev], [d[k % 5][1] for d in dev], dts)

    big = specs[2]
    lv, r_, c_ = [], big["rows"], big["cols"]
    for h in range(big["levels"]):
        lv.append(dict(rows=r_, cols=c_, max_flow_px=big["max_flow_px"], smooth=big["smooth"][h],
                       h=h))
        r_, c_ = (r_ + 1) // 2, (c_ + 1) // 2
    setting = tune.tune(tuned.ctx, lambda k: push(tuned, k), lv, pass_steps=(3, 8), frames=2,
                        warmup=1)
    log("tuned:", {k: v for k, v in setting.items() if k != "trials"})
    # restart both streams from the same first frame
    cams = [sp["camera"] for sp in specs]
    sflow.sf_set_cameras(plain.ctx, cams)
    sflow.sf_set_cameras(tuned.ctx, cams)
    for k in range(5):
        push(plain, k)
        push(tuned, k)
        for s in range(len(specs)):
            a = plain.flow(s, sflow.SF_FLOW_W_FRAME).cpu().numpy()
            b = tuned.flow(s, sflow.SF_FLOW_W_FRAME).cpu().numpy()
            assert np.array_equal(a, b), (k, s)


@pytest.mark.parametrize("storage", [0, 1])
def test_large_batch_reconstruction_tile(storage):
    """A batch whose finest reconstruction covers at least 4096 16 x 16 tiles runs it on 32 x 32
    tiles (four pixels per thread); a stream alone runs it on 16 x 16 tiles.  Both give bitwise
    the same flow and state, on ragged sizes, with and without a parent above the upper level."""
    from paper_2406_18031_amd import sflow
    dtype = np.float16 if storage == 1 else np.float32
    kinds = [
        dict(rows=250, cols=270, levels=3, max_flow_px=8.0, smooth=[2, 4, 4],
             camera=(200.0, 200.0, 134.5, 124.5)),          # 272 tiles at level 0
        dict(rows=301, cols=199, levels=2, max_flow_px=4.0, smooth=[2, 3],
             camera=(180.0, 180.0, 99.0, 150.0)),           # 247, the upper level is the top
        dict(rows=333, cols=250, levels=4, max_flow_px=16.0, smooth=[2, 4, 4, 4],
             camera=(220.0, 220.0, 124.5, 166.0)),          # 336
        dict(rows=100, cols=100, levels=1, max_flow_px=2.0, smooth=[2],
             camera=(60.0, 60.0, 49.5, 49.5)),              # no reconstruction
    ]
    specs = kinds * 5
    tiles = sum(((sp["rows"] + 15) // 16) * ((sp["cols"] + 15) // 16)
                for sp in specs if sp["levels"] >= 2)
    assert tiles >= 4096 and all(((sp["rows"] + 15) // 16) * ((sp["cols"] + 15) // 16) < 4096
                                 for sp in specs)
    rng = np.random.default_rng(57)
    nfr = 3
    frames = [_frames(rng, sp, nfr) for sp in specs]
    log(f"storage {storage}: batch of {len(specs)} streams, {tiles} tiles")
    batch = sflow.Batch(specs, storage=storage)
    singles = [sflow.Filter(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                            *sp["camera"], storage=storage) for sp in specs]
    for k in range(nfr):
        dev = [(to_dev(fr[k][0], dtype), to_dev(fr[k][1], dtype)) for fr in frames]
        dts = [0.01 * (1 + (s + k) % 3) for s in range(len(specs))]
        batch.push([d[0] for d in dev], [d[1] for d in dev], dts)
        for s, f in enumerate(singles):
            f.push(dev[s][0], dev[s][1], dts[s])
        got = batch.flows(sflow.SF_FLOW_W_FRAME)
        for s, f in enumerate(singles):
            a, b = got[s].cpu().numpy(), f.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (k, s)
    for s, f in enumerate(singles):
        sa, sb = batch.get_state(s)[0], f.get_state()[0]
        for la, lb in zip(sa, sb):
            for key in la:
                assert np.array_equal(la[key], lb[key], equal_nan=True), (s, key)
    batch.close()
    for f in singles:
        f.close()


@pytest.mark.parametrize("storage", [0, 1])
def test_stream_mix_workload(storage):
    """The 64-stream mix (256x256, 512x512 and 1024x1024 box scenes, 3-4 levels) at full size in
    the launch configuration the bench times (autotuned pass length and tiles, outputs of all
    streams in one call): every stream bitwise equal to the stream run alone, and the first
    256x256 and 512x512 streams (in FP32 storage also the first two frames of the first
    1024x1024 one, about 30 s of oracle time) against the oracle on every pixel."""
    import torch
    from oracle import Filter as Oracle
    from paper_2406_18031_amd import sflow, tune
    from synth.workloads import stream_mix
    from gpu_helpers import rounded

    nfr = 3
    dtype = torch.float16 if storage == 1 else torch.float32
    mix = stream_mix(64, n_frames=nfr, device="cuda")
    specs, frames, dt = [], [], None
    for m in mix:
        seq = m["build"]()
        c = seq.camera
        specs.append(dict(rows=seq.rows, cols=seq.cols, levels=m["levels"],
                          max_flow_px=m["max_flow_px"], smooth=m["smooth"],
                          camera=(c.fx, c.fy, c.cx, c.cy)))
        fr = []
        for k in range(nfr):
            f = seq.frame(k, "cuda")
            fr.append((f.Y.to(dtype).contiguous(), f.rho.to(dtype).contiguous()))
        frames.append(fr)
        dt = seq.dt
    log(f"storage {storage}: {len(specs)} streams, sizes",
        sorted({sp['rows'] for sp in specs}))
    batch = sflow.Batch(specs, storage=storage)
    dts = [dt] * len(specs)

    def push(k):
        batch.push([fr[k % nfr][0] for fr in frames], [fr[k % nfr][1] for fr in frames], dts)

    big = max(specs, key=lambda sp: sp["rows"] * sp["cols"])
    lv, r_, c_ = [], big["rows"], big["cols"]
    for h in range(big["levels"]):
        lv.append(dict(rows=r_, cols=c_, max_flow_px=big["max_flow_px"], smooth=big["smooth"][h],
                       h=h))
        r_, c_ = (r_ + 1) // 2, (c_ + 1) // 2
    setting = tune.tune(batch.ctx, push, lv)
    log("tuned:", setting["pass_steps"], setting["tiles"])
    sflow.sf_set_cameras(batch.ctx, [sp["camera"] for sp in specs])    # restart every stream
    singles = [sflow.Filter(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                            *sp["camera"], storage=storage) for sp in specs]
    sizes = [sp["rows"] for sp in specs]
    checked = {sizes.index(256): nfr, sizes.index(512): nfr}
    if storage == 0:
        checked[sizes.index(1024)] = 2
    oracles = {s: Oracle(specs[s]["rows"], specs[s]["cols"], specs[s]["levels"],
                         specs[s]["max_flow_px"], specs[s]["smooth"], *specs[s]["camera"])
               for s in checked}
    for k in range(nfr):
        log(f"  frame {k}")
        push(k)
        for s, f in enumerate(singles):
            f.push(frames[s][k][0], frames[s][k][1], dt)
        got = batch.flows(sflow.SF_FLOW_W_FRAME)
        for s, f in enumerate(singles):
            a, b = got[s].cpu().numpy(), f.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
            assert np.array_equal(a, b, equal_nan=True), (k, s)
        for s, o in oracles.items():
            if k >= checked[s]:
                continue
            Y, rho = (v.to(torch.float32).cpu().numpy() for v in frames[s][k])
            o.push(rounded(Y, storage), rounded(rho, storage), dt)
            e = epe_px(got[s].cpu().numpy().transpose(1, 2, 0), o.flow("w_frame"),
                       o.grids[0].dmu)
            log(f"    stream {s} ({sizes[s]}^2) EPE mean {e['mean']:.2e} p99 {e['p99']:.2e} "
                f"max {e['max']:.2e}")
            check_bar(e, storage, ("frame", k, "stream", s))
    batch.close()
    for f in singles:
        f.close()
