"""The learned update trained on the GPU beats the plain update on held-out sequences.

Training data: the filter runs seeded box sequences (textured boxes and planes, constant
linear velocity plus sinusoidal rotation, 1 % depth noise) and exports each frame's network
inputs; the targets are the corrections that reach the true structure flow.  The state does
not depend on the network, so these are the inputs the trained network will see.  The
fallback threshold is chosen on validation seeds (not trained on, not evaluated on) before the
evaluation.  Evaluation: other seeds, the plain and the learned filter side by side, the
endpoint error against the true flow in pixels per frame."""
import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu

R, C, H, MF, SMOOTH = 96, 128, 2, 4.0, [2, 4]
DT = 1.0 / 300.0
N_FRAMES = 24
TRAIN_SEEDS = range(300, 308)
VAL_SEEDS = range(350, 352)
EVAL_SEEDS = range(400, 404)


def _seq(seed):
    from synth.scenes import box_sequence
    return box_sequence(R, C, N_FRAMES, seed=seed, dt=DT, max_flow_px=MF, device="cuda")


def _filter(seq, update, params=None, threshold=-1.0):
    from paper_2406_18031_amd import sflow
    cam = seq.camera
    f = sflow.Filter(R, C, H, MF, SMOOTH, cam.fx, cam.fy, cam.cx, cam.cy, update=update)
    if update == sflow.SF_UPDATE_LEARNED:
        f.set_learned(params, threshold)
    return f


def _frames(seq):
    import torch
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        yield (k, fr.Y.to(torch.float32).contiguous(), fr.rho.to(torch.float32).contiguous(),
               (fr.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous())


def _collect(seeds, params, threshold):
    """Training pairs from the filter's own trajectories with the given parameters."""
    from paper_2406_18031_amd import learned, sflow
    data = []
    for s in seeds:
        seq = _seq(s)
        f = _filter(seq, sflow.SF_UPDATE_LEARNED, params, threshold)
        for k, Y, rho, w in _frames(seq):
            f.push(Y, rho, seq.dt)
            if k >= 1:
                inp, tgt = learned.sample(f.update_inputs(), w)
                data.append((inp.clone(), tgt.clone()))
        f.close()
    return data


def _epe(f, seq, dmu):
    """mean endpoint error (px/frame) against the truth over frames 4.. of the sequence"""
    from paper_2406_18031_amd import sflow
    errs = []
    for k, Y, rho, w in _frames(seq):
        f.push(Y, rho, seq.dt)
        if k >= 4:
            e = (f.flow(sflow.SF_FLOW_W_FRAME) - w).norm(dim=0) / dmu
            errs.append(float(e.mean()))
    return float(np.mean(errs))


def _train(data, params, steps, lr, seed):
    import torch
    from paper_2406_18031_amd import learned
    g = torch.Generator().manual_seed(seed)

    def batches(bs=8):
        for _ in range(steps):
            idx = torch.randperm(len(data), generator=g)[:bs].tolist()
            yield (torch.cat([data[i][0].reshape(-1) for i in idx]),
                   torch.cat([data[i][1].reshape(-1) for i in idx]))

    return learned.train([(R, C)] * 8, batches(), params, lr=lr)


def _evaluate(params, thresholds, seeds):
    from paper_2406_18031_amd import sflow
    plain_e, learned_e, fb_rate = [], {}, {}
    for s in seeds:
        seq = _seq(s)
        probe = _filter(seq, sflow.SF_UPDATE_LEARNED, params, -1.0)
        k, Y, rho, w = next(_frames(seq))
        probe.push(Y, rho, seq.dt)
        probe.push(Y, rho, seq.dt)
        dmu = probe.update_inputs()[21]
        probe.close()
        plain_e.append(_epe(_filter(seq, sflow.SF_UPDATE_PLAIN), seq, dmu))
        for t in thresholds:
            f = _filter(seq, sflow.SF_UPDATE_LEARNED, params, t)
            learned_e.setdefault(t, []).append(_epe(f, seq, dmu))
            fb, px = f.learned_stats()
            fb_rate.setdefault(t, []).append(fb / px)
            f.close()
    return (float(np.mean(plain_e)), {t: float(np.mean(v)) for t, v in learned_e.items()},
            {t: float(np.mean(v)) for t, v in fb_rate.items()})


def test_learned_update_beats_plain():
    from paper_2406_18031_amd import learned
    p0 = learned.init_params(0)
    thresholds = (float("inf"), 1.0, 0.1)
    log("collecting training data")
    data = _collect(TRAIN_SEEDS, p0, -1.0)
    log(f"  {len(data)} frames of {R}x{C}")
    params, losses = _train(data, p0, 300, 2e-3, 0)
    params, l2 = _train(data, params, 200, 5e-4, 1)
    losses += l2
    log(f"  loss {np.mean(losses[:10]):.4f} -> {np.mean(losses[-10:]):.4f}")
    assert np.mean(losses[-10:]) < np.mean(losses[:10])
    _, val, _ = _evaluate(params, thresholds, VAL_SEEDS)
    best = min(thresholds, key=lambda t: val[t] if np.isfinite(val[t]) else np.inf)
    log(f"  validation GT-EPE per threshold {val}: threshold {best}")
    plain, lrn, fb = _evaluate(params, (best,), EVAL_SEEDS)
    log(f"  plain GT-EPE {plain:.4f} px/frame; learned (threshold {best}) {lrn[best]:.4f}, "
        f"fallback rate {fb[best]:.3f}")
    assert lrn[best] <= 1.05 * plain
    assert lrn[best] < plain


def test_committed_parameters_on_a_held_out_stream():
    """The committed trained parameters (trained on the GPU on 9500 frames of 512x512 box
    sequences, seeds 10000-10099; threshold chosen on seeds 15000-15003; both fixed before
    this test was written) on a 512x512 three-level stream of a seed used nowhere else:
    the true-flow endpoint error over frames 10-59 is at most 1.05 x the plain filter's, and
    below it."""
    import torch
    from paper_2406_18031_amd import learned, sflow
    from synth.scenes import box_sequence
    params, threshold = learned.load_trained()
    seq = box_sequence(512, 512, 60, seed=20016, dt=DT, max_flow_px=8.0, device="cuda")
    c = seq.camera
    fs = {}
    for name, upd in (("plain", sflow.SF_UPDATE_PLAIN), ("learned", sflow.SF_UPDATE_LEARNED)):
        f = sflow.Filter(512, 512, 3, 8.0, [2, 4, 4], c.fx, c.fy, c.cx, c.cy, update=upd)
        if upd == sflow.SF_UPDATE_LEARNED:
            f.set_learned(params, threshold)
        fs[name] = f
    err = {"plain": [], "learned": []}
    dmu = None
    for k in range(seq.n_frames):
        fr = seq.frame(k, "cuda")
        Y, rho = fr.Y.to(torch.float32).contiguous(), fr.rho.to(torch.float32).contiguous()
        w = (fr.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32)
        for name, f in fs.items():
            f.push(Y, rho, seq.dt)
        if k >= 1 and dmu is None:
            dmu = fs["learned"].update_inputs()[21].clone()
        if k >= 10:
            for name, f in fs.items():
                e = (f.flow(sflow.SF_FLOW_W_FRAME) - w).norm(dim=0) / dmu
                err[name].append(float(e.mean()))
    fb, px = fs["learned"].learned_stats()
    for f in fs.values():
        f.close()
    plain, lrn = float(np.mean(err["plain"])), float(np.mean(err["learned"]))
    log(f"  held-out 512x512 stream: plain {plain:.4f} px/frame, learned {lrn:.4f} "
        f"(threshold {threshold}, fallback rate {fb / max(1, px):.3f})")
    assert lrn <= 1.05 * plain
    assert lrn < plain
