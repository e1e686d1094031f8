"""Train the learned update's network on the GPU and evaluate it against the plain update.

    python -m paper_2406_18031_amd.train [--size 512] [--train-seqs 100] [--train-frames 100]
        [--train-skip 5] [--steps 6000] [--val-streams 4] [--eval-streams 16]
        [--eval-frames 100] [--out weights.npz]

Training data: seeded box sequences (the synthetic ray-cast generator; seeds 10000 + i) run
through a batch of plain-state learned contexts, which export each frame's network inputs;
targets are the corrections that reach the true structure flow (paper_2406_18031_amd.learned).
The inputs are kept in BF16 on the device (they are BF16 values already: the filter exports
them as the network reads them), the targets in FP32.
Threshold: the fallback threshold with the lowest true-flow error on validation sequences
(seeds 15000 + i), chosen before any evaluation sequence is run.
Evaluation: held-out sequences (seeds 20000 + i) through a plain batch and a learned batch at
the chosen threshold (and, for the record, the other candidates), endpoint error against the
true flow in pixels per frame after a warm-up, fallback rates and aggregate frames/s.
Writes the parameters and the threshold to --out (npz: params float32, threshold float64) and
prints one JSON line.  Every numeric step runs in the library's kernels; this module arranges
tensors.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _specs(seqs, levels, max_flow, smooth):
    out = []
    for seq in seqs:
        c = seq.camera
        out.append(dict(rows=seq.rows, cols=seq.cols, levels=levels, max_flow_px=max_flow,
                        smooth=smooth, camera=(c.fx, c.fy, c.cx, c.cy)))
    return out


def _frame(seq, k):
    import torch
    f = seq.frame(k, "cuda")
    return (f.Y.to(torch.float32).contiguous(), f.rho.to(torch.float32).contiguous(),
            (f.w_gt * seq.dt).permute(2, 0, 1).to(torch.float32).contiguous())


def collect(seqs, specs, params, skip=1):
    import torch
    from . import learned, sflow
    b = sflow.Batch(specs, update=sflow.SF_UPDATE_LEARNED)
    b.set_learned(params, -1.0)
    data = []
    for k in range(seqs[0].n_frames):
        fr = [_frame(s, k) for s in seqs]
        b.push([f[0] for f in fr], [f[1] for f in fr], [s.dt for s in seqs])
        if k >= max(1, skip):
            for i, f in enumerate(fr):
                inp, tgt = learned.sample(b.update_inputs(i), f[2])
                data.append((inp.to(torch.bfloat16), tgt.clone()))
    b.close()
    return data


def evaluate(seqs, specs, params, thresholds, warm):
    import torch
    from . import sflow
    ctxs = {"plain": sflow.Batch(specs)}
    for t in thresholds:
        b = sflow.Batch(specs, update=sflow.SF_UPDATE_LEARNED)
        b.set_learned(params, t)
        ctxs[t] = b
    err = {key: [] for key in ctxs}
    elapsed = {key: 0.0 for key in ctxs}
    dmu = None
    for k in range(seqs[0].n_frames):
        fr = [_frame(s, k) for s in seqs]
        for key, b in ctxs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.push([f[0] for f in fr], [f[1] for f in fr], [s.dt for s in seqs])
            torch.cuda.synchronize()
            elapsed[key] += time.perf_counter() - t0
            if dmu is None and key != "plain" and k >= 1:
                dmu = [b.update_inputs(i)[21].clone() for i in range(len(seqs))]
            if k >= warm and dmu is not None:
                e = [float(((b.flow(i, sflow.SF_FLOW_W_FRAME) - f[2]).norm(dim=0) / dmu[i]).mean())
                     for i, f in enumerate(fr)]
                err[key].append(float(np.mean(e)))
    out = {}
    for key, b in ctxs.items():
        row = {"gt_epe_px": float(np.mean(err[key])),
               "frames_per_s": len(seqs) * seqs[0].n_frames / elapsed[key]}
        if key != "plain":
            fb, px = b.learned_stats()
            row["fallback_rate"] = fb / max(1, px)
        out["plain" if key == "plain" else f"learned_threshold_{key}"] = row
        b.close()
    return out


def choose_threshold(seqs, specs, params, candidates, warm):
    """The candidate with the lowest true-flow error on the validation sequences."""
    res = evaluate(seqs, specs, params, candidates, warm)
    scores = {t: res[f"learned_threshold_{t}"]["gt_epe_px"] for t in candidates}
    return min(candidates, key=lambda t: scores[t]), scores


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--levels", type=int, default=3)
    ap.add_argument("--max-flow", type=float, default=8.0)
    ap.add_argument("--train-seqs", type=int, default=100)
    ap.add_argument("--train-frames", type=int, default=100)
    ap.add_argument("--train-skip", type=int, default=5, help="first frame used for training")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--val-streams", type=int, default=4)
    ap.add_argument("--val-frames", type=int, default=50)
    ap.add_argument("--eval-streams", type=int, default=16)
    ap.add_argument("--eval-frames", type=int, default=100)
    ap.add_argument("--warm", type=int, default=10)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    from synth.scenes import box_sequence
    from . import learned

    smooth = [2] + [4] * (args.levels - 1)
    dt = 1.0 / 300.0
    t0 = time.perf_counter()
    p0 = learned.init_params(0)
    data = []
    for first in range(0, args.train_seqs, 16):   # up to 16 streams per collection batch
        seqs = [box_sequence(args.size, args.size, args.train_frames, seed=10000 + i, dt=dt,
                             max_flow_px=args.max_flow, device="cuda")
                for i in range(first, min(first + 16, args.train_seqs))]
        data += collect(seqs, _specs(seqs, args.levels, args.max_flow, smooth), p0,
                        args.train_skip)
        print(f"[train] collected {len(data)} frames ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    params, l1 = learned.train([(args.size, args.size)] * 8, _batches(data, args.steps, 0), p0,
                               lr=2e-3)
    params, l2 = learned.train([(args.size, args.size)] * 8,
                               _batches(data, args.steps // 3, 1), params, lr=5e-4)
    print(f"[train] loss {np.mean(l1[:20]):.4f} -> {np.mean(l2[-20:]):.4f} "
          f"({time.perf_counter() - t0:.0f} s)", flush=True)
    n_train = len(data)
    del data
    candidates = (float("inf"), 3.0, 1.0, 0.3, 0.1)
    vseqs = [box_sequence(args.size, args.size, args.val_frames, seed=15000 + i, dt=dt,
                          max_flow_px=args.max_flow, device="cuda")
             for i in range(args.val_streams)]
    threshold, scores = choose_threshold(vseqs, _specs(vseqs, args.levels, args.max_flow, smooth),
                                         params, candidates, args.warm)
    print(f"[train] validation GT-EPE per threshold {scores}: threshold {threshold}",
          flush=True)
    if args.out:
        np.savez(args.out, params=np.asarray(params, np.float32),
                 threshold=np.float64(threshold))
    seqs = [box_sequence(args.size, args.size, args.eval_frames, seed=20000 + i, dt=dt,
                         max_flow_px=args.max_flow, device="cuda")
            for i in range(args.eval_streams)]
    others = tuple(t for t in candidates if t != threshold)
    res = evaluate(seqs, _specs(seqs, args.levels, args.max_flow, smooth), params,
                   (threshold,) + others, args.warm)
    res["threshold"] = threshold
    res["config"] = {"size": args.size, "levels": args.levels, "max_flow_px": args.max_flow,
                     "train": f"{args.train_seqs} sequences x {args.train_frames} frames "
                              f"(from frame {args.train_skip}: {n_train} frames), seeds 10000+, "
                              f"{args.steps} + {args.steps // 3} Adam steps of 8",
                     "validation": f"{args.val_streams} streams x {args.val_frames} frames, "
                                   f"seeds 15000+",
                     "eval": f"{args.eval_streams} streams x {args.eval_frames} frames, seeds "
                             f"20000+, endpoint error over frames {args.warm}.."}
    print(json.dumps(res), flush=True)


def _batches(data, steps, seed, bs=8):
    import torch
    g = torch.Generator().manual_seed(seed)
    for _ in range(steps):
        idx = torch.randperm(len(data), generator=g)[:bs].tolist()
        yield (torch.cat([data[i][0].reshape(-1) for i in idx]).float(),
               torch.cat([data[i][1].reshape(-1) for i in idx]))


if __name__ == "__main__":
    main()
