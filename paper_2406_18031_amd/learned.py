"""The learned update: parameter layout, training targets and a GPU training loop.

Everything numeric runs in the library (include/sflow.h, sections "learned update" and
"training the learned update's network"): the filter writes each frame's network inputs,
the network object runs forward, loss, backward and Adam on the matrix cores.  This module
only arranges tensors.  At the finest level the network corrects the output flow of the
paper's update step (Section "State update"), the smoothed least-squares solution, where the
least-squares cost of the correction stays under a threshold; the filter's state and
recurrence stay the plain ones.
"""
from __future__ import annotations

import os
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import sflow

CHANNELS = (9, 16, 16, 16, 3)
N_PARAMS = sflow.SF_LEARNED_PARAMS
# parameters and fallback threshold trained for the 512x512 three-level box workload
# (python -m paper_2406_18031_amd.train --out <this file>; seeds and command in the design notes)
TRAINED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "learned_boxes512.npz")


def load_trained(path: str = TRAINED):
    """(parameters float32[N_PARAMS], threshold) from a file written by train.py."""
    with np.load(path, allow_pickle=False) as z:
        p = np.asarray(z["params"], dtype=np.float32)
        t = float(z["threshold"])
    if p.shape != (N_PARAMS,) or not np.all(np.isfinite(p)):
        raise ValueError(f"{path}: expected {N_PARAMS} finite parameters")
    return p, t


def layer_slices():
    """[(weight slice, weight shape, bias slice)] of the flat parameter vector."""
    out, off = [], 0
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        nw = 9 * cin * cout
        out.append((slice(off, off + nw), (3, 3, cin, cout), slice(off + nw, off + nw + cout)))
        off += nw + cout
    assert off == N_PARAMS
    return out


def init_params(seed: int = 0, last_scale: float = 0.1) -> np.ndarray:
    """He-normal weights, zero biases; the last layer scaled down so that a fresh network
    makes small corrections."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS, dtype=np.float32)
    sl = layer_slices()
    for li, (ws, shape, _) in enumerate(sl):
        std = np.sqrt(2.0 / (9 * shape[2]))
        w = rng.standard_normal(int(np.prod(shape))) * std
        if li == len(sl) - 1:
            w *= last_scale
        p[ws] = w.astype(np.float32)
    return p


def split_params(p: np.ndarray) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat vector -> [(W (3, 3, cin, cout), b)] per layer."""
    p = np.asarray(p)
    return [(p[ws].reshape(shape), p[bs]) for ws, shape, bs in layer_slices()]


def join_params(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([np.asarray(W).reshape(-1), np.asarray(b).reshape(-1)])
                           for W, b in layers]).astype(np.float32)


def sample(update_inputs, w_frame):
    """Network input (9, R, C) and target output (3, R, C) of one frame.

    update_inputs: the 22 planes of sf_get_update_inputs; w_frame: the true structure flow
    of that frame in rad/frame, (3, R, C).  The target is the correction (pixels per frame)
    that takes the smoothed least-squares field to the true one: (w - parent - S(x_ls)) / dmu.
    """
    xs = update_inputs[15:18]
    parent = update_inputs[18:21]
    dmu = update_inputs[21]
    return update_inputs[0:9], (w_frame - parent - xs) / dmu


def train(sizes: Sequence[Tuple[int, int]], batches: Iterable, params: np.ndarray,
          lr: float = 2e-3, stream=None, log_every: int = 0, loss_eps: float = 1e-3):
    """Adam over `batches`, an iterable of (inputs, targets) device tensors laid out as the
    network object expects (images one after the other, inputs [9][R][C], targets [3][R][C]).
    Returns (parameters, losses)."""
    net = sflow.Net(sizes, params, stream, loss_eps)
    losses = []
    try:
        for k, (inp, tgt) in enumerate(batches):
            loss, _ = net.train_step(inp, tgt, lr)
            losses.append(loss)
            if log_every and k % log_every == 0:
                print(f"train step {k}: loss {loss:.5f}", flush=True)
        return net.params(), losses
    finally:
        net.close()
