"""The learned update: parameter layout, training targets and a GPU training loop.

Everything numeric runs in the library (include/sflow.h, sections "learned update" and
"training the learned update's network"): the filter writes each frame's network inputs,
the network object runs forward, loss, backward and Adam on the matrix cores.  This module
only arranges tensors.  The update replaces, at the finest level, the least-squares solution
of the paper's update step (Section "State update") by the network's flow where the
least-squares cost increase stays under a threshold.
"""
from __future__ import annotations

from typing import Iterable, List, Sequence, Tuple

import numpy as np

from . import sflow

CHANNELS = (6, 16, 16, 16, 3)
N_PARAMS = sflow.SF_LEARNED_PARAMS


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
    """Network input (6, R, C) and target correction (3, R, C) of one frame.

    update_inputs: the 16 planes of sf_get_update_inputs; w_frame: the true structure flow
    of that frame in rad/frame, (3, R, C).  The target is the correction (pixels per frame)
    that takes the predicted field to the true one: (w - parent - x0) / dmu."""
    x0 = update_inputs[6:9]
    parent = update_inputs[12:15]
    dmu = update_inputs[15]
    return update_inputs[0:6], (w_frame - parent - x0) / dmu


def train(sizes: Sequence[Tuple[int, int]], batches: Iterable, params: np.ndarray,
          lr: float = 2e-3, stream=None, log_every: int = 0):
    """Adam over `batches`, an iterable of (inputs, targets) device tensors laid out as the
    network object expects (images one after the other, inputs [6][R][C], targets [3][R][C]).
    Returns (parameters, losses)."""
    net = sflow.Net(sizes, params, stream)
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
