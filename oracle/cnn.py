"""FP64 oracle of the learned update's network (test infrastructure only).

A 4-layer 3x3 convolutional network, 9 -> 16 -> 16 -> 16 -> 3 channels, ReLU after the
first three layers, zero padding at the image border ("same" size).  It maps per-pixel
update inputs to a refinement of the smoothed least-squares solution of the update step (the
learned form of the library):

    inputs  (9): Y_prev - 1/2, Y_new - 1/2, 4 rho_meas (0 where missing),
                 x0 / dmu / 4 (3), x_ls / dmu / 4 (3)
    output  (3): correction in pixels per frame, x = S(x_ls) + dmu * out

Layout: images are (H, W, C) arrays; weights W[l] are (3, 3, C_in, C_out) indexed by the
tap offset (dy + 1, dx + 1): out[p] = b + sum_{dy,dx,c} W[dy+1, dx+1, c, :] in[p + (dy, dx), c].
The loss is the mean Charbonnier endpoint error sqrt(|out - target|^2 + eps^2) over pixels.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (9, 16, 16, 16, 3)
EPS = 1e-3
IN_SHIFT = np.array([-0.5, -0.5, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
IN_SCALE = np.array([1.0, 1.0, 4.0, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25])


def init_params(seed: int = 0):
    """He-style initialisation; returns a list of (W, b) per layer, float64."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        std = np.sqrt(2.0 / (9 * cin))
        W = rng.standard_normal((3, 3, cin, cout)) * std
        b = np.zeros(cout)
        params.append((W, b))
    # small last layer: the network starts close to "no correction"
    W, b = params[-1]
    params[-1] = (W * 0.1, b)
    return params


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """'same' 3x3 convolution with zero padding, written as a sum over the nine taps."""
    H, Wd, _ = x.shape
    pad = np.zeros((H + 2, Wd + 2, x.shape[2]))
    pad[1:-1, 1:-1] = x
    out = np.broadcast_to(b, (H, Wd, W.shape[3])).copy()
    for dy in range(3):
        for dx in range(3):
            out += pad[dy:dy + H, dx:dx + Wd] @ W[dy, dx]
    return out


def forward(x: np.ndarray, params):
    """Returns (output, activations) where activations[l] is the input of layer l and
    pre[l] its pre-activation."""
    acts, pres = [x], []
    h = x
    for li, (W, b) in enumerate(params):
        z = conv3x3(h, W, b)
        pres.append(z)
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(h)
    return h, acts, pres


def loss_and_grad_out(out: np.ndarray, target: np.ndarray):
    d = out - target
    n = np.sqrt(np.sum(d * d, axis=-1) + EPS * EPS)
    npx = out.shape[0] * out.shape[1]
    return float(n.mean()), d / n[..., None] / npx


def backward(dout: np.ndarray, acts, pres, params):
    """Gradients [(dW, db)] of the loss given d loss / d output."""
    grads = [None] * len(params)
    g = dout
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        if li < len(params) - 1:
            g = g * (pres[li] > 0)
        x = acts[li]
        H, Wd, _ = x.shape
        pad = np.zeros((H + 2, Wd + 2, x.shape[2]))
        pad[1:-1, 1:-1] = x
        dW = np.zeros_like(W)
        for dy in range(3):
            for dx in range(3):
                dW[dy, dx] = pad[dy:dy + H, dx:dx + Wd].reshape(-1, x.shape[2]).T @ \
                    g.reshape(-1, g.shape[2])
        db = g.sum(axis=(0, 1))
        grads[li] = (dW, db)
        if li > 0:
            # d input = correlation of g with the flipped, transposed kernel
            gp = np.zeros((H + 2, Wd + 2, g.shape[2]))
            gp[1:-1, 1:-1] = g
            dx_ = np.zeros_like(x)
            for dy in range(3):
                for dxo in range(3):
                    # in[p + t] contributed to out[p] through W[t]; so d in[q] = sum_t W[t] g[q - t]
                    dx_ += gp[2 - dy:2 - dy + H, 2 - dxo:2 - dxo + Wd] @ W[dy, dxo].T
            g = dx_
    return grads


def normalise_inputs(Yprev, Ynew, rho, x0_px, xls_px):
    rho = np.where(np.isnan(rho), 0.0, rho)
    x = np.concatenate([Yprev[..., None], Ynew[..., None], rho[..., None], x0_px, xls_px],
                       axis=-1)
    return (x + IN_SHIFT) * IN_SCALE
