"""Pins for the learned update's FP64 network oracle: the convolution against a direct loop,
and every gradient against central finite differences."""
import numpy as np

from oracle import cnn


def _direct_conv(x, W, b):
    H, Wd, cin = x.shape
    out = np.zeros((H, Wd, W.shape[3]))
    for i in range(H):
        for j in range(Wd):
            acc = b.copy()
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ii, jj = i + dy, j + dx
                    if 0 <= ii < H and 0 <= jj < Wd:
                        acc = acc + x[ii, jj] @ W[dy + 1, dx + 1]
            out[i, j] = acc
    return out


def test_conv_matches_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 7, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(cnn.conv3x3(x, W, b), _direct_conv(x, W, b), atol=1e-12)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = cnn.init_params(3)
    # make the last layer as large as the others so that every gradient is exercised
    params[-1] = (params[-1][0] * 10.0, rng.standard_normal(3) * 0.1)
    params = [(W, b + 0.05 * rng.standard_normal(b.shape)) for W, b in params]
    x = rng.standard_normal((6, 5, 9))
    target = rng.standard_normal((6, 5, 3))

    def loss(ps):
        out, _, _ = cnn.forward(x, ps)
        return cnn.loss_and_grad_out(out, target)[0]

    out, acts, pres = cnn.forward(x, params)
    _, dout = cnn.loss_and_grad_out(out, target)
    grads = cnn.backward(dout, acts, pres, params)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[li][0][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (li, idx)
        for k in range(b.shape[0]):
            bp, bm = b.copy(), b.copy()
            bp[k] += h
            bm[k] -= h
            pp = list(params); pp[li] = (W, bp)
            pm = list(params); pm[li] = (W, bm)
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[li][1][k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (li, k)


def test_parameter_count():
    n = sum(W.size + b.size for W, b in cnn.init_params())
    assert n == 6387
