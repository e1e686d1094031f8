"""The learned update: the network's BF16 forward and backward kernels against the FP64 network
oracle, training, and the filter's learned mode (fallback rule, the network's flow,
smoothing)."""
import numpy as np
import pytest

from gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu

SIZES = [(19, 37), (8, 8), (33, 16), (5, 3)]


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _params(seed):
    from oracle import cnn
    rng = np.random.default_rng(seed)
    layers = cnn.init_params(seed)
    layers[-1] = (layers[-1][0] * 10.0, layers[-1][1])
    return [(W, b + 0.05 * rng.standard_normal(b.shape)) for W, b in layers]


def _flat(layers):
    from paper_2406_18031_amd import learned
    return learned.join_params(layers)


def _images(rng, C, sizes=SIZES):
    return [rng.standard_normal((C, r, c)) for r, c in sizes]


def _cat(imgs):
    return to_dev(np.concatenate([x.reshape(-1) for x in imgs]))


def _split(flat, C, sizes=SIZES):
    out, o = [], 0
    for r, c in sizes:
        out.append(flat[o:o + C * r * c].reshape(C, r, c))
        o += C * r * c
    return out


def test_network_forward_matches_oracle():
    from oracle import cnn
    from paper_2406_18031_amd import sflow
    log("network forward")
    rng = np.random.default_rng(5)
    layers = _params(1)
    flat = _flat(layers)
    rl = [(bf16(W), b) for W, b in layers]          # the weights the matrix cores see
    xs = _images(rng, 9)
    net = sflow.Net(SIZES, flat)
    out = _split(net.forward(_cat(xs)).cpu().numpy().astype(np.float64), 3)
    num = den = 0.0
    for x, o in zip(xs, out):
        ref, _, _ = cnn.forward(bf16(x).transpose(1, 2, 0), rl)
        ref = ref.transpose(2, 0, 1)
        num += float(np.sum((o - ref) ** 2))
        den += float(np.sum(ref ** 2))
        # each output within the rounding of three BF16 activations of its magnitude
        assert np.all(np.abs(o - ref) <= 2e-2 * np.abs(ref).max() + 1e-6)
    assert np.sqrt(num / den) <= 1e-2, np.sqrt(num / den)
    net.close()


def test_network_gradients_match_oracle():
    from oracle import cnn
    from paper_2406_18031_amd import learned, sflow
    log("network gradients")
    rng = np.random.default_rng(6)
    layers = _params(2)
    flat = _flat(layers)
    rl = [(bf16(W), b) for W, b in layers]
    xs = _images(rng, 9)
    ts = _images(rng, 3)
    net = sflow.Net(SIZES, flat)
    loss, grad = net.train_step(_cat(xs), _cat(ts), 0.0, want_grad=True)
    np.testing.assert_array_equal(net.params(), flat)     # lr = 0 leaves the parameters
    # the oracle's loss is per image; the library's is over all pixels of all images
    npx = sum(r * c for r, c in SIZES)
    ref_loss = 0.0
    ref_grads = [(np.zeros_like(W), np.zeros_like(b)) for W, b in rl]
    for x, t in zip(xs, ts):
        xi = bf16(x).transpose(1, 2, 0)
        o, acts, pres = cnn.forward(xi, rl)
        l_img, dout = cnn.loss_and_grad_out(o, t.transpose(1, 2, 0))
        w = x.shape[1] * x.shape[2] / npx
        ref_loss += l_img * w
        g = cnn.backward(dout * w, acts, pres, rl)
        ref_grads = [(a[0] + b[0], a[1] + b[1]) for a, b in zip(ref_grads, g)]
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss, (loss, ref_loss)
    got = learned.split_params(grad)
    for li, ((gw, gb), (rw, rb)) in enumerate(zip(got, ref_grads)):
        ew = np.linalg.norm(gw - rw) / np.linalg.norm(rw)
        eb = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        log(f"  layer {li}: weight gradient rel err {ew:.2e}, bias {eb:.2e}")
        assert ew <= 5e-2 and eb <= 5e-2, (li, ew, eb)
    net.close()


def test_fused_forward_equals_the_layer_by_layer_pass():
    """sf_net_forward runs the four layers in one launch (24 x 58 output tiles, activations in
    LDS); training runs them one launch each.  With the fused output as the training target the
    layer-by-layer output's endpoint loss has a derivative of exactly zero at every pixel, so
    the weight gradient is exactly zero if and only if the two outputs agree bit for bit (a
    one-ulp change of one target value makes it nonzero).  Images of several tiles with ragged
    tails, one exactly a tile, one pixel, one taller than wide."""
    import torch
    from paper_2406_18031_amd import sflow
    log("fused forward against the layer-by-layer pass")
    rng = np.random.default_rng(8)
    sizes = [(61, 130), (24, 58), (1, 1), (100, 59), (25, 117)]
    flat = _flat(_params(5))
    net = sflow.Net(sizes, flat)
    x = _cat(_images(rng, 9, sizes))
    out = net.forward(x).clone()
    assert bool(torch.isfinite(out).all())
    _, grad = net.train_step(x, out, 0.0, want_grad=True)
    assert np.all(grad == 0.0), float(np.abs(grad).max())
    bumped = out.clone()
    bumped[1234] = torch.nextafter(bumped[1234], torch.tensor(np.inf, device="cuda"))
    _, grad = net.train_step(x, bumped, 0.0, want_grad=True)
    assert np.any(grad != 0.0)
    net.close()


def test_training_reduces_loss():
    from oracle import cnn
    from paper_2406_18031_amd import learned, sflow
    log("training")
    rng = np.random.default_rng(7)
    sizes = [(32, 32), (24, 40)]
    teacher = _params(3)
    xs = _images(rng, 9, sizes)
    ts = [cnn.forward(x.transpose(1, 2, 0), teacher)[0].transpose(2, 0, 1) for x in xs]
    params, losses = learned.train(sizes, [(_cat(xs), _cat(ts))] * 150,
                                   learned.init_params(4), lr=3e-3)
    log(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
    assert np.all(np.isfinite(params))


# ---- the filter's learned mode ------------------------------------------------------------
def _scene(R, C, nfr, seed):
    rng = np.random.default_rng(seed)
    base = rng.random((R + 3 * nfr, C + 3 * nfr))
    from scipy.ndimage import uniform_filter
    base = uniform_filter(base, 3, mode="wrap")
    out = []
    for k in range(nfr):
        Y = np.roll(base, (k, -k), axis=(0, 1))[:R, :C]
        rho = 0.3 + 0.2 * rng.random((R, C))
        rho[rng.random((R, C)) < 0.05] = np.nan
        out.append((to_dev(Y), to_dev(rho)))
    return out


def _pair(spec, params, threshold, storage=0):
    from paper_2406_18031_amd import sflow
    plain = sflow.Filter(*spec["dims"], *spec["camera"], storage=storage)
    lrn = sflow.Filter(*spec["dims"], *spec["camera"], storage=storage,
                       update=sflow.SF_UPDATE_LEARNED)
    lrn.set_learned(params, threshold)
    return plain, lrn


SPEC = dict(dims=(48, 70, 2, 3.0, [2, 2]), camera=(60.0, 60.0, 34.5, 23.5))


@pytest.mark.parametrize("storage", [0, 1])
def test_negative_threshold_gives_the_plain_update(storage):
    from paper_2406_18031_amd import learned, sflow
    log("learned, threshold < 0, storage", storage)
    frames = _scene(48, 70, 4, 11)
    plain, lrn = _pair(SPEC, learned.init_params(5, last_scale=1.0), -1.0, storage)
    for k, (Y, rho) in enumerate(frames):
        Yi = Y.half() if storage else Y
        ri = rho.half() if storage else rho
        plain.push(Yi, ri, 0.05)
        lrn.push(Yi, ri, 0.05)
        a = plain.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
        b = lrn.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy()
        assert np.array_equal(a, b), k
    fb, px = lrn.learned_stats()
    assert px == 3 * 48 * 70 and fb == px


def test_network_flow_and_smoothing_match_oracle():
    """threshold = +inf: the flow is S(x_ls) + dmu * net(inputs); checked against the FP64
    network oracle on the inputs the filter exported and the oracle's smoothing."""
    from oracle import cnn
    from oracle.update import smooth
    from paper_2406_18031_amd import learned, sflow
    log("learned, threshold = inf")
    R, C = 40, 52
    spec = dict(dims=(R, C, 1, 2.0, [3]), camera=(50.0, 50.0, 25.5, 19.5))
    frames = _scene(R, C, 3, 12)
    p = learned.init_params(6, last_scale=1.0)
    _, lrn = _pair(spec, p, float("inf"))
    rl = [(bf16(W), b) for W, b in learned.split_params(p)]
    for k, (Y, rho) in enumerate(frames):
        lrn.push(Y, rho, 0.05)
        if k == 0:
            continue
        ui = lrn.update_inputs().cpu().numpy().astype(np.float64)
        dmu = ui[21][..., None]
        out, _, _ = cnn.forward(bf16(ui[0:9]).transpose(1, 2, 0), rl)
        xs = smooth(ui[12:15].transpose(1, 2, 0), 3)
        np.testing.assert_allclose(ui[15:18].transpose(1, 2, 0), xs, rtol=1e-5,
                                   atol=1e-6 * np.abs(xs).max())
        ref = xs + dmu * out
        got = lrn.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy().transpose(1, 2, 0)
        err = np.linalg.norm(got - ref) / np.linalg.norm(dmu * out)
        log(f"  frame {k}: rel err of the correction {err:.2e}")
        assert err <= 2e-2
        # the exported inputs hold x0 and x_ls in pixels / 4, rounded to BF16 as the network
        # reads them (relative rounding error <= 2^-9); a top level has no parent
        assert np.array_equal(bf16(ui[0:9]), ui[0:9])
        np.testing.assert_allclose(ui[3:6] * 4.0 * ui[21], ui[9:12], rtol=2.0 ** -8, atol=1e-9)
        np.testing.assert_allclose(ui[6:9] * 4.0 * ui[21], ui[12:15], rtol=2.0 ** -8, atol=1e-9)
        assert not ui[18:21].any()
    fb, px = lrn.learned_stats()
    assert fb == 0 and px == 2 * R * C


def test_fallback_fires_on_a_corrupted_network():
    """A network whose output is wildly off (huge last-layer bias) is rejected at every pixel
    by a moderate threshold, which leaves exactly the plain update; the fallback count never
    grows with the threshold."""
    from paper_2406_18031_amd import learned, sflow
    log("learned, corrupted network")
    frames = _scene(48, 70, 3, 13)
    p = learned.init_params(7)
    layers = learned.split_params(p)
    layers[-1] = (layers[-1][0], np.array([300.0, -200.0, 250.0]))
    bad = learned.join_params(layers)
    plain, lrn = _pair(SPEC, bad, 1.0)
    for Y, rho in frames:
        plain.push(Y, rho, 0.05)
        lrn.push(Y, rho, 0.05)
    assert np.array_equal(plain.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy(),
                          lrn.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy())
    fb, px = lrn.learned_stats()
    assert fb == px == 2 * 48 * 70
    counts = []
    for thr in (1e-4, 1e-2, 1.0, 1e3):
        _, f = _pair(SPEC, p, thr)
        for Y, rho in frames[:2]:     # one update: the same inputs for every threshold
            f.push(Y, rho, 0.05)
        counts.append(f.learned_stats()[0])
        f.close()
    log("  fallbacks vs threshold:", counts)
    assert all(a >= b for a, b in zip(counts, counts[1:]))


def test_learned_needs_parameters():
    from paper_2406_18031_amd import learned, sflow
    f = sflow.Filter(*SPEC["dims"], *SPEC["camera"], update=sflow.SF_UPDATE_LEARNED)
    Y, rho = _scene(48, 70, 1, 14)[0]
    with pytest.raises(sflow.SflowError) as e:
        f.push(Y, rho, 0.05)
    assert e.value.status == sflow.SF_ERR_STATE
    with pytest.raises(sflow.SflowError) as e:
        f.set_learned(np.full(learned.N_PARAMS, np.nan, np.float32), 1.0)
    assert e.value.status == sflow.SF_ERR_INVALID_ARG
    with pytest.raises(sflow.SflowError) as e:
        f.set_learned(learned.init_params(0), float("nan"))
    assert e.value.status == sflow.SF_ERR_INVALID_ARG
    plain = sflow.Filter(*SPEC["dims"], *SPEC["camera"])
    with pytest.raises(sflow.SflowError) as e:
        plain.set_learned(learned.init_params(0), 1.0)
    assert e.value.status == sflow.SF_ERR_STATE


def test_network_object_errors():
    """The trainer's calls validate their arguments before any device work."""
    import ctypes
    from paper_2406_18031_amd import learned, sflow
    lib = sflow.lib
    out = ctypes.c_void_p()
    rows = (ctypes.c_int32 * 1)(8)
    cols = (ctypes.c_int32 * 1)(8)
    assert lib.sf_net_create(rows, cols, 0, None, ctypes.byref(out)) == sflow.SF_ERR_INVALID_ARG
    bad = (ctypes.c_int32 * 1)(0)
    assert lib.sf_net_create(bad, cols, 1, None, ctypes.byref(out)) == sflow.SF_ERR_INVALID_ARG
    net = sflow.Net([(8, 8)], learned.init_params(0))
    p = learned.init_params(0)
    assert lib.sf_net_set_params(net.net, p.ctypes.data, p.size - 1) == sflow.SF_ERR_INVALID_ARG
    pn = p.copy()
    pn[5] = np.inf
    assert lib.sf_net_set_params(net.net, pn.ctypes.data, pn.size) == sflow.SF_ERR_INVALID_ARG
    x = to_dev(np.zeros(9 * 64))
    t = to_dev(np.zeros(3 * 64))
    host = np.zeros(9 * 64, np.float32)
    assert lib.sf_net_train_step(net.net, host.ctypes.data, t.data_ptr(), 1e-3, None, None) == \
        sflow.SF_ERR_INVALID_ARG
    assert lib.sf_net_train_step(net.net, x.data_ptr(), t.data_ptr(), -1.0, None, None) == \
        sflow.SF_ERR_INVALID_ARG
    assert lib.sf_net_set_loss(net.net, 0.0) == sflow.SF_ERR_INVALID_ARG
    # a valid step still works after the rejected calls, and leaves finite parameters
    loss, grad = net.train_step(x, t, 1e-3, want_grad=True)
    assert np.isfinite(loss) and np.all(np.isfinite(grad))
    assert np.all(np.isfinite(net.params()))
    net.close()
    assert lib.sf_net_destroy(None) == sflow.SF_OK
