"""The C ABI's error behaviour (include/sflow.h): validation before any device work, error
codes, state rules and the state blob round trip."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import log, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sf():
    from paper_2406_18031_amd import sflow
    return sflow


def _code(fn, *a):
    from paper_2406_18031_amd import sflow
    try:
        fn(*a)
    except sflow.SflowError as e:
        return e.status
    return 0


def test_config_validation(sf):
    log("config validation")
    bad = [
        sf.make_config(1, 10, 1, 1.0, [2]),            # too small
        sf.make_config(16, 16, 0, 1.0, [2]),           # no levels
        sf.make_config(16, 16, 9, 1.0, [2] * 8),       # too many levels
        sf.make_config(8, 8, 4, 1.0, [1] * 4),         # coarsest level 1x1
        sf.make_config(64, 64, 1, -1.0, [2]),          # negative max flow
        sf.make_config(64, 64, 1, float("nan"), [2]),
        sf.make_config(64, 64, 1, 1.0, [17]),          # too many smoothing passes
        sf.make_config(64, 64, 1, 1.0, [2], alpha=(1, 1, 0, 1, 1)),     # alpha_3 = 0
        sf.make_config(64, 64, 1, 1.0, [2], storage=5),
        sf.make_config(64, 64, 1, 1.0, [2], read_flags=8),
    ]
    for cfg in bad:
        assert _code(sf.sf_create, cfg, 0) == sf.SF_ERR_INVALID_ARG, sf.sf_last_error(None)
    # halo larger than the 64-pixel region even with the prediction split (16 smoothing passes);
    # the learned update with more than 4 smoothing passes
    assert _code(sf.sf_create, sf.make_config(256, 256, 1, 4.0, [16]), 0) == sf.SF_ERR_UNSUPPORTED
    assert _code(sf.sf_create, sf.make_config(64, 64, 1, 1.0, [5], update=1), 0) == \
        sf.SF_ERR_UNSUPPORTED
    assert _code(sf.sf_create, sf.make_config(64, 64, 1, 1.0, [2], update=2), 0) == \
        sf.SF_ERR_INVALID_ARG


def test_call_errors_and_state_rules(sf):
    import torch
    log("call errors")
    ctx = sf.sf_create(sf.make_config(32, 40, 2, 2.0, [2, 2]))
    Y = to_dev(np.random.default_rng(0).random((32, 40)))
    rho = to_dev(np.full((32, 40), 0.5))
    # push before the camera is set
    assert _code(sf.sf_push_frame, ctx, Y, rho, 0.01) == sf.SF_ERR_STATE
    assert _code(sf.sf_set_camera, ctx, 0.0, 40.0, 20.0, 16.0) == sf.SF_ERR_INVALID_ARG
    sf.sf_set_camera(ctx, 40.0, 40.0, 19.5, 15.5)
    out = torch.empty((3, 32, 40), device="cuda")
    assert _code(sf.sf_get_flow, ctx, sf.SF_FLOW_W_RAD_S, out) == sf.SF_ERR_STATE
    host = np.zeros((32, 40), np.float32)
    assert _code(sf.sf_push_frame, ctx, host.ctypes.data, rho, 0.01) == sf.SF_ERR_INVALID_ARG
    assert _code(sf.sf_push_frame, ctx, None, rho, 0.01) == sf.SF_ERR_INVALID_ARG
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        assert _code(sf.sf_push_frame, ctx, Y, rho, dt) == sf.SF_ERR_INVALID_ARG
    assert _code(sf.sf_get_flow, ctx, 99, out) == sf.SF_ERR_INVALID_ARG
    # the failed calls changed nothing: the next push is still the first frame -> zeros
    sf.sf_push_frame(ctx, Y, rho, 0.01)
    sf.sf_get_flow(ctx, sf.SF_FLOW_W_RAD_S, out)
    assert float(out.abs().max()) == 0.0
    sf.sf_get_flow(ctx, sf.SF_FLOW_RHO, out[:1])
    np.testing.assert_allclose(out[0].cpu().numpy(), 0.5)
    assert _code(sf.sf_get_flow, ctx, sf.SF_FLOW_W_RAD_S, host.ctypes.data) == sf.SF_ERR_INVALID_ARG
    # blob of the wrong size
    n = sf.sf_state_size(ctx)
    buf = ctypes.create_string_buffer(n - 4)
    assert sf.lib.sf_get_state(ctx, buf, n - 4) == sf.SF_ERR_INVALID_ARG
    assert sf.lib.sf_set_tile(ctx, 1, 60, 60) == sf.SF_ERR_INVALID_ARG
    assert sf.lib.sf_set_pass_steps(ctx, 0) == sf.SF_ERR_INVALID_ARG
    assert sf.lib.sf_set_pass_steps(ctx, 65) == sf.SF_ERR_INVALID_ARG
    assert sf.lib.sf_set_pass_steps(ctx, 1) == sf.SF_OK
    sf.sf_destroy(ctx)
    # a halo that fits only when the prediction is split: 30 steps with 4 smoothing passes
    big = sf.make_config(64, 64, 1, 30.0, [4])
    ctx = sf.sf_create(big)
    assert sf.lib.sf_set_pass_steps(ctx, 32) == sf.SF_ERR_UNSUPPORTED
    sf.sf_destroy(ctx)
    assert sf.lib.sf_destroy(None) == sf.SF_OK
    assert sf.lib.sf_push_frame(None, None, None, 1.0) == sf.SF_ERR_INVALID_ARG


def test_state_round_trip(sf):
    """get_state -> set_state on a fresh context continues the same stream bitwise."""
    log("state round trip")
    rng = np.random.default_rng(4)
    frames = [(to_dev(rng.random((48, 56))), to_dev(0.2 + rng.random((48, 56)))) for _ in range(5)]
    a = sf.Filter(48, 56, 2, 3.0, [2, 3], 50.0, 50.0, 27.5, 23.5)
    for Y, r in frames[:3]:
        a.push(Y, r, 0.01)
    blob = sf.sf_get_state(a.ctx)
    b = sf.Filter(48, 56, 2, 3.0, [2, 3], 50.0, 50.0, 27.5, 23.5)
    sf.sf_set_state(b.ctx, blob)
    for Y, r in frames[3:]:
        a.push(Y, r, 0.01)
        b.push(Y, r, 0.01)
    assert np.array_equal(a.flow().cpu().numpy(), b.flow().cpu().numpy())
    a.close()
    b.close()


def _with_failing_alloc(n, fn, *a):
    """Run fn with the n-th device allocation failing (SFLOW_FAIL_ALLOC); return its status."""
    import os
    os.environ["SFLOW_FAIL_ALLOC"] = str(n)
    try:
        return _code(fn, *a)
    finally:
        del os.environ["SFLOW_FAIL_ALLOC"]


def test_allocation_failure_leaves_the_context_unchanged(sf):
    """An allocation failure in a set-up call (creation, camera, pass length, tile) returns
    SF_ERR_OOM and leaves the context as it was: the next pushes are bitwise those of a
    context that never saw the failed call."""
    log("allocation failure injection")
    cfg = sf.make_config(48, 56, 2, 6.0, [2, 2])
    cam = (50.0, 50.0, 27.5, 23.5)
    assert _with_failing_alloc(1, sf.sf_create, cfg) == sf.SF_ERR_OOM
    rng = np.random.default_rng(8)
    frames = [(to_dev(rng.random((48, 56))), to_dev(0.2 + rng.random((48, 56)))) for _ in range(6)]
    ref = sf.Filter(48, 56, 2, 6.0, [2, 2], *cam)
    # a camera whose upload fails: no camera, pushes refused; then a camera that succeeds
    ctx = sf.sf_create(cfg)
    assert _with_failing_alloc(1, sf.sf_set_camera, ctx, *cam) == sf.SF_ERR_OOM
    assert _code(sf.sf_push_frame, ctx, frames[0][0], frames[0][1], 0.01) == sf.SF_ERR_STATE
    sf.sf_set_camera(ctx, *cam)
    for k, (Y, r) in enumerate(frames):
        if k == 2:
            # pass length 2 splits the 6-step level: the split fields (allocation 1) or the
            # larger pass table (allocation 2) cannot be allocated
            assert _with_failing_alloc(1, sf.sf_set_pass_steps, ctx, 2) == sf.SF_ERR_OOM
            assert _with_failing_alloc(2, sf.sf_set_pass_steps, ctx, 2) == sf.SF_ERR_OOM
        if k == 3:   # a tile change that needs no allocation still goes through
            sf.sf_set_tile(ctx, 1, 20, 20)
            sf.sf_set_tile(ctx, 1, 0, 0)
        sf.sf_push_frame(ctx, Y, r, 0.01)
        ref.push(Y, r, 0.01)
        out = ref.flow().cpu().numpy()
        got = torch_flow(sf, ctx, 48, 56)
        assert np.array_equal(got, out), k
    # the context still takes the change once memory is there
    sf.sf_set_pass_steps(ctx, 2)
    sf.sf_destroy(ctx)
    ref.close()


def torch_flow(sf, ctx, R, C):
    import torch
    out = torch.empty((3, R, C), dtype=torch.float32, device="cuda")
    sf.sf_get_flow(ctx, sf.SF_FLOW_W_FRAME, out)
    return out.cpu().numpy()


def test_learned_state_set_clears_the_correction(sf):
    """On a learned context, setting a state clears the output correction of the frame before
    it, so the flow read back is the state's, and the update inputs are refused until a push
    has run an update."""
    import torch
    from paper_2406_18031_amd import learned
    log("learned context: set_state")
    rng = np.random.default_rng(9)
    frames = [(to_dev(rng.random((40, 48))), to_dev(0.2 + rng.random((40, 48)))) for _ in range(4)]
    f = sf.Filter(40, 48, 2, 3.0, [2, 2], 45.0, 45.0, 23.5, 19.5, update=sf.SF_UPDATE_LEARNED)
    f.set_learned(learned.init_params(3, last_scale=1.0), float("inf"))
    for Y, r in frames[:3]:
        f.push(Y, r, 0.01)
    before = f.flow().cpu().numpy()
    blob = sf.sf_get_state(f.ctx)
    st, _, _ = sf.unpack_state(blob, 40, 48, 2)
    w_state = st[0]["w"].transpose(2, 0, 1)
    assert np.abs(before - w_state).max() > 0      # the network corrects the output
    sf.sf_set_state(f.ctx, blob)
    np.testing.assert_array_equal(f.flow().cpu().numpy(), w_state.astype(np.float32))
    out = torch.empty((sf.SF_UPDATE_INPUT_PLANES, 40, 48), device="cuda")
    assert _code(sf.sf_get_update_inputs, f.ctx, 0, out) == sf.SF_ERR_STATE
    f.push(*frames[3], 0.01)
    sf.sf_get_update_inputs(f.ctx, 0, out)
    f.close()
