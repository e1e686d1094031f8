"""Python binding of libsflow (include/sflow.h): argument marshalling only.

The functions below carry the C names and forward to the library through ctypes; every
step of the filter runs in the library's HIP kernels.  Torch is used for device memory and
streams: image and output arguments are torch CUDA tensors, and the context stream is the
torch stream current at sf_create (unless one is given).  If the library has not been
built, importing this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SFLOW_LIB may name another build of the library to load (the host-UB-trapping check build
# libsflow_ubsan.so, see build.py); by default the in-tree product library
LIB_PATH = os.environ.get("SFLOW_LIB") or os.path.join(_PKG, "libsflow.so")

SF_OK = 0
SF_ERR_INVALID_ARG = -1
SF_ERR_STATE = -2
SF_ERR_OOM = -3
SF_ERR_HIP = -4
SF_ERR_UNSUPPORTED = -5
SF_ERR_NUMERIC = -6

SF_FP32, SF_FP16 = 0, 1
SF_UPDATE_PLAIN, SF_UPDATE_LEARNED = 0, 1
SF_READ_DOMINANT_LITERAL, SF_READ_SOURCE_LITERAL, SF_READ_NO_CFL_CLAMP = 1, 2, 4
SF_FLOW_W_RAD_S, SF_FLOW_TANGENT_PX, SF_FLOW_NORMAL_PX, SF_FLOW_RHO, SF_FLOW_W_FRAME = 0, 1, 2, 3, 4
SF_MAX_LEVELS = 8
FLOW_COMPONENTS = {SF_FLOW_W_RAD_S: 3, SF_FLOW_TANGENT_PX: 2, SF_FLOW_NORMAL_PX: 1,
                   SF_FLOW_RHO: 1, SF_FLOW_W_FRAME: 3}
DEFAULT_ALPHA = (300.0, 1000.0, 1.0, 1.0, 1.0)
SF_LEARNED_PARAMS = 6387
SF_UPDATE_INPUT_PLANES = 22
SF_NOALLOC_MAX_PIXELS = 1 << 18


class sf_config(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("max_flow_px", ctypes.c_float),
                ("smooth_iters", ctypes.c_int32 * SF_MAX_LEVELS),
                ("alpha", ctypes.c_float * 5), ("storage", ctypes.c_int32),
                ("update", ctypes.c_int32), ("read_flags", ctypes.c_uint32)]


class sf_camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("eta", ctypes.c_void_p)]


def _camera(fx, fy, cx, cy, eta=None):
    """An sf_camera and the array its eta points to (kept alive by the caller for the call)."""
    if eta is None:
        return sf_camera(fx, fy, cx, cy, None), None
    a = np.ascontiguousarray(eta, dtype=np.float64)
    return sf_camera(fx, fy, cx, cy, a.ctypes.data), a


class SflowError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"sflow status {status}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2406_18031_amd.build")
    # Load torch's HIP runtime first: the library's libamdhip64.so.7 dependency then binds to
    # that same runtime instance, so torch's streams and allocations are valid in the library.
    # Loaded the other way round, the process can end up with two HIP runtimes (torch asks for
    # its bundled copy under another file name), which share no devices or streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, st = ctypes.c_void_p, ctypes.c_int
    sig = {
        "sf_create": (st, [ctypes.POINTER(sf_config), vp, ctypes.POINTER(vp)]),
        "sf_set_camera": (st, [vp, ctypes.POINTER(sf_camera)]),
        "sf_push_frame": (st, [vp, vp, vp, ctypes.c_double]),
        "sf_push_frame_ex": (st, [vp, vp, vp, ctypes.c_double, vp, vp, vp]),
        "sf_push_frames_ex": (st, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                   ctypes.POINTER(ctypes.c_double), vp, vp, vp]),
        "sf_get_flow": (st, [vp, ctypes.c_int32, vp]),
        "sf_state_size": (st, [vp, ctypes.POINTER(ctypes.c_size_t)]),
        "sf_get_state": (st, [vp, vp, ctypes.c_size_t]),
        "sf_set_state": (st, [vp, vp, ctypes.c_size_t]),
        "sf_destroy": (st, [vp]),
        "sf_last_error": (ctypes.c_char_p, [vp]),
        "sf_set_tile": (st, [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
        "sf_set_timing": (st, [vp, ctypes.c_int32]),
        "sf_set_graph": (st, [vp, ctypes.c_int32]),
        "sf_set_input_stream": (st, [vp, vp]),
        "sf_copy_probe": (st, [vp, vp, ctypes.c_size_t, vp]),
        "sf_set_source_camera": (st, [vp, ctypes.c_int32, ctypes.POINTER(sf_camera),
                                      ctypes.c_int32, ctypes.c_int32]),
        "sf_map_frame": (st, [vp, ctypes.c_int32, vp, vp, vp, vp]),
        "sf_set_stereo": (st, [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_double, ctypes.c_double]),
        "sf_stereo_depth": (st, [vp, ctypes.c_int32, vp, vp, vp]),
        "sf_set_pass_steps": (st, [vp, ctypes.c_int32]),
        "sf_kernel_times": (st, [vp, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
        "sf_create_batch": (st, [ctypes.POINTER(sf_config), ctypes.c_int32, vp,
                                 ctypes.POINTER(vp)]),
        "sf_stream_count": (st, [vp, ctypes.POINTER(ctypes.c_int32)]),
        "sf_set_cameras": (st, [vp, ctypes.POINTER(sf_camera)]),
        "sf_push_frames": (st, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                ctypes.POINTER(ctypes.c_double)]),
        "sf_get_flow_stream": (st, [vp, ctypes.c_int32, ctypes.c_int32, vp]),
        "sf_get_flows": (st, [vp, ctypes.c_int32, ctypes.POINTER(vp)]),
        "sf_state_size_stream": (st, [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
        "sf_get_state_stream": (st, [vp, ctypes.c_int32, vp, ctypes.c_size_t]),
        "sf_set_state_stream": (st, [vp, ctypes.c_int32, vp, ctypes.c_size_t]),
        "sf_set_learned": (st, [vp, vp, ctypes.c_size_t, ctypes.c_float]),
        "sf_learned_stats": (st, [vp, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
        "sf_get_update_inputs": (st, [vp, ctypes.c_int32, vp]),
        "sf_check_state": (st, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "sf_net_create": (st, [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                               ctypes.c_int32, vp, ctypes.POINTER(vp)]),
        "sf_net_set_params": (st, [vp, vp, ctypes.c_size_t]),
        "sf_net_get_params": (st, [vp, vp, ctypes.c_size_t]),
        "sf_net_forward": (st, [vp, vp, vp]),
        "sf_net_train_step": (st, [vp, vp, vp, ctypes.c_float, vp, vp]),
        "sf_net_set_loss": (st, [vp, ctypes.c_float]),
        "sf_net_destroy": (st, [vp]),
        "sf_net_last_error": (ctypes.c_char_p, [vp]),
        "sf_net_forward_noalloc": (st, [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
EXPORTED = ("sf_create", "sf_set_camera", "sf_push_frame", "sf_get_flow", "sf_state_size",
            "sf_get_state", "sf_set_state", "sf_destroy", "sf_last_error", "sf_set_tile",
            "sf_set_timing", "sf_kernel_times", "sf_set_pass_steps", "sf_create_batch", "sf_stream_count",
            "sf_set_cameras", "sf_push_frames", "sf_get_flow_stream", "sf_get_flows",
            "sf_state_size_stream",
            "sf_get_state_stream", "sf_set_state_stream", "sf_set_learned", "sf_learned_stats",
            "sf_get_update_inputs", "sf_net_create", "sf_net_set_params", "sf_net_get_params",
            "sf_net_forward", "sf_net_train_step", "sf_net_set_loss", "sf_net_destroy",
            "sf_net_last_error", "sf_net_forward_noalloc", "sf_push_frame_ex",
            "sf_push_frames_ex", "sf_set_graph", "sf_copy_probe", "sf_set_source_camera",
            "sf_map_frame", "sf_set_stereo", "sf_stereo_depth", "sf_set_input_stream",
            "sf_check_state")


def _check(status: int, ctx) -> None:
    if status != SF_OK:
        msg = lib.sf_last_error(ctx)
        raise SflowError(status, msg.decode() if msg else "")


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def make_config(rows: int, cols: int, levels: int, max_flow_px: float,
                smooth_iters: Sequence[int], alpha=DEFAULT_ALPHA, storage: int = SF_FP32,
                update: int = SF_UPDATE_PLAIN, read_flags: int = 0) -> sf_config:
    c = sf_config()
    c.rows, c.cols, c.levels = rows, cols, levels
    c.max_flow_px = max_flow_px
    for k, s in enumerate(list(smooth_iters)[:SF_MAX_LEVELS]):
        c.smooth_iters[k] = int(s)
    for k, a in enumerate(alpha):
        c.alpha[k] = float(a)
    c.storage, c.update, c.read_flags = storage, update, read_flags
    return c


# ---- the C calls, same names ------------------------------------------------------------
def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    return ctypes.c_void_p(stream)


def sf_create(cfg: sf_config, stream=None) -> int:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    out = ctypes.c_void_p()
    _check(lib.sf_create(ctypes.byref(cfg), ctypes.c_void_p(stream), ctypes.byref(out)), None)
    return out.value


def sf_set_camera(ctx: int, fx: float, fy: float, cx: float, cy: float, eta=None) -> None:
    """eta: None (pinhole) or the finest level's unit directions, (rows, cols, 3)."""
    cam, keep = _camera(fx, fy, cx, cy, eta)
    _check(lib.sf_set_camera(ctx, ctypes.byref(cam)), ctx)
    del keep


def sf_push_frame(ctx: int, Y, rho, dt: float) -> None:
    _check(lib.sf_push_frame(ctx, _ptr(Y), _ptr(rho), float(dt)), ctx)


def _vec3s(v, n):
    """None, or n 3-vectors as a flat ctypes double array."""
    if v is None:
        return None
    a = np.asarray(v, dtype=np.float64).reshape(-1)
    if a.size != 3 * n:
        raise ValueError(f"expected {3 * n} values")
    return (ctypes.c_double * a.size)(*a.tolist())


def sf_push_frame_ex(ctx: int, Y, rho, dt: float, omega=None, omega_dot=None,
                     acc=None) -> None:
    _check(lib.sf_push_frame_ex(ctx, _ptr(Y), _ptr(rho), float(dt), _vec3s(omega, 1),
                                _vec3s(omega_dot, 1), _vec3s(acc, 1)), ctx)


def sf_get_flow(ctx: int, kind: int, out) -> None:
    _check(lib.sf_get_flow(ctx, kind, _ptr(out)), ctx)


def sf_state_size(ctx: int) -> int:
    n = ctypes.c_size_t()
    _check(lib.sf_state_size(ctx, ctypes.byref(n)), ctx)
    return n.value


def sf_get_state(ctx: int) -> bytes:
    n = sf_state_size(ctx)
    buf = ctypes.create_string_buffer(n)
    _check(lib.sf_get_state(ctx, buf, n), ctx)
    return buf.raw


def sf_set_state(ctx: int, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib.sf_set_state(ctx, buf, len(blob)), ctx)


def sf_destroy(ctx: int) -> None:
    _check(lib.sf_destroy(ctx), None)


def sf_last_error(ctx: Optional[int]) -> str:
    m = lib.sf_last_error(ctx)
    return m.decode() if m else ""


def sf_set_tile(ctx: int, level: int, tw: int, th: int) -> None:
    _check(lib.sf_set_tile(ctx, level, tw, th), ctx)


def sf_set_pass_steps(ctx: int, steps: int) -> None:
    _check(lib.sf_set_pass_steps(ctx, steps), ctx)


def sf_set_timing(ctx: int, enable: bool) -> None:
    _check(lib.sf_set_timing(ctx, 1 if enable else 0), ctx)


def sf_copy_probe(src, dst, nbytes: int, stream=None) -> None:
    st = lib.sf_copy_probe(_ptr(src), _ptr(dst), int(nbytes), _stream(stream))
    if st != SF_OK:
        raise SflowError(st, "sf_copy_probe")


def sf_set_source_camera(ctx: int, stream: int, fx: float, fy: float, cx: float, cy: float,
                         rows: int, cols: int) -> None:
    cam = sf_camera(fx, fy, cx, cy, None)
    _check(lib.sf_set_source_camera(ctx, stream, ctypes.byref(cam), rows, cols), ctx)


def sf_map_frame(ctx: int, stream: int, Y_src, rho_src, Y_out, rho_out) -> None:
    _check(lib.sf_map_frame(ctx, stream, _ptr(Y_src), _ptr(rho_src), _ptr(Y_out),
                            _ptr(rho_out)), ctx)


def sf_set_stereo(ctx: int, stream: int, baseline: float, max_disparity: int,
                  iterations: int = 3, texture: float = 2.5e-3, residual: float = 0.05) -> None:
    _check(lib.sf_set_stereo(ctx, stream, float(baseline), int(max_disparity), int(iterations),
                             float(texture), float(residual)), ctx)


def sf_stereo_depth(ctx: int, stream: int, Y_left, Y_right, rho_out) -> None:
    _check(lib.sf_stereo_depth(ctx, stream, _ptr(Y_left), _ptr(Y_right), _ptr(rho_out)), ctx)


def sf_set_graph(ctx: int, enable: bool) -> None:
    _check(lib.sf_set_graph(ctx, 1 if enable else 0), ctx)


def sf_set_input_stream(ctx: int, stream) -> None:
    """stream: a torch.cuda.Stream, a raw hipStream_t value, or None (the context stream)."""
    if stream is not None and not isinstance(stream, int):
        stream = stream.cuda_stream
    _check(lib.sf_set_input_stream(ctx, ctypes.c_void_p(stream) if stream else None), ctx)


def sf_kernel_times(ctx: int, reset: bool = False):
    ms = (ctypes.c_double * 3)()
    n = (ctypes.c_int64 * 3)()
    _check(lib.sf_kernel_times(ctx, ms, n, 1 if reset else 0), ctx)
    return list(ms), list(n)


def sf_create_batch(cfgs: Sequence[sf_config], stream=None) -> int:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    arr = (sf_config * len(cfgs))(*cfgs)
    out = ctypes.c_void_p()
    _check(lib.sf_create_batch(arr, len(cfgs), ctypes.c_void_p(stream), ctypes.byref(out)), None)
    return out.value


def sf_stream_count(ctx: int) -> int:
    n = ctypes.c_int32()
    _check(lib.sf_stream_count(ctx, ctypes.byref(n)), ctx)
    return n.value


def sf_set_cameras(ctx: int, cams: Sequence[Sequence[float]]) -> None:
    """cams: per stream (fx, fy, cx, cy) or (fx, fy, cx, cy, eta)."""
    made = [_camera(*c) for c in cams]
    arr = (sf_camera * len(cams))(*[m[0] for m in made])
    _check(lib.sf_set_cameras(ctx, arr), ctx)
    del made


def sf_push_frames(ctx: int, Ys, rhos, dts) -> None:
    n = len(Ys)
    y = (ctypes.c_void_p * n)(*[_ptr(t) for t in Ys])
    r = (ctypes.c_void_p * n)(*[_ptr(t) for t in rhos])
    d = (ctypes.c_double * n)(*[float(v) for v in dts])
    _check(lib.sf_push_frames(ctx, y, r, d), ctx)


def sf_push_frames_ex(ctx: int, Ys, rhos, dts, omegas=None, omega_dots=None,
                      accs=None) -> None:
    n = len(Ys)
    y = (ctypes.c_void_p * n)(*[_ptr(t) for t in Ys])
    r = (ctypes.c_void_p * n)(*[_ptr(t) for t in rhos])
    d = (ctypes.c_double * n)(*[float(v) for v in dts])
    _check(lib.sf_push_frames_ex(ctx, y, r, d, _vec3s(omegas, n), _vec3s(omega_dots, n),
                                 _vec3s(accs, n)), ctx)


def sf_get_flow_stream(ctx: int, stream: int, kind: int, out) -> None:
    _check(lib.sf_get_flow_stream(ctx, stream, kind, _ptr(out)), ctx)


def sf_get_flows(ctx: int, kind: int, outs) -> None:
    """outs: one tensor (or None) per stream of the context."""
    if len(outs) != sf_stream_count(ctx):
        raise ValueError("sf_get_flows takes one output (or None) per stream")
    arr = (ctypes.c_void_p * len(outs))(*[None if o is None else _ptr(o) for o in outs])
    _check(lib.sf_get_flows(ctx, kind, arr), ctx)


def sf_state_size_stream(ctx: int, stream: int) -> int:
    n = ctypes.c_size_t()
    _check(lib.sf_state_size_stream(ctx, stream, ctypes.byref(n)), ctx)
    return n.value


def sf_get_state_stream(ctx: int, stream: int) -> bytes:
    n = sf_state_size_stream(ctx, stream)
    buf = ctypes.create_string_buffer(n)
    _check(lib.sf_get_state_stream(ctx, stream, buf, n), ctx)
    return buf.raw


def sf_set_state_stream(ctx: int, stream: int, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    _check(lib.sf_set_state_stream(ctx, stream, buf, len(blob)), ctx)


# ---- state blob layout (header + float32 planes, see include/sflow.h) ---------------------
def _f32(params) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if a.size != SF_LEARNED_PARAMS:
        raise ValueError(f"expected {SF_LEARNED_PARAMS} parameters, got {a.size}")
    return a


def sf_set_learned(ctx: int, params, threshold: float) -> None:
    a = _f32(params)
    _check(lib.sf_set_learned(ctx, a.ctypes.data, a.size, threshold), ctx)


def sf_check_state(ctx: int) -> int:
    """Mask of the streams whose stored flow was not finite since the last check (0: none);
    clears it.  Raises only for errors other than SF_ERR_NUMERIC."""
    m = ctypes.c_uint64()
    status = lib.sf_check_state(ctx, ctypes.byref(m))
    if status != SF_ERR_NUMERIC:
        _check(status, ctx)
    return m.value


def sf_learned_stats(ctx: int, reset: bool = False):
    fb, px = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.sf_learned_stats(ctx, ctypes.byref(fb), ctypes.byref(px), int(reset)), ctx)
    return fb.value, px.value


def sf_get_update_inputs(ctx: int, stream: int, out) -> None:
    _check(lib.sf_get_update_inputs(ctx, stream, _ptr(out)), ctx)


def _net_check(status: int, net) -> None:
    if status != SF_OK:
        msg = lib.sf_net_last_error(net)
        raise SflowError(status, msg.decode() if msg else "")


def sf_net_last_error(net: Optional[int]) -> str:
    msg = lib.sf_net_last_error(net)
    return msg.decode() if msg else ""


def sf_net_create(sizes: Sequence[Sequence[int]], stream=None) -> int:
    n = len(sizes)
    rows = (ctypes.c_int32 * max(n, 1))(*[int(r) for r, _ in sizes])
    cols = (ctypes.c_int32 * max(n, 1))(*[int(c) for _, c in sizes])
    out = ctypes.c_void_p()
    _net_check(lib.sf_net_create(rows, cols, n, _stream(stream), ctypes.byref(out)), None)
    return out.value


def sf_net_set_params(net: int, params) -> None:
    a = _f32(params)
    _net_check(lib.sf_net_set_params(net, a.ctypes.data, a.size), net)


def sf_net_get_params(net: int) -> np.ndarray:
    a = np.empty(SF_LEARNED_PARAMS, dtype=np.float32)
    _net_check(lib.sf_net_get_params(net, a.ctypes.data, a.size), net)
    return a


def sf_net_forward(net: int, inp, out) -> None:
    _net_check(lib.sf_net_forward(net, _ptr(inp), _ptr(out)), net)


def sf_net_forward_noalloc(params, rows: int, cols: int, inp, out, stream=None) -> None:
    """params, inp, out: device tensors (float32; SF_LEARNED_PARAMS, [9][rows][cols],
    [3][rows][cols])."""
    _net_check(lib.sf_net_forward_noalloc(_ptr(params), rows, cols, _ptr(inp), _ptr(out),
                                          _stream(stream)), None)


def sf_net_train_step(net: int, inp, target, lr: float, want_grad: bool = False):
    loss = np.zeros(1, dtype=np.float32)
    grad = np.empty(SF_LEARNED_PARAMS, dtype=np.float32) if want_grad else None
    _net_check(lib.sf_net_train_step(net, _ptr(inp), _ptr(target), lr, loss.ctypes.data,
                                     grad.ctypes.data if want_grad else None), net)
    return float(loss[0]), grad


def sf_net_set_loss(net: int, eps: float) -> None:
    _net_check(lib.sf_net_set_loss(net, eps), net)


def sf_net_destroy(net: int) -> None:
    _net_check(lib.sf_net_destroy(net), net)


def level_shapes(rows: int, cols: int, levels: int):
    out, r, c = [], rows, cols
    for _ in range(levels):
        out.append((r, c))
        r, c = (r + 1) // 2, (c + 1) // 2
    return out


def unpack_state(blob: bytes, rows: int, cols: int, levels: int):
    """-> (list of per-level dicts {w (R,C,3), dw (R,C,3), rho, Y}, dt_prev, frames)."""
    hdr = np.frombuffer(blob[:32], dtype=np.uint8)
    magic, version, nlev, init = np.frombuffer(hdr[:16].tobytes(), dtype=np.int32)
    dt_prev = float(np.frombuffer(hdr[16:24].tobytes(), dtype=np.float64)[0])
    frames = int(np.frombuffer(hdr[24:32].tobytes(), dtype=np.int64)[0])
    data = np.frombuffer(blob[32:], dtype=np.float32)
    out, off = [], 0
    for h, (R, C) in enumerate(level_shapes(rows, cols, levels)):
        n = R * C
        st = {}
        st["w"] = data[off:off + 3 * n].reshape(3, R, C).transpose(1, 2, 0).astype(np.float64)
        off += 3 * n
        if h < levels - 1:
            st["dw"] = data[off:off + 3 * n].reshape(3, R, C).transpose(1, 2, 0).astype(np.float64)
            off += 3 * n
        st["rho"] = data[off:off + n].reshape(R, C).astype(np.float64)
        off += n
        st["Y"] = data[off:off + n].reshape(R, C).astype(np.float64)
        off += n
        out.append(st)
    return out, dt_prev, frames


def pack_state(state, rows: int, cols: int, levels: int, dt_prev: float, frames: int = 1) -> bytes:
    head = np.zeros(32, dtype=np.uint8)
    head[:16] = np.frombuffer(np.array([0x54535346, 1, levels, 1], dtype=np.uint32).tobytes(),
                              dtype=np.uint8)
    head[16:24] = np.frombuffer(np.array([dt_prev], dtype=np.float64).tobytes(), dtype=np.uint8)
    head[24:32] = np.frombuffer(np.array([frames], dtype=np.int64).tobytes(), dtype=np.uint8)
    parts = [head.tobytes()]
    for h, st in enumerate(state):
        parts.append(np.ascontiguousarray(np.asarray(st["w"]).transpose(2, 0, 1), np.float32).tobytes())
        if h < levels - 1:
            parts.append(np.ascontiguousarray(np.asarray(st["dw"]).transpose(2, 0, 1), np.float32).tobytes())
        parts.append(np.ascontiguousarray(st["rho"], np.float32).tobytes())
        parts.append(np.ascontiguousarray(st["Y"], np.float32).tobytes())
    return b"".join(parts)


class Filter:
    """Convenience wrapper owning one context; inputs are torch CUDA tensors."""

    def __init__(self, rows, cols, levels, max_flow_px, smooth_iters, fx, fy, cx, cy,
                 alpha=DEFAULT_ALPHA, storage=SF_FP32, read_flags=0, stream=None,
                 update=SF_UPDATE_PLAIN, eta=None):
        self.rows, self.cols, self.levels = rows, cols, levels
        self.storage = storage
        self.cfg = make_config(rows, cols, levels, max_flow_px, smooth_iters, alpha, storage,
                               update, read_flags)
        self.ctx = sf_create(self.cfg, stream)
        sf_set_camera(self.ctx, fx, fy, cx, cy, eta)

    def push(self, Y, rho, dt, omega=None, acc=None, omega_dot=None):
        if omega is None and acc is None and omega_dot is None:
            sf_push_frame(self.ctx, Y, rho, dt)
        else:
            sf_push_frame_ex(self.ctx, Y, rho, dt, omega, omega_dot, acc)

    def flow(self, kind=SF_FLOW_W_FRAME, out=None):
        import torch
        if out is None:
            out = torch.empty((FLOW_COMPONENTS[kind], self.rows, self.cols), dtype=torch.float32,
                              device="cuda")
        sf_get_flow(self.ctx, kind, out)
        return out

    def update_inputs(self, out=None):
        import torch
        if out is None:
            out = torch.empty((SF_UPDATE_INPUT_PLANES, self.rows, self.cols), dtype=torch.float32,
                              device="cuda")
        sf_get_update_inputs(self.ctx, 0, out)
        return out

    def set_stereo(self, baseline, max_disparity, iterations=3, texture=2.5e-3, residual=0.05):
        sf_set_stereo(self.ctx, 0, baseline, max_disparity, iterations, texture, residual)

    def set_input_stream(self, stream):
        """The stream the pushed frames are produced on (None: the context stream)."""
        sf_set_input_stream(self.ctx, stream)

    def stereo_depth(self, Y_left, Y_right, rho_out=None):
        """The inverse-depth measurement of the left image from the rectified pair."""
        import torch
        if rho_out is None:
            dt = torch.float16 if self.storage == SF_FP16 else torch.float32
            rho_out = torch.empty((self.rows, self.cols), dtype=dt, device="cuda")
        sf_stereo_depth(self.ctx, 0, Y_left, Y_right, rho_out)
        return rho_out

    def set_source_camera(self, fx, fy, cx, cy, rows, cols):
        sf_set_source_camera(self.ctx, 0, fx, fy, cx, cy, rows, cols)

    def map(self, Y_src, rho_src, Y_out=None, rho_out=None):
        """One source-camera frame resampled onto the grid: (Y, rho) tensors of the grid."""
        import torch
        dt = torch.float16 if self.storage == SF_FP16 else torch.float32
        if Y_out is None:
            Y_out = torch.empty((self.rows, self.cols), dtype=dt, device="cuda")
        if rho_out is None:
            rho_out = torch.empty((self.rows, self.cols), dtype=dt, device="cuda")
        sf_map_frame(self.ctx, 0, Y_src, rho_src, Y_out, rho_out)
        return Y_out, rho_out

    def get_state(self):
        return unpack_state(sf_get_state(self.ctx), self.rows, self.cols, self.levels)

    def set_state(self, state, dt_prev, frames=1):
        sf_set_state(self.ctx, pack_state(state, self.rows, self.cols, self.levels, dt_prev, frames))

    def set_learned(self, params, threshold):
        sf_set_learned(self.ctx, params, threshold)

    def learned_stats(self, reset=False):
        return sf_learned_stats(self.ctx, reset)

    def check_state(self):
        """True if every stored flow value was finite since the last check (clears the flag)."""
        return sf_check_state(self.ctx) == 0

    def close(self):
        if self.ctx:
            sf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """Convenience wrapper owning one trainer network over a fixed list of image sizes."""

    def __init__(self, sizes, params, stream=None, loss_eps=None):
        self.sizes = [(int(r), int(c)) for r, c in sizes]
        self.net = sf_net_create(self.sizes, stream)
        sf_net_set_params(self.net, params)
        if loss_eps is not None:
            sf_net_set_loss(self.net, loss_eps)

    def forward(self, inp, out=None):
        import torch
        if out is None:
            out = torch.empty(3 * sum(r * c for r, c in self.sizes), dtype=torch.float32,
                              device="cuda")
        sf_net_forward(self.net, inp, out)
        return out

    def train_step(self, inp, target, lr, want_grad=False):
        return sf_net_train_step(self.net, inp, target, lr, want_grad)

    def params(self):
        return sf_net_get_params(self.net)

    def set_params(self, params):
        sf_net_set_params(self.net, params)

    def close(self):
        if self.net:
            sf_net_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Convenience wrapper owning one batch context (several camera streams)."""

    def __init__(self, specs, storage=SF_FP32, stream=None, update=SF_UPDATE_PLAIN):
        """specs: list of dicts with rows, cols, levels, max_flow_px, smooth, camera (fx, fy,
        cx, cy) and optionally alpha, read_flags."""
        self.specs = list(specs)
        cfgs = [make_config(sp["rows"], sp["cols"], sp["levels"], sp["max_flow_px"], sp["smooth"],
                            sp.get("alpha", DEFAULT_ALPHA), storage, update,
                            sp.get("read_flags", 0)) for sp in self.specs]
        self.ctx = sf_create_batch(cfgs, stream)
        sf_set_cameras(self.ctx, [tuple(sp["camera"]) + ((sp["eta"],) if sp.get("eta") is not None
                                                         else ()) for sp in self.specs])

    def set_input_stream(self, stream):
        """The stream the pushed frames are produced on (None: the context stream)."""
        sf_set_input_stream(self.ctx, stream)

    def push(self, Ys, rhos, dts, omegas=None, accs=None, omega_dots=None):
        if omegas is None and accs is None and omega_dots is None:
            sf_push_frames(self.ctx, Ys, rhos, dts)
        else:
            sf_push_frames_ex(self.ctx, Ys, rhos, dts, omegas, omega_dots, accs)

    def flow(self, stream, kind=SF_FLOW_W_FRAME, out=None):
        import torch
        sp = self.specs[stream]
        if out is None:
            out = torch.empty((FLOW_COMPONENTS[kind], sp["rows"], sp["cols"]), dtype=torch.float32,
                              device="cuda")
        sf_get_flow_stream(self.ctx, stream, kind, out)
        return out

    def flows(self, kind=SF_FLOW_W_FRAME, outs=None):
        """Every stream's output (sf_get_flows); outs: a list of tensors to fill, or None."""
        import torch
        if outs is None:
            outs = [torch.empty((FLOW_COMPONENTS[kind], sp["rows"], sp["cols"]),
                                dtype=torch.float32, device="cuda") for sp in self.specs]
        sf_get_flows(self.ctx, kind, outs)
        return outs

    def update_inputs(self, stream, out=None):
        import torch
        sp = self.specs[stream]
        if out is None:
            out = torch.empty((SF_UPDATE_INPUT_PLANES, sp["rows"], sp["cols"]),
                              dtype=torch.float32, device="cuda")
        sf_get_update_inputs(self.ctx, stream, out)
        return out

    def get_state(self, stream):
        sp = self.specs[stream]
        return unpack_state(sf_get_state_stream(self.ctx, stream), sp["rows"], sp["cols"],
                            sp["levels"])

    def set_learned(self, params, threshold):
        sf_set_learned(self.ctx, params, threshold)

    def learned_stats(self, reset=False):
        return sf_learned_stats(self.ctx, reset)

    def check_state(self):
        """Streams whose stored flow was not finite since the last check (clears the flag)."""
        m = sf_check_state(self.ctx)
        return [s for s in range(len(self.specs)) if (m >> s) & 1]

    def close(self):
        if self.ctx:
            sf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
