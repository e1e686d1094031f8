"""CPU checks of the boundary: the built library loads and exports every function that
include/sflow.h declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sflow.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("sf_create", "sf_set_camera", "sf_push_frame", "sf_get_flow", "sf_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2406_18031_amd", "libsflow.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2406_18031_amd import sflow
    assert set(_declared()) <= set(sflow.EXPORTED)


def test_create_without_device_fails_cleanly():
    from paper_2406_18031_amd import sflow
    import torch
    if torch.cuda.is_available():
        return
    cfg = sflow.make_config(64, 64, 1, 1.0, [2])
    try:
        sflow.sf_create(cfg, 0)
    except sflow.SflowError as e:
        assert e.status in (sflow.SF_ERR_HIP, sflow.SF_ERR_OOM)
        assert sflow.sf_last_error(None)
    else:
        raise AssertionError("create succeeded without a device")
