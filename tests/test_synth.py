"""The synthetic renderer's ground truth against finite differences of its own ray hits:
eta_dot = P_eta w (eq:optical_flow) and rho_dot = -rho <eta, w> (eq:totaldev_invdepth)."""
import numpy as np
import pytest
import torch

from synth.scenes import Sequence, box_sequence, sinusoid_plane_sequence


def _fd_check(seq: Sequence, k: int):
    """Track the scene points seen at frame k to frames k-1 and k+1 and compare the central
    differences of their directions and inverse depths with the rendered flow."""
    eta = seq.camera.rays().numpy()
    f = seq.frame(k)
    rho = f.rho_true.numpy()
    w = f.w_gt.numpy()
    ok = rho > 0
    lam = np.where(ok, 1.0 / np.where(ok, rho, 1.0), 0.0)
    X = seq.ps[k] + (lam[..., None] * eta) @ seq.Rs[k].T          # world points
    dirs, rhos = [], []
    for kk in (k - 1, k + 1):
        xc = (X - seq.ps[kk]) @ seq.Rs[kk]                          # R^T (X - p)
        n = np.linalg.norm(xc, axis=-1, keepdims=True)
        dirs.append(xc / n)
        rhos.append(1.0 / n[..., 0])
    h = seq.dt
    eta_dot = (dirs[1] - dirs[0]) / (2 * h)
    rho_dot = (rhos[1] - rhos[0]) / (2 * h)
    Pw = w - eta * np.sum(eta * w, -1, keepdims=True)
    m = ok
    scale = np.abs(Pw[m]).max()
    assert np.abs(eta_dot[m] - Pw[m]).max() < 1e-4 * scale
    ref = -rho * np.sum(eta * w, -1)
    assert np.abs(rho_dot[m] - ref[m]).max() < 1e-4 * np.abs(ref[m]).max() + 1e-12


def _fine(seq: Sequence, h: float) -> Sequence:
    """The same scene and motion sampled every h seconds."""
    return Sequence(seq.camera, seq.scene, seq.traj, h, 5)


def test_plane_ground_truth_kinematics():
    _fd_check(_fine(sinusoid_plane_sequence(32, 32, 5, seed=11, dt=1e-3), 1e-6), 2)


def test_box_scene_ground_truth_kinematics():
    _fd_check(_fine(box_sequence(48, 48, 5, seed=12, dt=1e-3, depth_noise=0.0), 1e-6), 2)


def test_sequences_are_seeded():
    a = box_sequence(32, 32, 3, seed=9).frame(2)
    b = box_sequence(32, 32, 3, seed=9).frame(2)
    assert torch.equal(a.Y, b.Y) and torch.equal(a.rho, b.rho)
    c = box_sequence(32, 32, 3, seed=10).frame(2)
    assert not torch.equal(a.Y, c.Y)


def test_flow_budget():
    seq = box_sequence(64, 64, 2, seed=13, max_flow_px=4.0)
    assert seq.max_flow_px(0) == pytest.approx(0.85 * 4.0, rel=1e-9)
