"""State update (Section "State update", eq:cost_top, eq:img_cost_top,
eq:invdepth_cost_top, eq:LS_update, eq:cost_bottom, eq:cost_invdepth).

Per pixel the new flow x (w at the top level, dw at lower levels) minimises

    gamma_1 E_Y^2 + gamma_2 E_rho^2 + gamma_3 |x - x0|^2
    E_Y   = grad_Y^T P x + dmu^2 (Yhat_new - Y_prev)
    E_rho = grad_rho^T P x + dmu^2 ((rhohat_new - rho_prev) + rhohat_new <eta, x>)

with x0 the predicted flow (the printed top-level E_t has a '+', read as '-' as at the
lower levels).  Top level: Y_prev = Yhat of frame k (stored), rho_prev = rho^k (stored).
Lower levels: Y_prev = predicted Yhat^{k+}, rho_prev = rho^{k+}.  gamma_2 = 0 where the
depth is missing.  Writing E_Y = a_Y . x + c_Y and E_rho = a_rho . x + c_rho gives the
3x3 normal equations

    (gamma_1 a_Y a_Y^T + gamma_2 a_rho a_rho^T + gamma_3 I) x
        = -gamma_1 c_Y a_Y - gamma_2 c_rho a_rho + gamma_3 x0,

solved here with a dense solver.  The solution is then smoothed by N_s passes of the 5x5
average (clamped borders).  Inverse depth: rho = (gamma_4 rhohat + gamma_5 rho^{k+}) /
(gamma_4 + gamma_5), or rho^{k+} where the measurement is missing.
"""
from __future__ import annotations

import numpy as np

from .models import _clamped


def ls_terms(grid, gradY, Ynew, Yprev, gradrho, rhonew, rhoprev):
    """a_Y, c_Y, a_rho, c_rho per pixel (rhonew NaN -> terms are NaN-free zeros)."""
    P = grid.P
    dmu2 = grid.dmu ** 2
    a_Y = np.einsum("rcab,rcb->rca", P, gradY)
    c_Y = dmu2 * (Ynew - Yprev)
    valid = ~np.isnan(rhonew)
    rn = np.where(valid, rhonew, 0.0)
    a_r = np.einsum("rcab,rcb->rca", P, gradrho) + (dmu2 * rn)[..., None] * grid.eta
    c_r = dmu2 * (rn - np.where(valid, rhoprev, 0.0))
    return a_Y, c_Y, a_r, c_r, valid


def ls_solve(a_Y, c_Y, a_r, c_r, valid, x0, g1, g2, g3):
    g2p = np.where(valid, g2, 0.0)
    A = (g1 * a_Y[..., :, None] * a_Y[..., None, :]
         + g2p[..., None, None] * a_r[..., :, None] * a_r[..., None, :]
         + g3 * np.eye(3))
    b = -g1 * c_Y[..., None] * a_Y - (g2p * c_r)[..., None] * a_r + g3 * x0
    return np.linalg.solve(A, b[..., None])[..., 0]


def box5(x: np.ndarray) -> np.ndarray:
    """One pass of the 5x5 average with clamped borders."""
    acc = np.zeros_like(x)
    for a in range(-2, 3):
        for b in range(-2, 3):
            acc += _clamped(x, a, b)
    return acc / 25.0


def smooth(x: np.ndarray, passes: int) -> np.ndarray:
    for _ in range(passes):
        x = box5(x)
    return x


def rho_update(rhonew, rhopred, g4, g5):
    valid = ~np.isnan(rhonew)
    return np.where(valid, (g4 * np.where(valid, rhonew, 0.0) + g5 * rhopred) / (g4 + g5),
                    rhopred)
