"""An independent per-pixel version of the filter for tiny images (brute force).

It re-derives every step pixel by pixel with explicit loops and explicit border
handling, and solves both least-squares problems as weighted least squares on their
stacked residual rows (np.linalg.lstsq) instead of through normal equations, so it
pins the vectorised oracle in filter.py against a second reading of the same text.
Only suitable for images of a few dozen pixels.
"""
from __future__ import annotations

import math

import numpy as np

from .readings import DEFAULT_ALPHA, Readings, gammas, iterations

G = [1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16]


def _cl(v, n):
    return 0 if v < 0 else (n - 1 if v > n - 1 else v)


def _eta(i, j, fx, fy, cx, cy):
    r = np.array([(j - cx) / fx, (i - cy) / fy, 1.0])
    return r / math.sqrt(r @ r)


def _geometry(R, C, fx, fy, cx, cy, ray=None):
    """Per-pixel (eta, P, b1, b2, dmu); ray(i, j) gives the unit direction of a general grid
    (default: the pinhole of the intrinsics)."""
    if ray is None:
        def ray(i, j):
            return _eta(i, j, fx, fy, cx, cy)
    geo = {}
    for i in range(R):
        for j in range(C):
            e = ray(i, j)
            P = np.eye(3) - np.outer(e, e)
            if j + 1 < C:
                q = P @ ray(i, j + 1)
                b1 = q / np.linalg.norm(q)
            else:
                q = P @ ray(i, j - 1)
                b1 = -q / np.linalg.norm(q)
            dmu = float(np.linalg.norm(q))
            b2 = np.cross(e, b1)
            b2 = b2 / np.linalg.norm(b2)
            if i + 1 < R:
                if b2 @ ray(i + 1, j) < 0:
                    b2 = -b2
            elif i - 1 >= 0:
                if b2 @ ray(i - 1, j) > 0:
                    b2 = -b2
            geo[i, j] = (e, P, b1, b2, dmu)
    return geo


def _blur_decimate(Y):
    R, C = Y.shape
    out = np.zeros(((R + 1) // 2, (C + 1) // 2))
    for I in range(out.shape[0]):
        for J in range(out.shape[1]):
            s = 0.0
            for a in range(5):
                for b in range(5):
                    s += G[a] * G[b] * Y[_cl(2 * I + a - 2, R), _cl(2 * J + b - 2, C)]
            out[I, J] = s
    return out


def _blur_decimate_valid(rho):
    R, C = rho.shape
    out = np.zeros(((R + 1) // 2, (C + 1) // 2))
    for I in range(out.shape[0]):
        for J in range(out.shape[1]):
            num = den = 0.0
            for a in range(5):
                for b in range(5):
                    v = rho[_cl(2 * I + a - 2, R), _cl(2 * J + b - 2, C)]
                    if not math.isnan(v):
                        num += G[a] * G[b] * v
                        den += G[a] * G[b]
            out[I, J] = num / den if den > 0 else float("nan")
    return out


def _image_model(Y, i, j):
    """Weighted LS fit of Y_q ~ c + g1 (q_j - j) + g2 (q_i - i) over the 5x5 window."""
    R, C = Y.shape
    rows, rhs = [], []
    for a in range(-2, 3):
        for b in range(-2, 3):
            wgt = math.sqrt(G[a + 2] * G[b + 2])
            rows.append([wgt, wgt * b, wgt * a])
            rhs.append(wgt * Y[_cl(i + a, R), _cl(j + b, C)])
    sol = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
    return sol[0], sol[1], sol[2]


def _depth_grad(rho, i, j):
    R, C = rho.shape
    if math.isnan(rho[i, j]):
        return 0.0, 0.0
    out = []
    for (pi, pj), (mi, mj) in (((i, _cl(j + 1, C)), (i, _cl(j - 1, C))),
                               ((_cl(i + 1, R), j), (_cl(i - 1, R), j))):
        fwd = rho[pi, pj] - rho[i, j]
        bwd = rho[i, j] - rho[mi, mj]
        if math.isnan(fwd) and math.isnan(bwd):
            out.append(0.0)
        elif math.isnan(fwd):
            out.append(bwd)
        elif math.isnan(bwd):
            out.append(fwd)
        else:
            out.append(fwd if abs(fwd) <= abs(bwd) else bwd)
    return out[0], out[1]


def _half_step(fields, geo, R, C, N, axis, rd):
    """fields: dict name -> dict[(i, j)] -> value (float or 3-vector)."""
    dt = 1.0 / N
    w = fields["w"]

    def comp(i, j):
        e, P, b1, b2, dmu = geo[i, j]
        b = b1 if axis == 1 else b2
        return float(b @ (P @ w[i, j])) / dmu

    new = {k: {} for k in fields}
    for i in range(R):
        for j in range(C):
            if axis == 1:
                prev, nxt = (i, _cl(j - 1, C)), (i, _cl(j + 1, C))
            else:
                prev, nxt = (_cl(i - 1, R), j), (_cl(i + 1, R), j)
            up, un = comp(*prev), comp(*nxt)
            if rd.dominant_literal:
                uh = up if abs(un) > abs(up) else un
            else:
                uh = un if abs(un) > abs(up) else up
            if rd.cfl_clamp:
                uh = min(max(uh, -N), N)
            e = geo[i, j][0]
            s = float(e @ w[i, j])
            for name, f in fields.items():
                if uh > 0:
                    D = f[i, j] - f[prev]
                else:
                    D = f[nxt] - f[i, j]
                sig = 0.0 if name == "Y" else rd.sigma
                new[name][i, j] = f[i, j] - dt * (uh * D + sig * f[i, j] * s)
    return new


def _cross(a, b):
    return np.array([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def _inertial_step(fields, geo, R, C, N, om, dom, acc):
    """Explicit step 1/N of the inertial source terms, pixel by pixel: w gains
    -2 Omega x w - (Omega (Omega . eta) - eta |Omega|^2) - dOmega x eta - rho a, dw gains
    -2 Omega x dw."""
    dt = 1.0 / N
    new = {k: dict(v) for k, v in fields.items()}
    oo = float(om @ om)
    for i in range(R):
        for j in range(C):
            e = geo[i, j][0]
            w = fields["w"][i, j]
            cen = om * float(om @ e) - e * oo
            new["w"][i, j] = w + dt * (-2.0 * _cross(om, w) - cen - _cross(dom, e)
                                       - fields["rho"][i, j] * acc)
            if "dw" in fields:
                new["dw"][i, j] = fields["dw"][i, j] - 2.0 * dt * _cross(om, fields["dw"][i, j])
    return new


def _to_dict(a):
    R, C = a.shape[:2]
    return {(i, j): (a[i, j].copy() if a.ndim == 3 else float(a[i, j]))
            for i in range(R) for j in range(C)}


def _to_array(d, R, C, vec):
    out = np.zeros((R, C, 3)) if vec else np.zeros((R, C))
    for (i, j), v in d.items():
        out[i, j] = v
    return out


def _box(x, R, C):
    out = np.zeros_like(x)
    for i in range(R):
        for j in range(C):
            s = np.zeros(3)
            for a in range(-2, 3):
                for b in range(-2, 3):
                    s = s + x[_cl(i + a, R), _cl(j + b, C)]
            out[i, j] = s / 25.0
    return out


def _up(W, R, C):
    Rc, Cc = W.shape[:2]
    out = np.zeros((R, C, 3))
    for i in range(R):
        for j in range(C):
            yi, xj = i / 2.0, j / 2.0
            i0, j0 = int(math.floor(yi)), int(math.floor(xj))
            ti, tj = yi - i0, xj - j0
            v = np.zeros(3)
            for di, wi in ((0, 1 - ti), (1, ti)):
                for dj, wj in ((0, 1 - tj), (1, tj)):
                    if wi * wj != 0:
                        v = v + wi * wj * W[_cl(i0 + di, Rc), _cl(j0 + dj, Cc)]
            out[i, j] = v
    return out


class LiteralFilter:
    """Same interface as oracle.Filter (push / flow('w_frame') / state)."""

    def __init__(self, rows, cols, levels, max_flow_px, smooth_iters, fx, fy, cx, cy,
                 alpha=DEFAULT_ALPHA, readings=Readings(), eta=None):
        self.R, self.C, self.H = rows, cols, levels
        self.smooth = list(smooth_iters)
        self.rd = readings
        self.sizes, self.geos, self.N, self.gam = [], [], [], []
        r, c = rows, cols
        for h in range(1, levels + 1):
            s = 2.0 ** (h - 1)
            self.sizes.append((r, c))
            if eta is None:
                self.geos.append(_geometry(r, c, fx / s, fy / s, cx / s, cy / s))
            else:
                step = int(s)

                def ray(i, j, step=step):
                    return np.asarray(eta[i * step, j * step], dtype=float)
                self.geos.append(_geometry(r, c, fx / s, fy / s, cx / s, cy / s, ray))
            self.N.append(max(1, math.ceil(max_flow_px / s)))
            self.gam.append(gammas(alpha, fx / s))
            r, c = (r + 1) // 2, (c + 1) // 2
        assert self.N == [iterations(max_flow_px, h) for h in range(1, levels + 1)]
        self.state = None
        self.dt_prev = None

    def push(self, Y, rho, dt, omega=None, acc=None, omega_dot=None):
        Ys, rhos = [np.asarray(Y, float)], [np.asarray(rho, float)]
        for _ in range(1, self.H):
            Ys.append(_blur_decimate(Ys[-1]))
            rhos.append(_blur_decimate_valid(rhos[-1]))
        models = []
        for h in range(self.H):
            R, C = self.sizes[h]
            m = {}
            for i in range(R):
                for j in range(C):
                    m[i, j] = (_image_model(Ys[h], i, j), _depth_grad(rhos[h], i, j))
            models.append(m)
        if self.state is None:
            self.state = []
            for h in range(self.H):
                R, C = self.sizes[h]
                Yhat = np.array([[models[h][i, j][0][0] for j in range(C)] for i in range(R)])
                rr = np.where(np.isnan(rhos[h]), 0.0, rhos[h])
                st = {"w": np.zeros((R, C, 3)), "rho": rr, "Y": Yhat}
                if h < self.H - 1:
                    st["dw"] = np.zeros((R, C, 3))
                self.state.append(st)
            self.dt_prev = dt
            return
        if dt != self.dt_prev:
            for st in self.state:
                for k in ("w", "dw"):
                    if k in st:
                        st[k] = st[k] * (dt / self.dt_prev)
        xs, rhonew = [], []
        for h in range(self.H):
            R, C = self.sizes[h]
            geo, st, N = self.geos[h], self.state[h], self.N[h]
            top = h == self.H - 1
            names = ("w", "rho") if top else ("w", "dw", "rho", "Y")
            f = {k: _to_dict(st[k]) for k in names}
            for _ in range(N):
                f = _half_step(f, geo, R, C, N, 1, self.rd)
                f = _half_step(f, geo, R, C, N, 0, self.rd)
                if omega is not None or acc is not None or omega_dot is not None:
                    om = np.zeros(3) if omega is None else np.asarray(omega, float) * dt
                    do = np.zeros(3) if omega_dot is None else np.asarray(omega_dot, float) * dt * dt
                    ac = np.zeros(3) if acc is None else np.asarray(acc, float) * dt * dt
                    f = _inertial_step(f, geo, R, C, N, om, do, ac)
            g1, g2, g3, g4, g5 = self.gam[h]
            x = np.zeros((R, C, 3))
            rn = np.zeros((R, C))
            for i in range(R):
                for j in range(C):
                    e, P, b1, b2, dmu = geo[i, j]
                    (c0, gy1, gy2), (gr1, gr2) = models[h][i, j]
                    gradY = dmu * (b1 * gy1 + b2 * gy2)
                    gradR = dmu * (b1 * gr1 + b2 * gr2)
                    if top:
                        x0, Yp, rp = f["w"][i, j], st["Y"][i, j], st["rho"][i, j]
                    else:
                        x0, Yp, rp = f["dw"][i, j], f["Y"][i, j], f["rho"][i, j]
                    meas = rhos[h][i, j]
                    rows = [math.sqrt(g1) * (P @ gradY)]
                    rhs = [-math.sqrt(g1) * dmu * dmu * (c0 - Yp)]
                    if not math.isnan(meas):
                        rows.append(math.sqrt(g2) * (P @ gradR + dmu * dmu * meas * e))
                        rhs.append(-math.sqrt(g2) * dmu * dmu * (meas - rp))
                    for k in range(3):
                        unit = np.zeros(3)
                        unit[k] = math.sqrt(g3)
                        rows.append(unit)
                        rhs.append(math.sqrt(g3) * x0[k])
                    x[i, j] = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)[0]
                    pr = f["rho"][i, j]
                    rn[i, j] = pr if math.isnan(meas) else (g4 * meas + g5 * pr) / (g4 + g5)
            for _ in range(self.smooth[h]):
                x = _box(x, R, C)
            xs.append(x)
            rhonew.append(rn)
        self.state[-1]["w"] = xs[-1]
        for h in range(self.H - 2, -1, -1):
            R, C = self.sizes[h]
            self.state[h]["dw"] = xs[h]
            self.state[h]["w"] = _up(self.state[h + 1]["w"], R, C) + xs[h]
        for h in range(self.H):
            R, C = self.sizes[h]
            self.state[h]["rho"] = rhonew[h]
            self.state[h]["Y"] = np.array([[models[h][i, j][0][0] for j in range(C)]
                                           for i in range(R)])
        self.dt_prev = dt

    def flow(self, kind="w_frame"):
        assert kind == "w_frame"
        return self.state[0]["w"].copy()
