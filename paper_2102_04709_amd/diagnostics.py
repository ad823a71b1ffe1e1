"""Measurements on computed phase fields for the paper's validation cases (Sec. III): interface
contours, circle fits, contact angles on flat and circular walls, the angles of a triple
junction, spurious capillary numbers, and the capillary-intrusion front with the analytical
solution of Eq. (24)-(26).  numpy only; the inputs are the mass fractions C_k = rho_k / rho
([3, ny, nx], node (i, j) at (x, y) = (i, j)) and the velocity field.

An interface between fluid sets A and B is the level C_A - C_B = 0 (C_A the summed fractions of
the fluids in A) where the fluids outside A and B are absent (C_A + C_B > purity); its points
are the linearly interpolated crossings along grid rows and columns.  Circles are fitted by
geometric least squares (Gauss-Newton on the point-to-circle distances, started from the
algebraic fit); an interface that is straight to within the fit's resolution is fitted as a line.
"""
from __future__ import annotations

import math
from typing import Iterable, Sequence, Tuple

import numpy as np


def fractions(rho: np.ndarray, solid: np.ndarray) -> np.ndarray:
    """C_k = rho_k / sum_l rho_l at fluid nodes, 0 at solid nodes."""
    fl = np.asarray(solid) == 0
    tot = np.where(fl, rho.sum(0), 1.0)
    return np.where(fl, rho / tot, 0.0)


def _group(C: np.ndarray, fluids) -> np.ndarray:
    idx = [fluids] if isinstance(fluids, (int, np.integer)) else list(fluids)
    return C[idx].sum(0)


def contour(C: np.ndarray, a, b, purity: float = 0.8, solid=None) -> np.ndarray:
    """Points [(x, y)] of the a|b interface (a, b: a fluid index or a list of them)."""
    ca, cb = _group(C, a), _group(C, b)
    d, s = ca - cb, ca + cb
    ok = s > purity
    if solid is not None:
        ok &= np.asarray(solid) == 0
    out = []
    # crossings along x (between (i, j) and (i + 1, j))
    d0, d1 = d[:, :-1], d[:, 1:]
    m = (d0 * d1 < 0) & ok[:, :-1] & ok[:, 1:]
    jj, ii = np.nonzero(m)
    t = d0[jj, ii] / (d0[jj, ii] - d1[jj, ii])
    out.append(np.c_[ii + t, jj])
    # crossings along y
    d0, d1 = d[:-1, :], d[1:, :]
    m = (d0 * d1 < 0) & ok[:-1, :] & ok[1:, :]
    jj, ii = np.nonzero(m)
    t = d0[jj, ii] / (d0[jj, ii] - d1[jj, ii])
    out.append(np.c_[ii, jj + t])
    return np.concatenate(out).astype(float)


class Circle:
    """A fitted circle (or a line when `line` is True: points x with n . x = c)."""

    def __init__(self, cx=0.0, cy=0.0, r=0.0, line=False, n=(0.0, 1.0), c=0.0, rms=0.0):
        self.cx, self.cy, self.r, self.line = cx, cy, r, line
        self.n, self.c, self.rms = np.asarray(n, float), c, rms

    def normal_at(self, x, y) -> np.ndarray:
        if self.line:
            return self.n.copy()
        v = np.array([x - self.cx, y - self.cy])
        return v / np.linalg.norm(v)

    def tangent_at(self, x, y, towards) -> np.ndarray:
        n = self.normal_at(x, y)
        t = np.array([-n[1], n[0]])
        return t if t @ (np.asarray(towards, float) - (x, y)) > 0 else -t

    def meet_horizontal(self, y0: float, near_x: float) -> float:
        """x where the curve crosses the line y = y0, the crossing nearest near_x."""
        if self.line:
            return (self.c - self.n[1] * y0) / self.n[0]
        h = self.r ** 2 - (y0 - self.cy) ** 2
        if h < 0:
            raise ValueError("fitted circle does not reach the wall line")
        xs = (self.cx - math.sqrt(h), self.cx + math.sqrt(h))
        return min(xs, key=lambda v: abs(v - near_x))


def fit_circle(p: np.ndarray, straight_tol: float = 1e-3) -> Circle:
    """Geometric least-squares circle through points p [n, 2]; a line when the points are straight
    (the sagitta over the chord below straight_tol)."""
    p = np.asarray(p, float)
    if len(p) < 3:
        raise ValueError("need at least 3 points")
    m = p.mean(0)
    q = p - m
    u, s, vt = np.linalg.svd(q, full_matrices=False)
    n_line = vt[1]
    chord = 2 * s[0] / math.sqrt(len(p)) * math.sqrt(3)  # extent of the points along the line
    if s[1] / math.sqrt(len(p)) < straight_tol * max(chord, 1.0):
        return Circle(line=True, n=n_line, c=float(n_line @ m), rms=float(s[1] / math.sqrt(len(p))))
    # algebraic start: |q|^2 = 2 a.q + k
    A = np.c_[2 * q, np.ones(len(q))]
    sol, *_ = np.linalg.lstsq(A, (q ** 2).sum(1), rcond=None)
    c = sol[:2]
    r = math.sqrt(max(sol[2] + c @ c, 1e-12))
    for _ in range(50):  # Gauss-Newton on d_i = |q_i - c| - r
        v = q - c
        dist = np.hypot(v[:, 0], v[:, 1])
        res = dist - r
        J = np.c_[-v[:, 0] / dist, -v[:, 1] / dist, -np.ones(len(q))]
        step, *_ = np.linalg.lstsq(J, -res, rcond=None)
        c = c + step[:2]
        r = r + step[2]
        if np.abs(step).max() < 1e-12 * max(1.0, r):
            break
    v = q - c
    res = np.hypot(v[:, 0], v[:, 1]) - r
    if r > 1e4 * max(chord, 1.0):  # numerically a line
        return Circle(line=True, n=n_line, c=float(n_line @ m), rms=float(np.sqrt((res ** 2).mean())))
    return Circle(c[0] + m[0], c[1] + m[1], abs(r), rms=float(np.sqrt((res ** 2).mean())))


def flat_contact_angle(C: np.ndarray, a, b, inside, wall_y: float = 0.5, band=(2.0, 40.0),
                       x_range=None) -> float:
    """Contact angle (degrees) of the a|b interface on the flat wall y = wall_y (above it),
    measured inside the fluid set `inside`: the interface points with wall_y + band[0] <= y <=
    wall_y + band[1] (and x in x_range) are fitted, the fit is followed to the wall, and the angle
    lies between its tangent there and the wall on the side of `inside`."""
    p = contour(C, a, b)
    sel = (p[:, 1] >= wall_y + band[0]) & (p[:, 1] <= wall_y + band[1])
    if x_range is not None:
        sel &= (p[:, 0] >= x_range[0]) & (p[:, 0] <= x_range[1])
    p = p[sel]
    fit = fit_circle(p)
    lowest = p[p[:, 1] <= p[:, 1].min() + 1.5, 0].mean()
    xa = fit.meet_horizontal(wall_y, lowest)
    t = fit.tangent_at(xa, wall_y, (xa, wall_y + 10.0))
    ci = _group(C, inside)
    ny, nx = C.shape[1:]
    j = int(round(wall_y + 2.0))
    left, right = ci[j, int(math.floor(xa - 3)) % nx], ci[j, int(math.ceil(xa + 3)) % nx]
    w = np.array([1.0, 0.0]) if right > left else np.array([-1.0, 0.0])
    return math.degrees(math.acos(float(np.clip(t @ w, -1.0, 1.0))))


def cylinder_contact_angle(C: np.ndarray, drop, ambient, cylinder: Tuple[float, float, float],
                           margin: float = 3.0) -> dict:
    """Eq. (23), Sec. III B: fit the droplet's outer contour (drop | ambient, points farther than
    R_s + margin from the cylinder centre) with a circle of radius R_j and centre O_j; the angle
    inside the droplet follows from the law of cosines D_sj^2 = R_s^2 + R_j^2 - 2 R_s R_j cos(theta)."""
    cx, cy, Rs = cylinder
    p = contour(C, drop, ambient, purity=0.5)
    p = p[np.hypot(p[:, 0] - cx, p[:, 1] - cy) > Rs + margin]
    fit = fit_circle(p)
    D = math.hypot(fit.cx - cx, fit.cy - cy)
    cos = (Rs ** 2 + fit.r ** 2 - D ** 2) / (2 * Rs * fit.r)
    return {"theta": math.degrees(math.acos(max(-1.0, min(1.0, cos)))), "R_j": fit.r, "D_sj": D,
            "rms": fit.rms}


def eq23_distance(Rs: float, Rj: float, theta_deg: float) -> float:
    """D_sj of Eq. (23) (law of cosines in the triangle O_j A O_s)."""
    return math.sqrt(Rs * Rs + Rj * Rj - 2 * Rs * Rj * math.cos(math.radians(theta_deg)))


def junction_angles(C: np.ndarray, near, radius: float, exclude: float = 3.0) -> dict:
    """Interior angles (degrees) inside fluids 0, 1, 2 at the triple junction near `near`: the three
    pair interfaces are fitted within `radius` of it (but beyond `exclude`); the junction is the
    point nearest to all three fits (least squares over their tangent lines, iterated), and the
    angle inside fluid m lies between the two interfaces that bound m."""
    near = np.asarray(near, float)
    pairs = ((0, 1), (0, 2), (1, 2))
    fits, cent = {}, {}
    for k, l in pairs:
        p = contour(C, k, l)
        r = np.hypot(p[:, 0] - near[0], p[:, 1] - near[1])
        p = p[(r < radius) & (r > exclude)]
        fits[(k, l)] = fit_circle(p)
        cent[(k, l)] = p.mean(0)
    J = near.copy()
    for _ in range(30):  # the point closest to the three curves
        rows, rhs = [], []
        for key, f in fits.items():
            n = f.normal_at(*J)
            if f.line:
                d = f.c - n @ J
            else:
                d = f.r - math.hypot(J[0] - f.cx, J[1] - f.cy)
            rows.append(n)
            rhs.append(d)
        step, *_ = np.linalg.lstsq(np.array(rows), np.array(rhs), rcond=None)
        J = J + step
        if np.abs(step).max() < 1e-10:
            break
    t = {key: f.tangent_at(J[0], J[1], cent[key]) for key, f in fits.items()}

    def between(a, b):
        return math.degrees(math.acos(float(np.clip(t[a] @ t[b], -1.0, 1.0))))

    ang = [between((0, 1), (0, 2)), between((0, 1), (1, 2)), between((0, 2), (1, 2))]
    return {"angles": ang, "junction": J.tolist()}


def neumann_angles(sigma12: float, sigma13: float, sigma23: float) -> list:
    """Interior angles (degrees) inside fluids 1, 2, 3 of the Neumann triangle of the tensions:
    the angle inside fluid m lies between the two interfaces bounding m and faces the tension of
    the third pair."""
    def a(opp, s1, s2):
        return math.degrees(math.acos((opp * opp - s1 * s1 - s2 * s2) / (2 * s1 * s2)))
    return [a(sigma23, sigma12, sigma13), a(sigma13, sigma12, sigma23), a(sigma12, sigma13, sigma23)]


def spurious(u: np.ndarray, solid, mu: float, sigma: float) -> dict:
    """|u|_max over fluid nodes and the spurious capillary number Ca = |u|_max mu / sigma (Sec. III A)."""
    fl = np.asarray(solid) == 0
    umax = float(np.hypot(u[0], u[1])[fl].max())
    return {"umax": umax, "Ca": umax * mu / sigma}


# ---- Sec. III C: capillary intrusion of ternary fluids -------------------------------------

def front_position(C: np.ndarray, a, b, rows: Iterable[int]) -> float:
    """Mean x of the a|b interface over the given rows (the crossing of C_a - C_b along x)."""
    xs = []
    ca, cb = _group(C, a), _group(C, b)
    for j in rows:
        d = ca[j] - cb[j]
        i = np.nonzero((d[:-1] > 0) & (d[1:] <= 0))[0]
        if len(i):
            i = i[0]
            xs.append(i + d[i] / (d[i] - d[i + 1]))
    return float(np.mean(xs)) if xs else float("nan")


def intrusion_eq25(t, s0: float, L: float, Lg: float, H: float, sigma_gb: float, theta_gb_deg: float,
                   sigma_gr: float, theta_gr_deg: float, mu_r: float, mu_g: float, mu_b: float):
    """s(t) of Eq. (25)-(26) for the front between red and green (Sec. III C):
    A = H (sigma_gb cos theta_gb - sigma_gr cos theta_gr) / 6, B = mu_g Lg + mu_b (L - Lg),
    C = mu_r - mu_b; s = (A / B) t + s0 if C = 0, else s = (-B + sqrt(B^2 - 2 C f)) / C with
    f = -C s0^2 / 2 - B s0 - A t."""
    t = np.asarray(t, float)
    A = H * (sigma_gb * math.cos(math.radians(theta_gb_deg)) - sigma_gr * math.cos(math.radians(theta_gr_deg))) / 6.0
    B = mu_g * Lg + mu_b * (L - Lg)
    Cc = mu_r - mu_b
    if abs(Cc) < 1e-300:
        return A / B * t + s0
    f = -0.5 * Cc * s0 * s0 - B * s0 - A * t
    return (-B + np.sqrt(B * B - 2 * Cc * f)) / Cc


def intrusion_eq24_rate(s: float, L: float, Lg: float, H: float, sigma_gb: float, theta_gb_deg: float,
                        sigma_gr: float, theta_gr_deg: float, mu_r: float, mu_g: float, mu_b: float) -> float:
    """ds/dt of Eq. (24)."""
    num = sigma_gb * math.cos(math.radians(theta_gb_deg)) - sigma_gr * math.cos(math.radians(theta_gr_deg))
    return H / 6.0 * num / (mu_r * s + mu_g * Lg + mu_b * (L - Lg - s))
