"""Angle measurements on computed phase fields for the oracle's physics pins (Sec. III A, III B).

An interface between fluids k and l is the zero level of C_k - C_l where the third fluid is
absent (C_k + C_l > 0.8); its points are the linear-interpolation crossings along grid rows and
columns.  A circle (or, in the limit, a line) is fitted to them by the Pratt algebraic fit, which
treats both alike: A (x^2 + y^2) + D x + E y + F = 0 with D^2 + E^2 - 4 A F = 1.  Contact angles
are read where the fitted curve meets the wall, junction angles from the fitted curves' tangents
where they meet.
"""
import math

import numpy as np


def interface_points(C, k, l, ymin=-1e9, ymax=1e9, purity=0.8):
    d = C[k] - C[l]
    s = C[k] + C[l]
    ny, nx = d.shape
    pts = []
    for j in range(ny):
        if not (ymin <= j <= ymax):
            continue
        a, b = d[j, :-1], d[j, 1:]
        ii = np.nonzero((a * b < 0) & (s[j, :-1] > purity) & (s[j, 1:] > purity))[0]
        for i in ii:
            pts.append((i + a[i] / (a[i] - b[i]), j))
    for j in range(ny - 1):
        a, b = d[j], d[j + 1]
        ii = np.nonzero((a * b < 0) & (s[j] > purity) & (s[j + 1] > purity))[0]
        for i in ii:
            y = j + a[i] / (a[i] - b[i])
            if ymin <= y <= ymax:
                pts.append((i, y))
    return np.array(pts, dtype=float).reshape(-1, 2)


def pratt_fit(p):
    """(A, D, E, F) of A (x^2 + y^2) + D x + E y + F = 0 through points p (Pratt's constraint)."""
    c = p.mean(0)
    q = p - c
    z = (q ** 2).sum(1)
    Z = np.c_[z, q[:, 0], q[:, 1], np.ones(len(q))]
    M = Z.T @ Z
    B = np.array([[0, 0, 0, -2.0], [0, 1, 0, 0], [0, 0, 1, 0], [-2.0, 0, 0, 0]])
    w, v = np.linalg.eig(np.linalg.solve(B, M) if False else np.linalg.pinv(B) @ M)
    w = np.real(w)
    v = np.real(v)
    best = None
    for i in range(4):
        th = v[:, i]
        nrm = th @ B @ th
        if nrm <= 0:
            continue
        th = th / math.sqrt(nrm)
        res = th @ M @ th
        if best is None or res < best[0]:
            best = (res, th)
    A, D, E, F = best[1]
    # back to the original coordinates: x = q + c
    cx, cy = c
    D2 = D - 2 * A * cx
    E2 = E - 2 * A * cy
    F2 = F + A * (cx * cx + cy * cy) - D * cx - E * cy
    return np.array([A, D2, E2, F2])


def conic_gradient(th, x, y):
    A, D, E, F = th
    return np.array([2 * A * x + D, 2 * A * y + E])


def wall_contact(th, yw, near_x):
    """Intersection of the fitted curve with the line y = yw nearest to near_x."""
    A, D, E, F = th
    c0 = A * yw * yw + E * yw + F
    if abs(A) < 1e-14:
        return -c0 / D
    disc = D * D - 4 * A * c0
    r = math.sqrt(max(disc, 0.0))
    xs = [(-D + r) / (2 * A), (-D - r) / (2 * A)]
    return min(xs, key=lambda v: abs(v - near_x))


def tangent_into(th, x, y, towards):
    g = conic_gradient(th, x, y)
    t = np.array([-g[1], g[0]]) / np.hypot(*g)
    return t if t @ (np.asarray(towards, float) - (x, y)) > 0 else -t


def contact_angle(C, k, l, m, yw, band, side_probe=2.0):
    """Angle (degrees) between the wall y = yw and the k|l interface where it meets the wall,
    measured inside fluid m (k or l).  band = (y0, y1): rows whose interface points are fitted."""
    p = interface_points(C, k, l, yw + band[0], yw + band[1])
    th = pratt_fit(p)
    low = p[p[:, 1] <= p[:, 1].min() + 2.0]
    xa = wall_contact(th, yw, low[:, 0].mean())
    t = tangent_into(th, xa, yw, (xa, yw + 10.0))
    # which way along the wall lies fluid m: probe a little above the wall on either side
    ny, nx = C.shape[1:]
    j = int(round(yw + 1.5))
    il, ir = int(math.floor(xa - side_probe)), int(math.ceil(xa + side_probe))
    wdir = np.array([1.0, 0.0]) if C[m, j, ir % nx] > C[m, j, il % nx] else np.array([-1.0, 0.0])
    return math.degrees(math.acos(float(np.clip(t @ wdir, -1, 1)))), th, (xa, yw)


def curve_intersections(t1, t2, guess):
    """Intersection of two fitted curves nearest to guess (Newton from the guess)."""
    x = np.array(guess, float)
    for _ in range(60):
        f = np.array([t1[0] * (x @ x) + t1[1] * x[0] + t1[2] * x[1] + t1[3],
                      t2[0] * (x @ x) + t2[1] * x[0] + t2[2] * x[1] + t2[3]])
        J = np.array([conic_gradient(t1, *x), conic_gradient(t2, *x)])
        dx = np.linalg.solve(J, -f)
        x = x + dx
        if np.abs(dx).max() < 1e-12:
            break
    return x


def junction_angles(C, near, radius, exclude=2.0):
    """Interior angles (degrees, inside fluids 0, 1, 2) at the triple junction near `near`, from
    the three pair interfaces fitted within `radius` of it (beyond `exclude`): the junction is where
    the 0|1 and 1|2... fits meet (the intersection of the two fits nearest `near`); each fit's
    tangent there points along its own interface; the angle inside fluid m lies between the two
    interfaces that bound m."""
    near = np.asarray(near, float)
    fits, cents = {}, {}
    for k, l in ((0, 1), (0, 2), (1, 2)):
        p = interface_points(C, k, l)
        r = np.hypot(*(p - near).T)
        p = p[(r < radius) & (r > exclude)]
        fits[(k, l)] = pratt_fit(p)
        cents[(k, l)] = p.mean(0)
    J = curve_intersections(fits[(0, 1)], fits[(1, 2)], near)
    tang = {}
    for key, th in fits.items():
        tang[key] = tangent_into(th, J[0], J[1], cents[key])
    def ang(a, b):
        return math.degrees(math.acos(float(np.clip(tang[a] @ tang[b], -1, 1))))
    return np.array([ang((0, 1), (0, 2)), ang((0, 1), (1, 2)), ang((0, 2), (1, 2))]), J
