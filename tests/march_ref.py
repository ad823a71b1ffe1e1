"""Brute-force reference of the characteristic-line crossing (Sec. II B) for the oracle's pins."""
import numpy as np


def brute_force_march(solid, y_periodic, pi, pj, dx, dy, t_max=24.0, eps=1e-9):
    """The characteristic-line crossing of the wetting fill written straight from its reading:
    every crossing of the ray (pi, pj) + t (dx, dy), 0 < t <= t_max, with a grid line x = integer
    or y = integer, in increasing t; a crossing within eps of a node is that node, otherwise the
    two nodes of the crossed grid line bracket it; the first crossing whose nodes are all fluid is
    the hit.  Periodic x; y periodic or solid outside the grid.  Returns (ok, n0, n1, w) with the
    nodes mapped into the grid (rows outside a non-periodic y axis clamped to -2 .. ny + 1)."""
    ny, nx = solid.shape

    def mapped(i, j):
        i %= nx
        j = j % ny if y_periodic else min(max(j, -2), ny + 1)
        return i, j

    def fluid(i, j):
        i, j = mapped(i, j)
        return 0 <= j < ny and solid[j, i] == 0

    cands = []  # (t, kind, line index)
    for d, p, kind in ((dx, pi, "v"), (dy, pj, "h")):
        if abs(d) < 1e-12:
            continue
        s = 1 if d > 0 else -1
        k = p + s
        while True:
            t = (k - p) / d
            if t > t_max:
                break
            cands.append((t, kind, k))
            k += s
    cands.sort()
    seen_nodes = set()
    for t, kind, k in cands:
        if kind == "v":
            x, y = float(k), pj + t * dy
        else:
            x, y = pi + t * dx, float(k)
        xr, yr = round(x), round(y)
        if abs(x - xr) < eps and abs(y - yr) < eps:
            node = (int(xr), int(yr))
            if node in seen_nodes:
                continue
            seen_nodes.add(node)
            if fluid(*node):
                return True, mapped(*node), mapped(*node), 0.0
            continue
        if kind == "v":
            j0 = int(np.floor(y))
            a, b, w = (int(k), j0), (int(k), j0 + 1), y - j0
        else:
            i0 = int(np.floor(x))
            a, b, w = (i0, int(k)), (i0 + 1, int(k)), x - i0
        if fluid(*a) and fluid(*b):
            return True, mapped(*a), mapped(*b), w
    return False, None, None, 0.0
