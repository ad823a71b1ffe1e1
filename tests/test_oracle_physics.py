"""Pins of the whole FP64 oracle step against invariants, closed forms and physics.

Each test names the passage or law it checks.  Sizes are kept small so that the CPU suite runs
in a few minutes; the oracle uses all host threads (its per-node arithmetic does not depend on
the thread count).
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_2102_04709_amd import workloads as W


def _feq_all(rho, ux, uy):
    """Equilibria for arrays (from the lattice and Eq. 3, written out independently)."""
    ex, ey, w = po.lattice()
    eu = ex[:, None, None] * ux + ey[:, None, None] * uy
    uu = ux * ux + uy * uy
    return rho * w[:, None, None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)


def _velocity(o):
    ex, ey, _ = po.lattice()
    f = o.f().sum(0)
    rho = f.sum(0)
    return (f * ex[:, None, None]).sum(0) / np.where(rho > 0, rho, 1), (f * ey[:, None, None]).sum(0) / np.where(rho > 0, rho, 1), rho


# ---- conservation (Eq. 13 + Eq. 16 with halfway bounce-back) ------------------------------

def test_per_fluid_mass_conserved_flat_janus():
    o = po.Oracle(W.flat_janus())  # 120 x 60, walls, theta (60, 120) -> theta12 = 0
    m0 = o.mass()
    o.step(1000)
    m1 = o.mass()
    np.testing.assert_allclose(m1, m0, rtol=1e-12, atol=0)
    r = o.rho()
    assert np.all(np.isfinite(r))


def test_momentum_conserved_fully_periodic():
    """Sum over a periodic domain of div T vanishes (Eq. 12 telescopes), and recolouring keeps
    the total distribution, so total momentum changes by nothing."""
    w = W.random_mixture(40, 32, seed=3, walls=False)
    o = po.Oracle(w)
    ex, ey, _ = po.lattice()
    p0 = None
    for _ in range(5):
        o.step(20)
        f = o.f().sum(0)
        p = np.array([(f * ex[:, None, None]).sum(), (f * ey[:, None, None]).sum()])
        if p0 is None:
            p0 = p
        np.testing.assert_allclose(p, p0, atol=1e-13)
    o.prepare()
    F = o.crop(o.ext_force())
    assert abs(F[0].sum()) < 1e-15 and abs(F[1].sum()) < 1e-15
    assert np.abs(F).max() > 1e-6  # the force is not trivially zero


def test_swap_periodic_conservation():
    """Sec. III C modified periodic boundary: fluids 1 and 3 exchange labels across x; fluid 2
    mass, M1 + M3 and the total are conserved, M1 alone is not (flow carries it across)."""
    w = W.capillary_intrusion(nx=96, ny=14, slug=20, lg=20, ratio=1.0)
    o = po.Oracle(w)
    m0 = o.mass()
    o.step(400)
    m = o.mass()
    assert abs(m[1] - m0[1]) < 1e-12 * m0[1]
    assert abs((m[0] + m[2]) - (m0[0] + m0[2])) < 1e-12 * m0.sum()


# ---- single-fluid flows: collision, forcing and boundaries --------------------------------

def _channel(nx, ny, nu, g, circles=None):
    solid = np.zeros((ny, nx), np.uint8)
    if circles is None:
        solid[0] = solid[-1] = 1
    rho = np.zeros((3, ny, nx))
    rho[0][solid == 0] = 1.0
    wl = W.Workload("channel", nx, ny, 1 if circles is not None else 0, 0, (nu,) * 3, (0.01,) * 3,
                    (90.0, 90.0), solid, rho, body_force=(g, 0.0))
    return wl, solid


@pytest.mark.parametrize("nu", [0.1, 0.5])
def test_poiseuille_exact_with_halfway_walls(nu):
    """MRT with the Eq. (6) relaxation rates places halfway bounce-back walls exactly midway,
    so body-force Poiseuille flow is reproduced to round-off: u = g (y - y0)(y1 - y)/(2 nu)."""
    ny, g = 18, 1e-6
    wl, _ = _channel(4, ny, nu, g)
    o = po.Oracle(wl)
    steps = 6000 if nu == 0.1 else 1500
    o.step(steps)
    o.prepare()
    u = o.crop(o.ext_velocity())[0]
    y = np.arange(ny, dtype=float)
    y0, y1 = 0.5, ny - 1.5
    exact = g * (y - y0) * (y1 - y) / (2 * nu)
    fluid = slice(1, ny - 1)
    err = np.abs(u[fluid, 2] - exact[fluid]).max() / exact.max()
    assert err < 1e-9, err


def test_interpolated_bounce_back_places_walls_off_grid():
    """Bouzidi interpolated bounce-back with the exact wall position: walls at y = 0.7 and
    y = H - 0.2 (huge circles standing in for flat walls) give the Poiseuille profile between
    those positions, far closer than halfway bounce-back would."""
    nx, ny, nu, g = 4, 14, 0.1, 1e-6
    big = 1e6
    yb, yt = 0.7, ny - 1 - 0.2
    circles = np.array([[1.5, yb - big, big], [1.5, yt + big, big]])
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    solid = np.zeros((ny, nx), np.uint8)
    for cx, cy, r in circles:
        solid |= ((xx - cx) ** 2 + (yy - cy) ** 2 <= r * r).astype(np.uint8)
    assert solid[0].all() and solid[-1].all() and not solid[1:-1].any()
    rho = np.zeros((3, ny, nx))
    rho[0][solid == 0] = 1.0
    wl = W.Workload("ibb", nx, ny, 1, 0, (nu,) * 3, (0.01,) * 3, (90.0, 90.0), solid, rho,
                    circles=circles, body_force=(g, 0.0))
    o = po.Oracle(wl)
    assert abs(o.link_q(1, 1, 2) - 0.3) < 1e-6 and abs(o.link_q(1, ny - 2, 4) - 0.8) < 1e-6
    o.step(8000)
    o.prepare()
    u = o.crop(o.ext_velocity())[0][:, 2]
    y = np.arange(ny, dtype=float)
    exact = g * (y - yb) * (yt - y) / (2 * nu)
    fl = slice(1, ny - 1)
    err_ibb = np.abs(u[fl] - exact[fl]).max() / exact.max()
    half = g * (y - 0.5) * (ny - 1.5 - y) / (2 * nu)
    err_half = np.abs(half[fl] - exact[fl]).max() / exact.max()
    assert err_ibb < 0.01 and err_half > 0.05, (err_ibb, err_half)


def test_link_fractions_match_geometry():
    """q = fraction of the link from the fluid node to the circle, computed here by bisection."""
    w = W.cylinder_janus(nx=80, ny=80, Rs=17.3, Rj=8, centre=(40.2, 38.7))
    o = po.Oracle(w)
    ex, ey, _ = po.lattice()
    cx, cy, R = 40.2, 38.7, 17.3
    count = 0
    for j in range(2, 78):
        for i in range(80):
            if w.solid[j, i]:
                continue
            for a in range(1, 9):
                si, sj = (i - ex[a]) % 80, j - ey[a]
                if not w.solid[sj, si] or not (2 <= sj < 78):
                    continue
                lo, hi = 0.0, 1.0  # inside(hi) is True, inside(lo) False
                for _ in range(80):
                    mid = 0.5 * (lo + hi)
                    px, py = i - mid * ex[a], j - mid * ey[a]
                    if (px - cx) ** 2 + (py - cy) ** 2 <= R * R:
                        hi = mid
                    else:
                        lo = mid
                assert abs(o.link_q(i, j, a) - hi) < 1e-12
                count += 1
    assert count > 100


def test_shear_wave_decay_gives_mixture_viscosity():
    """Eq. (7): a uniform three-fluid mixture has the harmonic-mean viscosity; a shear wave
    u_x = U sin(k y) decays as exp(-nu k^2 t)."""
    n = 48
    C = np.array([0.2, 0.3, 0.5])
    nu = (0.05, 0.1, 0.3)
    numix = 1.0 / (C / np.array(nu)).sum()
    rho = np.ones((3, n, 4)) * C[:, None, None]
    wl = W.Workload("shear", 4, n, 1, 0, nu, (0.01,) * 3, (90.0, 90.0), np.zeros((n, 4), np.uint8), rho)
    o = po.Oracle(wl)
    y = np.arange(n, dtype=float)[:, None] * np.ones((1, 4))
    k = 2 * np.pi / n
    ux = 1e-4 * np.sin(k * y)
    feq = _feq_all(np.ones_like(ux), ux, np.zeros_like(ux))
    o.set_f(C[:, None, None, None] * feq[None])
    o.step(100)
    a0 = (_velocity(o)[0][:, 0] * np.sin(k * y[:, 0])).sum()
    o.step(400)
    a1 = (_velocity(o)[0][:, 0] * np.sin(k * y[:, 0])).sum()
    nu_meas = -math.log(a1 / a0) / (400 * k * k)
    assert abs(nu_meas / numix - 1) < 5e-3, (nu_meas, numix)


def test_zou_he_uniform_flow_is_a_fixed_point():
    """Sec. III D inlet/outlet: uniform flow (u_in, 0) at rho = 1 of pure fluid 3 satisfies the
    velocity inlet and the pressure outlet, so one step must reproduce it."""
    nx, ny, u = 24, 8, 0.01
    rho = np.zeros((3, ny, nx))
    rho[2] = 1.0
    wl = W.Workload("zh", nx, ny, 1, W.BC_ZOUHE, (0.1,) * 3, (0.01,) * 3, (90.0, 90.0),
                    np.zeros((ny, nx), np.uint8), rho, u_in=u, rho_out=1.0)
    o = po.Oracle(wl)
    feq = _feq_all(np.ones((ny, nx)), np.full((ny, nx), u), np.zeros((ny, nx)))
    f0 = np.zeros((3, 9, ny, nx))
    f0[2] = feq
    o.set_f(f0)
    o.step(50)
    f = o.f()
    np.testing.assert_allclose(f, f0, atol=1e-15)


# ---- interfacial force and wetting --------------------------------------------------------

def test_laplace_law_static_disk():
    """Eq. (10) normalisation: a disk of fluid 1 in fluid 3 holds a pressure jump
    dp = c_s^2 (rho_in - rho_out) = sigma / R (within 5 %)."""
    sigma = 0.01
    for R in (10.0, 14.0):
        n = 56
        o = po.Oracle(W.static_disk(n=n, R=R, sigma13=sigma, nu=0.5))
        o.step(2000)
        r = o.rho().sum(0)
        yy, xx = np.mgrid[0:n, 0:n]
        d = np.hypot(xx - (n - 1) / 2, yy - (n - 1) / 2)
        dp = (r[d < R - 5].mean() - r[d > R + 6].mean()) / 3.0
        assert abs(dp / (sigma / R) - 1) < 0.05, (R, dp, sigma / R)


def _interface_bend(theta, steps=1000):
    nx, ny = 40, 24
    solid = W._walls(nx, ny)
    rho = np.zeros((3, ny, nx))
    x = np.arange(nx)
    rho[0][:, (x >= 5) & (x < 15)] = 1
    rho[1][:, (x >= 15) & (x < 25)] = 1
    rho[2][:, (x < 5) | (x >= 25)] = 1
    rho[:, solid.astype(bool)] = 0
    wl = W.Workload("flat", nx, ny, 0, 0, (0.1, 0.2, 0.05), (0.01, 0.012, 0.015), theta, solid, rho)
    o = po.Oracle(wl)
    o.step(steps)
    o.prepare()
    u = o.crop(o.ext_velocity())
    r = o.rho()
    C1 = r[0] / np.maximum(r.sum(0), 1e-12)
    pos = []
    for j in range(1, ny - 1):  # C1 = 0.5 crossing of the 1|2 interface in every fluid row
        row = C1[j]
        for i in range(12, 20):
            if (row[i] - 0.5) * (row[i + 1] - 0.5) < 0:
                pos.append(i + (0.5 - row[i]) / (row[i + 1] - row[i]))
    pos = np.array(pos)
    assert len(pos) == ny - 2
    return np.abs(u).max(), pos.max() - pos.min(), o


def test_flat_interfaces_at_90_degrees_relax_straight_and_at_rest():
    """Vertical interfaces meeting flat walls with all wall angles 90 degrees (theta12 from
    Eq. 18 is then 90 too): the wetting fill keeps the contact lines perpendicular, so the
    interfaces stay straight and the flow dies out.  A 60 degree control bends the 1|2 interface
    by several lattice units, so the test is sensitive to the fill."""
    umax, bend, o = _interface_bend((90.0, 90.0))
    assert abs(math.degrees(o.theta12()) - 90) < 1e-9
    assert umax < 1e-6 and bend < 1e-3, (umax, bend)
    umax, bend, _ = _interface_bend((60.0, 90.0), steps=600)
    assert bend > 1.0, bend


def _fill_case(C1, C2, theta):
    nx, ny = len(C1), 12
    solid = W._walls(nx, ny)
    rho = np.zeros((3, ny, nx))
    rho[0] = C1[None, :]
    rho[1] = C2[None, :]
    rho[2] = 1 - rho[0] - rho[1]
    rho[:, solid.astype(bool)] = 0
    o = po.Oracle(W.Workload("fill", nx, ny, 0, 0, (0.1,) * 3, (0.01,) * 3, theta, solid, rho))
    o.prepare()
    return o, o.ext_C()


@pytest.mark.parametrize("theta13", [60.0, 120.0, 35.0])
def test_fill_closed_form_flat_wall(theta13):
    """Eq. (21)-(22) on a flat wall: the characteristic lines from P = (i, 0) leave at
    +-phi = |90 - theta| from the normal (0, 1) and first meet fluid on row 1 at
    x = i +- tan(phi) (and at x = i +- 2 tan(phi) from the second solid layer), where C is
    interpolated linearly; Eq. (22) takes the larger value when theta <= 90."""
    x = np.arange(40, dtype=float)
    b = 0.015
    C1 = 0.2 + b * (x - 20)
    C2 = np.zeros(40)
    o, Cext = _fill_case(C1, C2, (theta13, 90.0))
    PY = o.PY
    phi = math.radians(abs(90 - theta13))
    for i in range(8, 32):
        for depth, row in ((1, 0), (2, -1)):
            expect = C1[i] + (1 if theta13 <= 90 else -1) * depth * abs(b) * math.tan(phi)
            got = Cext[0, row + PY, i]
            assert abs(got - expect) < 1e-13, (i, row, got, expect)
            assert abs(Cext[1, row + PY, i]) < 1e-15
            assert abs(Cext[2, row + PY, i] - (1 - got)) < 1e-15
        # the top wall is the mirror image
        top = o.ny - 1
        expect = C1[i] + (1 if theta13 <= 90 else -1) * abs(b) * math.tan(phi)
        assert abs(Cext[0, top + PY, i] - expect) < 1e-13


@pytest.mark.parametrize("theta13, clamped", [(2.0, 5.0), (178.0, 175.0), (5.0, 5.0)])
def test_fill_line_angle_clamped(theta13, clamped):
    """The line-angle clamp (reading: theta_k within [5, 175] degrees for the line construction):
    at 2 degrees the lines leave at |90 - 5| = 85 degrees from the normal, so they meet row 1 at
    x = i +- tan(85) and row 1 from the second layer at i +- 2 tan(85) (line lengths 11.5 and 22.9,
    inside t = 24); unclamped, 88 degrees would put the second-layer crossing beyond t = 24."""
    nx = 200
    x = np.arange(nx, dtype=float)
    b = 0.002
    C1 = 0.3 + b * (x - nx / 2)
    C2 = np.zeros(nx)
    o, Cext = _fill_case(C1, C2, (theta13, 90.0))
    PY = o.PY
    t = math.tan(math.radians(abs(90 - clamped)))
    for i in range(60, 140):
        for depth, row in ((1, 0), (2, -1)):
            expect = C1[i] + (1 if clamped <= 90 else -1) * depth * b * t
            got = Cext[0, row + PY, i]
            assert abs(got - expect) < 1e-12, (theta13, i, row, got, expect)


def test_fill_weighted_angle_from_C_at_D0():
    """Eq. (21) with all three fluids at a flat wall: theta_1 = (C3 theta13 + C2 theta12) /
    (C2 + C3) and theta_2 = (C3 theta23 + C1 theta21) / (C1 + C3), theta21 = 180 - theta12, with
    the C's taken at D0 (reading: the first crossing of the normal line, here the node above P);
    each fluid's lines then meet row 1 at x = i +- tan|90 - theta_k| and Eq. (22) keeps the larger
    value for theta_k <= 90, the smaller above."""
    nx = 120
    x = np.arange(nx, dtype=float)
    C1 = 0.25 + 0.002 * (x - nx / 2)
    C2 = 0.35 - 0.0015 * (x - nx / 2)
    theta = (60.0, 100.0)
    o, Cext = _fill_case(C1, C2, theta)
    PY = o.PY
    t12 = math.degrees(o.theta12())
    C3 = 1 - C1 - C2
    for i in range(30, 90):
        for k, (Ck, th_a, th_b, wa, wb) in enumerate(((C1, theta[0], t12, C2[i], C3[i]),
                                                      (C2, theta[1], 180 - t12, C1[i], C3[i]))):
            th = (wb * th_a + wa * th_b) / (wa + wb)
            phi = math.radians(abs(90 - th))
            vals = []
            for sgn in (1, -1):
                xc = i + sgn * math.tan(phi)
                i0 = int(math.floor(xc))
                vals.append(Ck[i0] + (xc - i0) * (Ck[i0 + 1] - Ck[i0]))
            expect = max(vals) if th <= 90 else min(vals)
            got = Cext[k, PY, i]
            assert abs(got - expect) < 1e-12, (k, i, got, expect)


def test_fill_uses_pair_angle_between_fluids_1_and_2():
    """With fluid 3 absent, Eq. (21) reduces to theta_1 = theta12 and theta_2 = 180 - theta12."""
    x = np.arange(40, dtype=float)
    C1 = 0.5 + 0.01 * (x - 20)
    C2 = 1 - C1
    theta = (60.0, 90.0)  # equal tensions: theta12 = 60 (Table I, case d)
    o, Cext = _fill_case(C1, C2, theta)
    phi = math.radians(30.0)
    for i in range(8, 32):
        e1 = C1[i] + 0.01 * math.tan(phi)    # theta_1 = 60 <= 90: max
        e2 = C2[i] + 0.01 * math.tan(phi) * -1 * -1  # theta_2 = 120 > 90: min of C2 = 1 - C1
        e2 = min(C2[i] + 0.01 * math.tan(phi), C2[i] - 0.01 * math.tan(phi))
        assert abs(Cext[0, o.PY, i] - e1) < 1e-13
        assert abs(Cext[1, o.PY, i] - e2) < 1e-13


def _contact_angle(C, yw, side_rows=3):
    """Circle fit to the C = 0.5 contour of a drop on the wall y = yw; angle inside the drop."""
    ny, nx = C.shape
    pts = []
    for j in range(int(yw) + side_rows, ny - 1):
        row = C[j]
        for i in range(nx - 1):
            a, b = row[i], row[i + 1]
            if (a - 0.5) * (b - 0.5) < 0:
                pts.append((i + (0.5 - a) / (b - a), j))
    pts = np.array(pts)
    A = np.c_[2 * pts[:, 0], 2 * pts[:, 1], np.ones(len(pts))]
    rhs = (pts ** 2).sum(1)
    (xc, yc, c0), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    r = math.sqrt(c0 + xc * xc + yc * yc)
    return math.degrees(math.acos((yw - yc) / r))


@pytest.mark.parametrize("theta13", [60.0, 120.0])
def test_static_contact_angle_single_drop(theta13):
    """Sec. II B wetting condition, physics: a drop of fluid 1 in fluid 3 on a flat wall relaxes
    to the prescribed angle (within 4 degrees at this small radius)."""
    nx, ny, R = 100, 46, 14.0
    x, y = np.mgrid[0:ny, 0:nx][::-1]
    solid = W._walls(nx, ny)
    d = (x - nx / 2) ** 2 + (y - 0.5) ** 2 < R * R
    rho = np.zeros((3, ny, nx))
    rho[0][d] = 1
    rho[2][~d] = 1
    rho[:, solid.astype(bool)] = 0
    o = po.Oracle(W.Workload("drop", nx, ny, 0, 0, (0.1,) * 3, (0.01,) * 3, (theta13, 90.0), solid, rho))
    o.step(4000)
    C1 = o.rho()[0] / np.maximum(o.rho().sum(0), 1e-12)
    ang = _contact_angle(C1[: ny // 2 + 10], 0.5)
    assert abs(ang - theta13) < 4.0, ang


def _arc_points(C, k, l):
    ny, nx = C.shape[1:]
    pts = []
    D = C[k] - C[l]
    for j in range(ny):
        for i in range(nx - 1):
            if D[j, i] * D[j, i + 1] < 0 and C[k, j, i] + C[l, j, i] > 0.8:
                pts.append((i + D[j, i] / (D[j, i] - D[j, i + 1]), j))
    for j in range(ny - 1):
        for i in range(nx):
            if D[j, i] * D[j + 1, i] < 0 and C[k, j, i] + C[l, j, i] > 0.8:
                pts.append((i, j + D[j, i] / (D[j, i] - D[j + 1, i])))
    return np.array(pts)


def _circle(p):
    A = np.c_[2 * p[:, 0], 2 * p[:, 1], np.ones(len(p))]
    (xc, yc, c0), *_ = np.linalg.lstsq(A, (p ** 2).sum(1), rcond=None)
    return np.array([xc, yc]), math.sqrt(c0 + xc * xc + yc * yc)


@pytest.mark.parametrize("sig", [(0.01, 0.01, 0.01), (0.008, 0.01, 0.012)])
def test_neumann_lens_angle(sig):
    """Eq. (10) + Eq. (13)-(15) with a full range of tensions: a lens of fluid 1 at a flat 2|3
    interface meets it at a triple junction whose angle inside fluid 1 obeys the Neumann force
    balance sigma23^2 = sigma12^2 + sigma13^2 + 2 sigma12 sigma13 cos(theta_1) (120 degrees for
    equal tensions), within 3 degrees."""
    nx, ny, R = 120, 80, 16.0
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    rho = np.zeros((3, ny, nx))
    d = (x - nx / 2) ** 2 + (y - ny / 2) ** 2 < R * R
    rho[0][d] = 1
    rho[1][~d & (y < ny / 2)] = 1
    rho[2][~d & (y >= ny / 2)] = 1
    wl = W.Workload("lens", nx, ny, 1, 0, (1 / 6,) * 3, sig, (90.0, 90.0),
                    np.zeros((ny, nx), np.uint8), rho)
    o = po.Oracle(wl)
    o.step(4000)
    r = o.rho()
    C = r / r.sum(0)
    (c12, r12), (c13, r13) = _circle(_arc_points(C, 0, 1)), _circle(_arc_points(C, 0, 2))
    dd = np.linalg.norm(c13 - c12)
    a = (r12 ** 2 - r13 ** 2 + dd ** 2) / (2 * dd)
    h = math.sqrt(max(r12 ** 2 - a * a, 0.0))
    mid = c12 + a * (c13 - c12) / dd
    perp = np.array([c13[1] - c12[1], -(c13[0] - c12[0])]) / dd
    P = mid + h * perp
    if P[0] > nx / 2:
        P = mid - h * perp

    def tangent_towards(c, target):
        v = P - c
        t = np.array([-v[1], v[0]]) / np.linalg.norm(v)
        return t if t @ (target - P) > 0 else -t

    t12 = tangent_towards(c12, np.array([nx / 2, P[1] - 10]))
    t13 = tangent_towards(c13, np.array([nx / 2, P[1] + 10]))
    theta1 = math.degrees(math.acos(float(t12 @ t13)))
    s12, s13, s23 = sig
    expect = math.degrees(math.acos((s23 ** 2 - s12 ** 2 - s13 ** 2) / (2 * s12 * s13)))
    assert abs(theta1 - expect) < 3.0, (theta1, expect)
