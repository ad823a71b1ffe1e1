"""Pins of the FP64 oracle's building blocks against closed forms and invariants.

Each test names the passage it pins.  None of them re-types the oracle's formula: they check
properties that a dropped term, a wrong sign or a transposed index would break.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import pyoracle as po
from march_ref import brute_force_march as _brute_force_march
from paper_2102_04709_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lat():
    ex, ey, w = po.lattice()
    return ex.astype(float), ey.astype(float), w


# ---- D2Q9 lattice and the transformation matrix, Sec. II A, Eq. (4) ------------------------

def test_lattice_isotropy():
    ex, ey, w = _lat()
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(9):  # every velocity has its opposite
        assert any(ex[b] == -ex[a] and ey[b] == -ey[a] for b in range(9))
    assert abs((w * ex * ex).sum() - 1 / 3) < 1e-15
    assert abs((w * ey * ey).sum() - 1 / 3) < 1e-15
    assert abs((w * ex * ey).sum()) < 1e-16
    # fourth-order isotropy: sum w e_x^4 = 3 sum w e_x^2 e_y^2 = 1/3
    assert abs((w * ex ** 4).sum() - 1 / 3) < 1e-15
    assert abs((w * ex ** 2 * ey ** 2).sum() - 1 / 9) < 1e-15


def test_matrix_rows_are_the_moment_basis():
    """Each row of M is the Lallemand-Luo moment polynomial evaluated on the lattice vectors."""
    ex, ey, _ = _lat()
    M, _ = po.matrices()
    e2 = ex * ex + ey * ey
    rows = [np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 * e2, ex, (-5 + 3 * e2) * ex,
            ey, (-5 + 3 * e2) * ey, ex * ex - ey * ey, ex * ey]
    for i, r in enumerate(rows):
        np.testing.assert_array_equal(M[i], r, err_msg=f"row {i}")


def test_matrix_orthogonal_and_inverse():
    M, Mi = po.matrices()
    G = M @ M.T
    np.testing.assert_array_equal(G, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]).astype(float))
    np.testing.assert_allclose(Mi @ M, np.eye(9), atol=2e-15)
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=2e-15)


# ---- equilibrium, forcing, relaxation rates: Eq. (3), (5), (6), (8), (9) -------------------

@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.02, -0.05), (0.97, -0.1, 0.07)])
def test_equilibrium_moments(rho, ux, uy):
    ex, ey, _ = _lat()
    M, _ = po.matrices()
    feq = po.equilibrium(rho, ux, uy)
    uu = ux * ux + uy * uy
    expect = [rho, -2 * rho + 3 * rho * uu, rho - 3 * rho * uu, rho * ux, -rho * ux, rho * uy,
              -rho * uy, rho * (ux * ux - uy * uy), rho * ux * uy]
    np.testing.assert_allclose(M @ feq, expect, atol=1e-15)
    # hydrodynamic moments: density, momentum, momentum flux rho (c_s^2 I + u u)
    assert abs(feq.sum() - rho) < 1e-15
    assert abs((feq * ex).sum() - rho * ux) < 1e-15
    assert abs((feq * ex * ey).sum() - rho * ux * uy) < 1e-15
    assert abs((feq * ex * ex).sum() - rho * (1 / 3 + ux * ux)) < 1e-15


@pytest.mark.parametrize("ux,uy,fx,fy", [(0.0, 0.0, 1e-3, 0.0), (0.03, -0.02, 2e-4, -5e-4)])
def test_forcing_moments(ux, uy, fx, fy):
    ex, ey, _ = _lat()
    M, _ = po.matrices()
    ft = po.force_populations(ux, uy, fx, fy)
    uf = ux * fx + uy * fy
    expect = [0, 6 * uf, -6 * uf, fx, -fx, fy, -fy, 2 * (ux * fx - uy * fy), ux * fy + uy * fx]
    np.testing.assert_allclose(M @ ft, expect, atol=1e-18)
    assert abs(ft.sum()) < 1e-18
    assert abs((ft * ex).sum() - fx) < 1e-18
    assert abs((ft * ex * ex).sum() - 2 * ux * fx) < 1e-18
    assert abs((ft * ex * ey).sum() - (ux * fy + uy * fx)) < 1e-18


@pytest.mark.parametrize("tau", [0.5105, 0.8, 1.0, 3.5])
def test_magic_parameter(tau):
    """Eq. (6): s4 = 8(2 - s1)/(8 - s1) is the choice with (1/s1 - 1/2)(1/s4 - 1/2) = 3/16."""
    s = po.relaxation_rates(tau)
    assert s[0] == s[3] == s[5] == 0.0
    assert s[1] == s[2] == s[7] == s[8] == 1.0 / tau
    assert s[4] == s[6]
    assert abs((1 / s[1] - 0.5) * (1 / s[4] - 0.5) - 3 / 16) < 1e-14


def test_mixture_relaxation_time():
    """Eq. (7): mu = (tau - 1/2) rho c_s^2 equals the harmonic mean rho / sum(rho_k / mu_k)."""
    rk = np.array([0.2, 0.3, 0.5]) * 1.02
    nu = np.array([0.05, 0.1, 0.3])
    tau = po.relaxation_time(rk, nu)
    rho = rk.sum()
    mu = (tau - 0.5) * rho / 3.0
    assert abs(rho / mu - (rk / nu).sum()) < 1e-12
    # pure fluid: tau = 1/2 + 3 nu
    assert abs(po.relaxation_time(np.array([1.0, 0, 0]), nu) - (0.5 + 3 * 0.05)) < 1e-15


def test_collision_moments():
    """Eq. (1)-(2), (8), (11): conserved moments and the relaxation of each non-conserved one,
    computed from lattice polynomials (not from M)."""
    rng = np.random.default_rng(1)
    ex, ey, w = _lat()
    e2 = ex * ex + ey * ey
    nu = np.array([0.1, 0.04, 0.2])
    rk = np.array([0.5, 0.3, 0.21])
    rho = rk.sum()
    f = po.equilibrium(rho, 0.03, -0.01) + 1e-3 * rng.standard_normal(9)
    f *= rho / f.sum()
    fx, fy = 3e-4, -2e-4
    fd, u = po.collide(f, rk, nu, fx, fy)
    jx, jy = (f * ex).sum(), (f * ey).sum()
    assert abs(u[0] - (jx + fx / 2) / rho) < 1e-16 and abs(u[1] - (jy + fy / 2) / rho) < 1e-16
    assert abs(fd.sum() - f.sum()) < 1e-15
    assert abs((fd * ex).sum() - (jx + fx)) < 1e-15
    assert abs((fd * ey).sum() - (jy + fy)) < 1e-15
    tau = 0.5 + 3.0 / (rk / nu).sum()
    s1 = 1 / tau
    s4 = 8 * (2 - s1) / (8 - s1)
    ux, uy = u
    uu = ux * ux + uy * uy
    uf = ux * fx + uy * fy
    checks = [  # (moment polynomial, equilibrium, forcing moment, rate)
        (-4 + 3 * e2, -2 * rho + 3 * rho * uu, 6 * uf, s1),
        (4 - 10.5 * e2 + 4.5 * e2 * e2, rho - 3 * rho * uu, -6 * uf, s1),
        ((-5 + 3 * e2) * ex, -rho * ux, -fx, s4),
        ((-5 + 3 * e2) * ey, -rho * uy, -fy, s4),
        (ex * ex - ey * ey, rho * (ux * ux - uy * uy), 2 * (ux * fx - uy * fy), s1),
        (ex * ey, rho * ux * uy, ux * fy + uy * fx, s1),
    ]
    for poly, meq, mf, s in checks:
        m = (poly * f).sum()
        expect = m - s * (m - meq) + (1 - s / 2) * mf
        assert abs((poly * fd).sum() - expect) < 1e-15


# ---- segregation parameter, Eq. (14)-(15) -------------------------------------------------

def test_g_is_continuous_and_bounded():
    for X in (-1.0, 0.0, 1.0):
        for d in (1e-9, 1e-12):
            assert abs(po.g_of_X(X - d) - po.g_of_X(X + d)) < 1e-4
    assert po.g_of_X(-5) == 1.0 and po.g_of_X(5) == -1.0
    assert abs(po.g_of_X(0.5) - (math.sqrt(3) / 2 - 1)) < 1e-15
    xs = np.linspace(-2, 2, 401)
    gs = np.array([po.g_of_X(x) for x in xs])
    assert np.all(np.diff(gs) <= 1e-15)  # non-increasing


def test_X_is_cosine_of_the_neumann_triangle_angle():
    """X_kl = (s_mk^2 + s_ml^2 - s_kl^2) / (2 s_mk s_ml) is, by the law of cosines, the cosine
    of the triangle angle between sides s_mk and s_ml (opposite side s_kl)."""
    ang = np.radians([50.0, 60.0, 70.0])  # angles opposite sides a, b, c
    a, b, c = np.sin(ang)  # law of sines
    # sides: sigma12 = a, sigma13 = b, sigma23 = c  -> X12 opposite a, X13 opposite b, X23 opposite c
    X = po.segregation_X([a, b, c])
    np.testing.assert_allclose(X, np.cos(ang), atol=1e-14)
    np.testing.assert_allclose(po.segregation_X([0.01, 0.01, 0.01]), [0.5] * 3, atol=1e-15)


# ---- recolouring, Eq. (13) ----------------------------------------------------------------

def _rand_normals(rng):
    n = np.zeros((3, 3, 2))
    for k in range(3):
        for l in range(k + 1, 3):
            t = rng.uniform(0, 2 * np.pi)
            n[k, l] = [np.cos(t), np.sin(t)]
            n[l, k] = -n[k, l]
    return n


def test_recolour_partition_and_flux():
    rng = np.random.default_rng(7)
    ex, ey, w = _lat()
    for _ in range(5):
        fdag = po.equilibrium(1.0, 0.02, 0.01) + 1e-3 * rng.standard_normal(9)
        rk = rng.uniform(0.05, 0.6, 3)
        rho = rk.sum()
        n = _rand_normals(rng)
        gX = np.array([po.g_of_X(x) for x in rng.uniform(-1, 1, 3)])
        out = po.recolour(fdag, rk, n, gX, 0.7)
        np.testing.assert_allclose(out.sum(0), fdag, rtol=0, atol=1e-15)
        np.testing.assert_allclose(out.sum(1), rk / rho * fdag.sum(), rtol=0, atol=1e-15)
        # segregation flux: sum_a f''_k e_a = C_k j + sum_l beta_kl (rho_k rho_l / rho) n_kl / 3
        r3 = min(max(35 * rk.prod() / rho ** 3, 0.0), 1.0)
        pair = {(0, 1): 0, (0, 2): 1, (1, 2): 2}
        for k in range(3):
            jx = (out[k] * ex).sum()
            jy = (out[k] * ey).sum()
            ex_ = rk[k] / rho * (fdag * ex).sum()
            ey_ = rk[k] / rho * (fdag * ey).sum()
            for l in range(3):
                if l == k:
                    continue
                beta = 0.7 * (1 + r3 * gX[pair[tuple(sorted((k, l)))]])
                ex_ += beta * rk[k] * rk[l] / rho * n[k, l, 0] / 3
                ey_ += beta * rk[k] * rk[l] / rho * n[k, l, 1] / 3
            assert abs(jx - ex_) < 1e-15 and abs(jy - ey_) < 1e-15


# ---- Eq. (12) gradient, Eq. (19)-(20) normal stencil ---------------------------------------

def test_gradient_exact_on_quadratics():
    w = W.static_disk(n=24, R=5)
    o = po.Oracle(w)
    y, x = np.mgrid[0:o.NYE, 0:o.NXE].astype(float)
    a, b, c, d, e, f = 0.3, -0.2, 0.15, 0.01, -0.02, 0.005
    psi = a + b * x + c * y + d * x * x + e * x * y + f * y * y
    g = o.gradient(psi)
    inner = (slice(1, o.NYE - 1), slice(1, o.NXE - 1))
    np.testing.assert_allclose(g[0][inner], (b + 2 * d * x + e * y)[inner], atol=1e-13)
    np.testing.assert_allclose(g[1][inner], (c + e * x + 2 * f * y)[inner], atol=1e-13)
    # a cubic is not reproduced (the stencil is exact to second order only)
    g3 = o.gradient(x ** 3)
    assert np.abs(g3[0][inner] - (3 * x * x)[inner]).max() > 0.5


def test_normal_stencil_isotropy():
    """Eq. (20) weights: sum w c c = I (linear fields exact) and isotropy of the fourth and sixth
    moments (sum w c_x^4 = 3 sum w c_x^2 c_y^2, sum w c_x^6 = 5 sum w c_x^4 c_y^2)."""
    cy, cx = np.mgrid[-2:3, -2:3]
    s = po.isotropic_sum
    assert tuple(s(np.ones((5, 5)))) == (0, 0)
    assert tuple(s(3 * cx - 5 * cy)) == (3 * 5040, -5 * 5040)
    assert tuple(s(cx * cx + cy * cy)) == (0, 0)
    x4 = s(cx ** 3)[0]
    x2y2 = s(cx * cy * cy)[0]
    assert x4 == 3 * x2y2 and x4 * 7 == 12 * 5040
    x6 = s(cx ** 5)[0]
    x4y2 = s(cx ** 3 * cy * cy)[0]
    assert x6 == 5 * x4y2 and x6 * 7 == 32 * 5040


def test_normals_flat_diagonal_and_circle():
    # flat walls: exactly (0, +-1) pointing into the fluid
    o = po.Oracle(W.flat_janus(nx=40, ny=20, R=6))
    idx, nrm = o.fill_nodes()
    for (i, j, t, _), n in zip(idx, nrm):
        assert n[0] == 0.0 and abs(abs(n[1]) - 1.0) == 0.0
        assert (n[1] > 0) == (j < 10)
    # diamond |x - c| + |y - c| <= r: faces away from corners have normals (+-1, +-1)/sqrt(2)
    nx = 64
    y, x = np.mgrid[0:nx, 0:nx]
    solid = (np.abs(x - 32) + np.abs(y - 32) <= 14).astype(np.uint8)
    rho = np.zeros((3, nx, nx))
    rho[2][solid == 0] = 1.0
    wl = W.Workload("diamond", nx, nx, 1, 0, (0.1,) * 3, (0.01,) * 3, (90.0, 90.0), solid, rho)
    o = po.Oracle(wl)
    idx, nrm = o.fill_nodes()
    for (i, j, t, _), n in zip(idx, nrm):
        if min(abs(i - 32), abs(j - 32)) >= 4 and t == 1:
            sx, sy = np.sign(i - 32), np.sign(j - 32)
            assert abs(n[0] - sx / math.sqrt(2)) < 1e-15 and abs(n[1] - sy / math.sqrt(2)) < 1e-15
    # circle: Eq. (19) on a binary staircase is a noisy estimate of the radial direction.  Pin
    # what is exact -- the mirror symmetry of a circle centred on a half-integer axis -- and that
    # the deviation has no bias and a small mean.
    for R in (8.0, 24.0, 60.0):
        wc = W.cylinder_janus(nx=200, ny=200, Rs=R, Rj=10, centre=(99.5, 90.3))
        o = po.Oracle(wc)
        idx, nrm = o.fill_nodes()
        by_node = {(int(i), int(j)): n for (i, j, t, _), n in zip(idx, nrm)}
        devs = []
        for (i, j, t, _), n in zip(idx, nrm):
            if j <= 1 or j >= 198:
                continue
            m = by_node[(199 - int(i), int(j))]
            assert m[0] == -n[0] and m[1] == n[1]
            if t == 1:
                r = np.array([i - 99.5, j - 90.3])
                r /= np.linalg.norm(r)
                devs.append(math.degrees(math.atan2(r[0] * n[1] - r[1] * n[0], float(r @ n))))
        devs = np.array(devs)
        assert abs(devs.mean()) < 1e-9 and np.abs(devs).mean() < 10.0, (R, np.abs(devs).mean())


# ---- Young relations, Eq. (17)-(18), against Table I -------------------------------------

def test_theta12_reproduces_table1_angle_sets():
    cases = json.load(open(os.path.join(GOLDEN, "table1_contact_angles.json")))["cases"]
    for case in cases:
        rg, br, gb = case["analytical"]
        # fluids r, g, b -> 1, 2, 3: theta13 = theta_rb = 180 - theta_br, theta23 = theta_gb
        w = W.flat_janus(nx=30, ny=12, R=4, theta=(180.0 - br, gb))
        o = po.Oracle(w)
        assert abs(math.degrees(o.theta12()) - rg) < 1e-6, case


def test_inconsistent_angles_rejected():
    w = W.flat_janus(nx=30, ny=12, R=4, theta=(40.0, 110.0), sigma=(0.01, 0.01, 0.01))
    with pytest.raises(ValueError, match="Eq. \\(18\\)"):
        po.Oracle(w)


@pytest.mark.parametrize("seed, walls", [(3, True), (4, False), (5, True)])
def test_march_matches_brute_force_crossings(seed, walls):
    """The oracle's characteristic-line march (Eq. 22's crossing D) against the brute-force
    enumeration of all grid-line crossings, from every fill node, along random directions and
    along lattice directions that pass exactly through nodes."""
    w = W.random_mixture(48, 36, seed, walls=walls, circles=[(17.3, 16.6, 6.1), (34.2, 20.7, 4.4)])
    o = po.Oracle(w)
    idx, _ = o.fill_nodes()
    rng = np.random.Generator(np.random.PCG64(seed))
    lattice = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (1, -1), (-1, -1), (2, 1), (1, -2), (-3, 1)]
    checked = hits = 0
    for n, (i, j) in enumerate(idx[:, :2]):
        dirs = [(np.cos(a), np.sin(a)) for a in rng.uniform(0, 2 * np.pi, 6)]
        dirs += [(a / np.hypot(a, b), b / np.hypot(a, b)) for a, b in lattice[n % 3::3]]
        for dx, dy in dirs:
            ok, n0, n1, wt = o.march(int(i), int(j), float(dx), float(dy))
            bok, b0, b1, bw = _brute_force_march(w.solid, w.y_periodic, int(i), int(j), dx, dy)
            assert ok == bok, (i, j, dx, dy)
            if ok:
                hits += 1
                assert (n0, n1) == (b0, b1), (i, j, dx, dy, n0, n1, b0, b1)
                assert abs(wt - bw) <= 1e-12, (wt, bw)
            checked += 1
    assert checked > 500 and hits > checked // 4  # (directions into the solid may find no fluid)
