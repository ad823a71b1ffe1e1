"""Pins of the oracle's boundary rules that the closed-form pins do not reach: the Zou-He columns
of Sec. III D under non-uniform flow, their composition readings, and the fallbacks of the
characteristic-line fill (Sec. II B) when a line finds no fluid within its reach.

Zou-He: whatever the flow, the unknown populations of the inlet column make its velocity
(sum_a f_a e_a) / rho equal to (u_in, 0), and those of the outlet column make its density equal
to rho_out with no transverse momentum; these are the conditions the rule is solved from, so a
wrong sign of the transverse correction or a wrong outlet velocity breaks them as soon as
f_2 != f_4 at the column.
"""
import math

import numpy as np
import pytest

from march_ref import brute_force_march
from oracle import pyoracle as po
from paper_2102_04709_amd import workloads as W


def _feq(rho, ux, uy):
    ex, ey, w = po.lattice()
    eu = ex[:, None, None] * ux + ey[:, None, None] * uy
    uu = ux * ux + uy * uy
    return rho * w[:, None, None] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu)


def _zou_he_channel(C, u_in=0.01, rho_out=1.02, pillar=True, seed=0):
    """Channel, periodic in y, Zou-He inlet/outlet, a pillar close to the inlet (which makes the flow
    through the inlet column non-uniform), uniform composition C and a random initial flow."""
    nx, ny = 64, 28
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    circles = [(9.6, 13.3, 5.2)] if pillar else []
    solid = np.zeros((ny, nx), np.uint8)
    for cx, cy, r in circles:
        solid |= ((x - cx) ** 2 + (y - cy) ** 2 <= r * r).astype(np.uint8)
    rho = np.asarray(C, float)[:, None, None] * (solid == 0)
    w = W.Workload("zh", nx, ny, 1, W.BC_ZOUHE, (0.1, 0.07, 0.13), (0.01, 0.012, 0.011), (90.0, 90.0),
                   solid, rho, circles=np.array(circles).reshape(-1, 3), u_in=u_in, rho_out=rho_out)
    o = po.Oracle(w)
    rng = np.random.Generator(np.random.PCG64(seed))
    ux = u_in + 0.01 * rng.standard_normal((ny, nx))
    uy = 0.01 * rng.standard_normal((ny, nx))
    dens = 1.0 + 0.01 * rng.standard_normal((ny, nx))
    feq = _feq(dens, ux, uy) * (solid == 0)
    o.set_f(np.asarray(C, float)[:, None, None, None] * feq[None])
    return o, w


def test_zou_he_inlet_velocity_and_outlet_density_exact():
    """Sec. III D, single fluid (no interfacial force, so the stored velocity is sum f e / rho):
    after every step the inlet column carries exactly (u_in, 0) and the outlet column exactly
    rho_out with zero transverse momentum, under a flow that is far from uniform there."""
    u_in, rho_out = 0.01, 1.02
    o, w = _zou_he_channel((0.0, 0.0, 1.0), u_in, rho_out)
    ex, ey, _ = po.lattice()
    asym = 0.0
    for step in range(40):
        o.step(1)
        f = o.f().sum(0)  # total populations [9, ny, nx]
        rho = f.sum(0)
        jx = (f * ex[:, None, None]).sum(0)
        jy = (f * ey[:, None, None]).sum(0)
        np.testing.assert_allclose(jx[:, 0] / rho[:, 0], u_in, rtol=0, atol=1e-15)
        np.testing.assert_allclose(jy[:, 0] / rho[:, 0], 0.0, rtol=0, atol=5e-16)
        np.testing.assert_allclose(rho[:, -1], rho_out, rtol=0, atol=2e-15)
        np.testing.assert_allclose(jy[:, -1], 0.0, rtol=0, atol=5e-16)
        asym = max(asym, np.abs(f[2, :, 0] - f[4, :, 0]).max(), np.abs(f[2, :, -1] - f[4, :, -1]).max())
    assert asym > 1e-4, asym  # the transverse correction of the rule is exercised


def test_zou_he_composition_readings():
    """Sec. III D composition readings: the inlet's incoming populations carry pure fluid 3
    (fluids 1 and 2 have none), and the outlet's unknown populations carry the node's own
    composition, so a uniform mixture leaving through the outlet keeps its composition exactly
    (the inlet's disturbance has not reached the outlet in 12 steps)."""
    C = (0.2, 0.3, 0.5)
    o, w = _zou_he_channel(C, pillar=False, seed=1)
    for _ in range(12):
        o.step(1)
        f = o.f()
        for a in (1, 5, 8):
            assert np.abs(f[0, a, :, 0]).max() == 0.0 and np.abs(f[1, a, :, 0]).max() == 0.0
        r = o.rho()
        comp = r / r.sum(0)
        for k in range(3):
            np.testing.assert_allclose(comp[k][:, -8:], C[k], rtol=0, atol=2e-15)
    # and fluid 3 enters: the inlet column holds more of it than the initial mixture
    assert (comp[2][:, 0] > C[2] + 1e-3).all()


# ---- characteristic-line fallbacks (Sec. II B, reading of the march's ends) -------------------

def _slot_domain(open_right):
    """A one-column fluid slot at x = 10 between walls (rows 0 and ny-1 solid), fluid 1 graded up
    the slot, fluid 3 elsewhere.  With open_right, an open fluid region x >= 11, y >= 3 joins the
    slot, so from the slot's bottom node (10, 0) the right characteristic line reaches fluid and
    the left one cannot."""
    nx, ny = 40, 30
    solid = np.ones((ny, nx), np.uint8)
    solid[1:ny - 1, 10] = 0
    if open_right:
        solid[3:ny - 1, 11:25] = 0  # (the left line, wrapping round x, meets only solid)
    rho = np.zeros((3, ny, nx))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c1 = np.clip(0.15 + 0.02 * y + 0.01 * (x - 10), 0, 1)
    fl = solid == 0
    rho[0][fl] = c1[fl]
    rho[2][fl] = 1 - c1[fl]
    return W.Workload("slot", nx, ny, 0, W.BC_PERIODIC, (0.1,) * 3, (0.01,) * 3, (30.0, 90.0), solid, rho)


@pytest.mark.parametrize("open_right", [False, True])
def test_fill_march_fallbacks(open_right):
    """Fluid 1 at 30 degrees (fluid 2 absent, so Eq. 21 gives theta_1 = theta13 and the lines leave
    60 degrees off the normal (0, 1) of the slot's bottom node P = (10, 0)).  Both lines into the
    solid: no crossing within t <= 24 has all-fluid nodes (brute force), and P takes C(D0), the
    normal line's first fluid crossing, the node (10, 1).  One line open: P takes that line's
    interpolated value (brute-force crossing), not the Eq. 22 max over two lines."""
    w = _slot_domain(open_right)
    o = po.Oracle(w)
    o.prepare()
    idx, nrm = o.fill_nodes()
    p = [n for n, (i, j, t, _) in enumerate(idx) if (i, j) == (10, 0)]
    assert len(p) == 1
    p = p[0]
    np.testing.assert_allclose(nrm[p], (0.0, 1.0), atol=1e-15)
    r = o.rho()
    C1 = r[0] / np.where(w.solid == 0, r.sum(0), 1.0)
    phi = math.radians(60.0)
    hits = []
    for sgn in (1, -1):  # l1 = cos(phi) n + sin(phi) tau, tau = (-n_y, n_x) = (-1, 0)
        dx, dy = -sgn * math.sin(phi), math.cos(phi)
        hits.append(brute_force_march(w.solid, 0, 10, 0, dx, dy))
    Cext = o.ext_C()
    got = Cext[0, o.PY + 0, 10]
    fail_bits = idx[p, 3] & 3
    if not open_right:
        assert not hits[0][0] and not hits[1][0]
        assert fail_bits == 3
        assert got == C1[1, 10]  # C(D0): the normal line meets the node (10, 1)
    else:
        ok = [h[0] for h in hits]
        assert ok.count(True) == 1
        h = hits[ok.index(True)]
        (i0, j0), (i1, j1), wt = h[1], h[2], h[3]
        expect = C1[j0, i0] + wt * (C1[j1, i1] - C1[j0, i0])
        assert (i0, j0) != (i1, j1) and 0 < wt < 1
        assert abs(got - expect) < 1e-15, (got, expect)
        assert fail_bits == (2 if ok[0] else 1)
    np.testing.assert_allclose(Cext[2, o.PY, 10], 1 - got, atol=1e-15)
