"""The measurement module (paper_2102_04709_amd/diagnostics.py) on fields whose answer is known in
closed form: diffuse interfaces built from exact circles and lines, and Eq. (24)-(26)."""
import math

import numpy as np
import pytest

from paper_2102_04709_amd import diagnostics as dg


def _profile(dist, width=2.0):
    """Mass fraction across a diffuse interface at signed distance dist (positive inside)."""
    return 0.5 * (1.0 + np.tanh(dist / width))


def _wall_drop(theta_deg, R=30.0, nx=200, ny=100, xc=100.0, yw=0.5):
    """A drop (fluid 0) in fluid 2 on the wall y = yw meeting it at theta inside the drop: its
    circle has radius R and centre (xc, yw - R cos(theta))."""
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    yc = yw - R * math.cos(math.radians(theta_deg))
    c0 = _profile(R - np.hypot(x - xc, y - yc))
    C = np.zeros((3, ny, nx))
    C[0], C[2] = c0, 1 - c0
    return C


@pytest.mark.parametrize("theta", [45.0, 60.0, 90.0, 120.0, 150.0])
def test_flat_contact_angle_of_exact_circles(theta):
    C = _wall_drop(theta)
    got = dg.flat_contact_angle(C, 0, 2, 0, 0.5, band=(2.0, 25.0))
    assert abs(got - theta) < 0.3, (got, theta)
    # measured inside the other fluid: the supplement
    got2 = dg.flat_contact_angle(C, 0, 2, 2, 0.5, band=(2.0, 25.0))
    assert abs(got2 - (180 - theta)) < 0.3


def test_flat_contact_angle_of_a_straight_interface():
    ny, nx = 60, 80
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    ang = math.radians(70.0)  # the line leaves the wall at 70 degrees measured on its right
    d = (x - 40.0) * math.sin(ang) - (y - 0.5) * math.cos(ang)
    C = np.zeros((3, ny, nx))
    C[0] = _profile(d)
    C[2] = 1 - C[0]
    got = dg.flat_contact_angle(C, 0, 2, 0, 0.5, band=(2.0, 30.0))
    assert abs(got - 70.0) < 0.1, got


@pytest.mark.parametrize("theta", [45.0, 90.0, 120.0, 150.0])
def test_cylinder_angle_recovers_eq23(theta):
    Rs, Rj, cx, cy = 40.0, 45.0, 100.0, 60.0
    D = dg.eq23_distance(Rs, Rj, theta)
    ny = nx = 200
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    c0 = _profile(Rj - np.hypot(x - cx, y - cy - D))
    C = np.zeros((3, ny, nx))
    C[0] = c0 * (x < cx)
    C[1] = c0 * (x >= cx)
    C[2] = 1 - c0
    r = dg.cylinder_contact_angle(C, [0, 1], 2, (cx, cy, Rs))
    assert abs(r["theta"] - theta) < 0.3 and abs(r["R_j"] - Rj) < 0.2 and abs(r["D_sj"] - D) < 0.2, r


def test_junction_angles_of_three_rays():
    """Three straight interfaces meeting at (60, 50) with fluid sectors of 100, 120 and 140 degrees."""
    ny, nx = 100, 120
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    phi = np.degrees(np.arctan2(y - 50.0, x - 60.0)) % 360.0
    bounds = [(0.0, 100.0), (100.0, 220.0), (220.0, 360.0)]
    C = np.zeros((3, ny, nx))
    for k, (a, b) in enumerate(bounds):
        C[k] = ((phi >= a) & (phi < b)).astype(float)
    # smooth a little so that crossings interpolate
    for _ in range(2):
        C = (C + np.roll(C, 1, 1) + np.roll(C, -1, 1) + np.roll(C, 1, 2) + np.roll(C, -1, 2)) / 5.0
    r = dg.junction_angles(C, (60.0, 50.0), radius=30.0, exclude=4.0)
    assert np.allclose(r["angles"], [100.0, 120.0, 140.0], atol=1.0), r
    assert np.allclose(r["junction"], [60.0, 50.0], atol=0.5)


def test_neumann_angles():
    assert np.allclose(dg.neumann_angles(0.01, 0.01, 0.01), [120.0, 120.0, 120.0])
    a = dg.neumann_angles(0.008, 0.01, 0.012)
    assert abs(sum(a) - 360.0) < 1e-9


@pytest.mark.parametrize("mus", [(0.35, 0.35, 0.35), (0.35, 0.0035, 0.35), (0.35, 0.0035, 0.0035)])
def test_intrusion_solution_solves_eq24(mus):
    """Eq. (25)-(26) solve Eq. (24) with s(0) = s0: central differences of s(t) against the rate."""
    mr, mg, mb = mus
    kw = dict(L=450.0, Lg=100.0, H=30.0, sigma_gb=0.01, theta_gb_deg=30.0, sigma_gr=0.01,
              theta_gr_deg=60.0, mu_r=mr, mu_g=mg, mu_b=mb)
    s0 = 50.0
    t = np.linspace(0.0, 2e5, 41)
    s = dg.intrusion_eq25(t, s0, **kw)
    assert abs(s[0] - s0) < 1e-9
    h = 1.0
    for tk in t[1:-1]:
        ds = (dg.intrusion_eq25(tk + h, s0, **kw) - dg.intrusion_eq25(tk - h, s0, **kw)) / (2 * h)
        rate = dg.intrusion_eq24_rate(float(dg.intrusion_eq25(tk, s0, **kw)), **kw)
        assert abs(ds - rate) <= 1e-6 * abs(rate)
