"""Seeded synthetic workloads for the three-phase D2Q9 step: geometry and initial fields only.

This module holds none of the method's arithmetic.  It turns the problem set-ups of the
paper's Sec. III (flat-wall Janus droplet, Janus droplet on a cylinder, ternary capillary
intrusion, compound droplet among pillars) into plain arrays -- a solid mask, the exact
circles, the initial partial densities -- and the physical parameters.  Both the GPU library
and the CPU oracle take their inputs from here.

Conventions: node (i, j) sits at (x, y) = (i, j); arrays are [ny, nx] (x fastest); a node is
inside a circle when |x - c|^2 < R^2 for the initial phases (strict) and solid when
|x - c|^2 <= R^2.  Fluids 1, 2, 3 are the paper's red, green, blue unless a set-up says
otherwise.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

BC_PERIODIC = 0
BC_PERIODIC_SWAP13 = 1
BC_ZOUHE = 2


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    y_periodic: int
    bc_x: int
    nu: Tuple[float, float, float]
    sigma: Tuple[float, float, float]          # sigma12, sigma13, sigma23
    theta_deg: Tuple[float, float]             # theta13, theta23
    solid: np.ndarray                          # uint8 [ny, nx]
    rho_init: np.ndarray                       # float64 [3, ny, nx]
    circles: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    u_in: float = 0.0
    rho_out: float = 1.0
    beta0: float = 0.7
    body_force: Tuple[float, float] = (0.0, 0.0)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny

    def with_params(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def _walls(nx: int, ny: int) -> np.ndarray:
    s = np.zeros((ny, nx), np.uint8)
    s[0, :] = 1
    s[ny - 1, :] = 1
    return s


def _disk(x, y, cx, cy, r):
    return (x - cx) ** 2 + (y - cy) ** 2 < r * r


def _solid_disk(x, y, cx, cy, r):
    return (x - cx) ** 2 + (y - cy) ** 2 <= r * r


def _phases(masks: Sequence[np.ndarray], solid: np.ndarray) -> np.ndarray:
    """Sharp partial densities: masks for fluids 1 and 2 (fluid 3 is the rest), zero in solid."""
    ny, nx = solid.shape
    rho = np.zeros((3, ny, nx))
    m1 = masks[0] & ~solid.astype(bool)
    m2 = masks[1] & ~solid.astype(bool) & ~m1
    rho[0][m1] = 1.0
    rho[1][m2] = 1.0
    rho[2][~(m1 | m2) & ~solid.astype(bool)] = 1.0
    return rho


# ---- Sec. III A: Janus droplet on a flat wall --------------------------------------------

def flat_janus(nx=120, ny=60, R=20.0, theta=(60.0, 120.0), sigma=(0.01, 0.01, 0.01),
               nu=(0.1, 0.1, 0.1), two_half_disks=True, name="flat_janus") -> Workload:
    """Walls are the solid rows j = 0 and j = ny-1 (halfway bounce-back puts the wall surface
    at y = 0.5).  Two half-disks of radius R centred on the wall surface at x = nx/3 and 2nx/3
    (fluid 1 left, fluid 2 right, touching at x = nx/2), or, with two_half_disks=False, one
    half-disk centred at x = nx/2 split at its centre line.  Fluid 3 is ambient."""
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny)
    yc = 0.5
    if two_half_disks:
        m1 = _disk(x, y, nx / 3.0, yc, R)
        m2 = _disk(x, y, 2.0 * nx / 3.0, yc, R)
    else:
        d = _disk(x, y, nx / 2.0, yc, R)
        m1 = d & (x < nx / 2.0)
        m2 = d & (x >= nx / 2.0)
    return Workload(name, nx, ny, 0, BC_PERIODIC, tuple(nu), tuple(sigma), tuple(theta),
                    solid, _phases([m1, m2], solid))


# Table I of Sec. III A: (theta_rg, theta_br, theta_gb) in degrees, theta_kl measured inside fluid k.
TABLE1 = {"a": (90.0, 60.0, 120.0), "b": (60.0, 90.0, 120.0), "c": (120.0, 60.0, 90.0),
          "d": (60.0, 120.0, 90.0), "e": (90.0, 90.0, 90.0), "f": (90.0, 120.0, 60.0)}


def janus_flat_table1(case="c", scale=1.0, R=None) -> Workload:
    """Sec. III A with the paper's labels (red -> fluid 1, green -> fluid 2, blue -> fluid 3): a
    semicircular Janus droplet of radius 80 s (red left half, blue right half) resting on the wall
    surface y = 0.5 at the centre of a (320 s) x (180 s) domain, surrounded by green; walls are the
    solid rows 0 and ny-1, periodic in x; viscosities 0.1, tensions 0.01.  Table I's angles enter
    as theta13 = theta_rb = 180 - theta_br and theta23 = theta_gb (theta12 = theta_rg follows from
    Eq. 18).  R overrides the radius (Fig. 3's resolution series keeps the domain 4 R x 2.25 R)."""
    rg, br, gb = TABLE1[case]
    if R is None:
        R = 80.0 * scale
    nx, ny = int(round(4.0 * R)), int(round(2.25 * R))
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny)
    d = _disk(x, y, nx / 2.0, 0.5, R)
    fl = solid == 0
    rho = np.zeros((3, ny, nx))
    rho[0][d & (x < nx / 2.0) & fl] = 1.0
    rho[2][d & (x >= nx / 2.0) & fl] = 1.0
    rho[1][~d & fl] = 1.0
    return Workload(f"table1_{case}_R{R:g}", nx, ny, 0, BC_PERIODIC, (0.1, 0.1, 0.1), (0.01, 0.01, 0.01),
                    (180.0 - br, gb), solid, rho)


def janus_cylinder(theta=90.0, scale=1.0) -> Workload:
    """Sec. III B with the paper's labels (red -> 1, green -> 2, blue -> 3): a perfect Janus droplet
    (red left, blue right; the negligible red-blue tension taken as 1e-4) on a cylinder of radius
    40 s centred at (100 s, 60 s) in a (200 s) x (200 s) domain, surrounded by green; walls are the
    solid rows 0 and ny-1, periodic in x; viscosities 0.1, sigma_rg = sigma_gb = 0.01 and
    theta_rg = theta_bg = theta.  With sigma_rb -> 0, Eq. (18) leaves theta_br = 90, so the inputs
    are theta13 = theta_rb = 90 and theta23 = theta_gb = 180 - theta (theta12 = theta_rg = theta).
    The droplet starts as a disk of radius 45 s centred 66 s above the cylinder's centre (the
    paper does not give the start; the equilibrium radius R_j and distance D_sj are measured)."""
    nx = ny = int(round(200 * scale))
    Rs, Rj = 40.0 * scale, 45.0 * scale
    cx, cy, D0 = 100.0 * scale, 60.0 * scale, 66.0 * scale
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny) | _solid_disk(x, y, cx, cy, Rs).astype(np.uint8)
    fl = solid == 0
    d = _disk(x, y, cx, cy + D0, Rj) & fl
    rho = np.zeros((3, ny, nx))
    rho[0][d & (x < cx)] = 1.0
    rho[2][d & (x >= cx)] = 1.0
    rho[1][~d & fl] = 1.0
    return Workload(f"janus_cylinder_{theta:g}_s{scale:g}", nx, ny, 0, BC_PERIODIC, (0.1, 0.1, 0.1),
                    (0.01, 1e-4, 0.01), (90.0, 180.0 - theta), solid, rho, circles=np.array([[cx, cy, Rs]]))


# ---- Sec. III B: Janus droplet on a cylinder ---------------------------------------------

def cylinder_janus(nx=400, ny=400, Rs=60.0, Rj=50.0, centre=None, theta=(90.0, 90.0),
                   sigma=(0.005, 0.005, 0.005), nu=(0.05, 0.1, 0.2), name="cylinder_janus"
                   ) -> Workload:
    """Flat solid rows at j = 0 and j = ny-1, a solid cylinder of radius Rs (exact circle, for
    the interpolated bounce-back), and a Janus droplet of radius Rj resting tangent on top of
    it, split vertically through the cylinder axis: fluid 1 left, fluid 2 right."""
    x, y = _grid(nx, ny)
    cx, cy = centre if centre is not None else ((nx - 1) / 2.0, (ny - 1) / 2.0)
    solid = _walls(nx, ny)
    solid |= _solid_disk(x, y, cx, cy, Rs).astype(np.uint8)
    dy = cy + Rs + Rj
    d = _disk(x, y, cx, dy, Rj)
    m1 = d & (x < cx)
    m2 = d & (x >= cx)
    return Workload(name, nx, ny, 0, BC_PERIODIC, tuple(nu), tuple(sigma), tuple(theta),
                    solid, _phases([m1, m2], solid), circles=np.array([[cx, cy, Rs]]))


def cylinder_janus_hbm(scale=10) -> Workload:
    """The cylinder case scaled by `scale` in every length (4000 x 4000 for scale 10)."""
    return cylinder_janus(nx=400 * scale, ny=400 * scale, Rs=60.0 * scale, Rj=50.0 * scale,
                          name=f"cylinder_janus_x{scale}")


# ---- Sec. III C: ternary capillary intrusion ---------------------------------------------

def capillary_intrusion(nx=1024, ny=64, ratio=1.0, slug=200, lg=200,
                        sigma=(0.01, 0.012, 0.015), theta=(45.0, 90.0), nu_low=0.01,
                        name="capillary_intrusion") -> Workload:
    """Channel between the solid rows j = 0 and j = ny-1, periodic in x with fluids 1 and 3
    exchanged at the x boundary.  Fluid 1 fills x < slug, fluid 2 slug <= x < slug + lg,
    fluid 3 the rest.  Viscosities (nu_low * ratio, nu_low, nu_low)."""
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny)
    m1 = x < slug
    m2 = (x >= slug) & (x < slug + lg)
    nu = (nu_low * ratio, nu_low, nu_low)
    return Workload(name, nx, ny, 0, BC_PERIODIC_SWAP13, nu, tuple(sigma), tuple(theta),
                    solid, _phases([m1, m2], solid))


def intrusion_sec3c(theta_gr=60.0, theta_gb=30.0, mu=(0.35, 0.35, 0.35), L=450, H=30, s0=50, Lg=100,
                    name=None) -> Workload:
    """Sec. III C with the paper's labels (red -> 1, green -> 2, blue -> 3): a capillary tube of
    length L and width H (solid rows 0 and H+1, so H fluid rows between halfway walls), red on
    x < s0, green on s0 <= x < s0 + Lg, blue beyond; the modified periodic x boundary exchanges red
    and blue; equal tensions 0.01; viscosities mu = (mu_r, mu_g, mu_b) (mu_k = nu_k, rho_k^0 = 1).
    The wall angles theta_gr and theta_gb (inside green) enter as theta13 = theta_rb with
    cos theta_br = cos theta_gr - cos theta_gb (Eq. 18, equal tensions) and theta23 = theta_gb.
    s0 and Lg are not given in the paper (chosen here)."""
    nx, ny = L, H + 2
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny)
    fl = solid == 0
    rho = np.zeros((3, ny, nx))
    rho[0][(x < s0) & fl] = 1.0
    rho[1][(x >= s0) & (x < s0 + Lg) & fl] = 1.0
    rho[2][(x >= s0 + Lg) & fl] = 1.0
    c_br = math.cos(math.radians(theta_gr)) - math.cos(math.radians(theta_gb))
    theta13 = 180.0 - math.degrees(math.acos(c_br))
    return Workload(name or f"intrusion_{theta_gr:g}_{theta_gb:g}_{mu[1] / mu[0]:g}_{mu[2] / mu[0]:g}", nx, ny, 0,
                    BC_PERIODIC_SWAP13, tuple(mu), (0.01, 0.01, 0.01), (theta13, theta_gb), solid, rho)


# ---- Sec. III D: compound droplet among random pillars -----------------------------------

def _place_pillars(rng, nx, ny, count, rmin, rmax, drop, clear, gap, edge):
    pillars: List[Tuple[float, float, float]] = []
    tries = 0
    while len(pillars) < count and tries < 20000:
        tries += 1
        r = float(rng.uniform(rmin, rmax))
        cx = float(rng.uniform(edge + r, nx - 1 - edge - r))
        cy = float(rng.uniform(r + 3.0, ny - 1 - 3.0 - r))
        if math.hypot(cx - drop[0], cy - drop[1]) < clear + r:
            continue
        if any(math.hypot(cx - px, cy - py) < r + pr + gap for px, py, pr in pillars):
            continue
        pillars.append((cx, cy, r))
    return pillars


def pillar_domain(seed: int, nx: Optional[int] = None, ny: Optional[int] = None,
                  n_pillars: Optional[int] = None, theta=None, sigma=None, nu=(1 / 6, 1 / 6, 1 / 6),
                  u_in=0.005, r_core=15.0, r_shell=25.0, name=None) -> Workload:
    """A compound droplet (core fluid 1 of radius r_core inside a shell of fluid 2 of radius
    r_shell, centred at (2 r_shell, ny/2)) in ambient fluid 3, upstream of circular pillars.
    Periodic in y; Zou-He velocity inlet (u_in, 0) at x = 0 and pressure outlet (rho = 1) at
    x = nx-1.  Sizes, pillar count, radii (8..24) and centres are drawn from numpy's PCG64
    with the given seed; pillars keep a gap of 4 between each other, a clear disk of radius 40
    around the droplet centre and stay 8 columns away from the inlet and outlet."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if nx is None:
        nx = int(rng.integers(256, 1025))
    if ny is None:
        ny = int(rng.integers(128, 513))
    if n_pillars is None:
        n_pillars = int(rng.integers(4, 21))
    drop = (2.0 * r_shell, ny / 2.0)
    pillars = _place_pillars(rng, nx, ny, n_pillars, 8.0, 24.0, drop, 40.0, 4.0, 8.0)
    if theta is None:
        tw = float(rng.choice([30.0, 90.0, 150.0]))
        theta = (tw, tw)
    if sigma is None:
        s = 0.005 * nu[2] / 0.04  # capillary number U mu / sigma = 0.04
        sigma = (s, s, s)
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), np.uint8)
    for cx, cy, r in pillars:
        solid |= _solid_disk(x, y, cx, cy, r).astype(np.uint8)
    m1 = _disk(x, y, drop[0], drop[1], r_core)
    m2 = _disk(x, y, drop[0], drop[1], r_shell)
    return Workload(name or f"pillars_{seed}", nx, ny, 1, BC_ZOUHE, tuple(nu), tuple(sigma),
                    tuple(theta), solid, _phases([m1, m2], solid),
                    circles=np.array(pillars, dtype=np.float64).reshape(-1, 3), u_in=u_in,
                    rho_out=1.0)


def pillar_sweep(n_domains=96, base_seed=2102_000) -> List[Workload]:
    """The batched sweep: domain i uses seed base_seed + i."""
    return [pillar_domain(base_seed + i) for i in range(n_domains)]


def inverse_problem(hidden=False) -> Workload:
    """The inverse problem: a 512 x 256 channel (periodic in y, Zou-He inlet u = 0.005 at x = 0,
    outlet rho = 1 at x = nx-1) with 12 random pillars (seed 4709; radii 8..24, gap 4, 8
    columns from the inlet and outlet) and the compound droplet of the sweep (core fluid 1 of
    radius 15 inside a shell of fluid 2 of radius 25) resting against the upstream side of a
    pillar, its centre 13 nodes from the pillar surface, so that both fluids touch the solid from
    the first step and the contact angles shape the phase fields.  The host pillar is the first
    one (in drawing order) with room for the droplet (2 nodes clear of every other pillar, 12
    columns from the inlet, inside the periodic strip).  hidden=True gives the parameters that
    produce the target phase fields, otherwise the point at which gradients are taken."""
    if hidden:
        theta, sigma = (40.0, 110.0), (0.020, 0.012, 0.010)
    else:
        theta, sigma = (50.0, 100.0), (0.018, 0.011, 0.011)
    nx, ny, r_core, r_shell, gap_core = 512, 256, 15.0, 25.0, 13.0
    rng = np.random.Generator(np.random.PCG64(4709))
    pillars = _place_pillars(rng, nx, ny, 12, 8.0, 24.0, (-1e9, -1e9), 0.0, 4.0, 8.0)
    drop = None
    for cx, cy, r in pillars:
        dx, dy = cx - r - gap_core, cy
        if dx - r_shell < 12.0 or dy - r_shell < 2.0 or dy + r_shell > ny - 3.0:
            continue
        if any(math.hypot(dx - px, dy - py) < pr + r_shell + 2.0
               for px, py, pr in pillars if (px, py, pr) != (cx, cy, r)):
            continue
        drop = (dx, dy)
        break
    assert drop is not None
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), np.uint8)
    for cx, cy, r in pillars:
        solid |= _solid_disk(x, y, cx, cy, r).astype(np.uint8)
    m1 = _disk(x, y, drop[0], drop[1], r_core)
    m2 = _disk(x, y, drop[0], drop[1], r_shell)
    nu = (1 / 6, 1 / 6, 1 / 6)
    return Workload("inverse_hidden" if hidden else "inverse_guess", nx, ny, 1, BC_ZOUHE, nu, sigma, theta,
                    solid, _phases([m1, m2], solid), circles=np.array(pillars, dtype=np.float64).reshape(-1, 3),
                    u_in=0.005, rho_out=1.0)


# ---- small cases used by tests ------------------------------------------------------------

def static_disk(n=96, R=20.0, sigma13=0.01, nu=0.1, inner=0, outer=2) -> Workload:
    """Fully periodic box with a disk of fluid `inner` in fluid `outer` (Laplace test)."""
    x, y = _grid(n, n)
    solid = np.zeros((n, n), np.uint8)
    rho = np.zeros((3, n, n))
    d = _disk(x, y, (n - 1) / 2.0, (n - 1) / 2.0, R)
    rho[inner][d] = 1.0
    rho[outer][~d] = 1.0
    return Workload("static_disk", n, n, 1, BC_PERIODIC, (nu, nu, nu), (sigma13, sigma13, sigma13),
                    (90.0, 90.0), solid, rho)


def random_mixture(nx, ny, seed, walls=True, y_periodic=None, bc_x=BC_PERIODIC, circles=(),
                   theta=(60.0, 100.0), sigma=(0.01, 0.012, 0.011), nu=(0.1, 0.07, 0.13),
                   smooth=2) -> Workload:
    """Smooth random three-fluid field (for parity tests): three random fields, box-filtered,
    turned into positive partial densities summing to one.  Optional walls and circles."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = _grid(nx, ny)
    solid = _walls(nx, ny) if walls else np.zeros((ny, nx), np.uint8)
    for cx, cy, r in circles:
        solid |= _solid_disk(x, y, cx, cy, r).astype(np.uint8)
    raw = rng.random((3, ny, nx))
    for _ in range(smooth):
        raw = (raw + np.roll(raw, 1, 1) + np.roll(raw, -1, 1) + np.roll(raw, 1, 2) + np.roll(raw, -1, 2)) / 5.0
    raw = np.maximum(raw - raw.mean() * 0.6, 1e-3) ** 3
    rho = raw / raw.sum(0, keepdims=True)
    rho[:, solid.astype(bool)] = 0.0
    yp = (0 if walls else 1) if y_periodic is None else y_periodic
    return Workload(f"random_{seed}", nx, ny, yp, bc_x, tuple(nu), tuple(sigma), tuple(theta),
                    solid, rho, circles=np.array(circles, dtype=np.float64).reshape(-1, 3),
                    u_in=0.004 if bc_x == BC_ZOUHE else 0.0)
