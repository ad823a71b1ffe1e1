// lbm3_internal.h -- device layout and helpers shared by the host set-up and the gfx950
// kernels of liblbm3 (never by the CPU checker).
//
// Data layout in HBM, per domain d with plane size P_d = pitch_d * (ny_d + 4):
//   distributions : 9 planes of storage type S, the shift f_a - w_a (rho^0 = 1)
//   densities     : 3 planes of compute type T, the partial densities rho_k at fluid nodes and
//                   the filled mass fractions C_k at the solid boundary nodes
//   flags         : 1 plane of uint8
// A plane holds rows -2 .. ny+1 (two padding rows on each side hold the off-grid solid layers
// of a non-periodic y boundary); row j starts at element pitch*(j+2).  All domains' planes
// are concatenated: domain d starts at element base_d = sum of P over the earlier domains
// (times 9 for the distributions and 3 for the densities).  x is the fastest index, so a
// wavefront reads 64 consecutive nodes of one row.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#ifndef __HIPCC__
#define __host__
#define __device__
#endif

namespace lbm3 {

constexpr int kThreads = 256;  // work-group size of every kernel but the fill
constexpr int kFillNodes = 32;  // fill nodes per work-group of the fill kernel (four lanes each)

// A work-group of the fill kernel: fill nodes first .. first + count - 1 (count <= kFillNodes),
// all of domain dom.
struct FillBlock {
  int32_t dom, first, count, pad_;
};

enum : uint8_t {
  FL_SOLID = 1,   // solid node (mask, or off-grid row of a non-periodic y boundary)
  FL_FILL = 2,    // solid node whose C is filled by the wetting condition (C_SB or C_SB2)
  FL_CURVED = 4,  // fluid node with at least one interpolated-bounce-back link
  FL_IBBSRC = 8,  // fluid node whose post-collision population a neighbour's interpolated
                  // bounce-back reads (a link cut at q < 1/2 with this node behind it)
};

enum { BCX_PERIODIC = 0, BCX_SWAP13 = 1, BCX_ZOUHE = 2 };

// Per-domain constants, in device memory.
struct DomainDev {
  int32_t nx, ny, pitch, yper;
  int32_t bcx, n_fill, fill_off, n_ibb;
  int32_t ibb_off, work_off, n_work, pad_;
  int64_t base;   // element offset of plane 0 of this domain (before the x9 / x3 factors)
  int64_t plane;  // P = pitch * (ny + 4)
  int64_t abase;  // element offset of this domain in the adjoint's extended planes
  int64_t goff;   // element offset of this domain in flat [3][ny][nx] field arrays
  double u_in, rho_out;
  double nu[3];
  double inu[3];   // 1 / nu_k, formed on the host (IEEE FP64 division)
  double sig[3];   // sigma12, sigma13, sigma23
  double gX[3];    // g(X_kl) of Eq. (15) for the pairs 12, 13, 23
  double beta0;
  double th13, th23, th12;  // radians
  double g[2];     // body acceleration
};

// Fluid indicator of the 11 x 11 block around a fill node (offsets -kMaskR..kMaskR): bit
// (dy + kMaskR) * kMaskW + (dx + kMaskR) of the two words.  Most characteristic lines hit within
// it, so their march reads no memory.
constexpr int kMaskR = 5, kMaskW = 2 * kMaskR + 1;

struct FluidMask {
  uint64_t w[2];
  __host__ __device__ static bool inside(int dx, int dy) {
    return dx >= -kMaskR && dx <= kMaskR && dy >= -kMaskR && dy <= kMaskR;
  }
  __host__ __device__ bool fluid(int dx, int dy) const {  // for offsets inside the block
    const int b = (dy + kMaskR) * kMaskW + dx + kMaskR;
    return ((b < 64 ? w[0] >> b : w[1] >> (b - 64)) & 1) != 0;
  }
  void set(int dx, int dy) {
    const int b = (dy + kMaskR) * kMaskW + dx + kMaskR;
    w[b >> 6] |= (uint64_t)1 << (b & 63);
  }
};

// A solid node whose C is filled (C_SB or C_SB2), with its fluid-pointing unit normal and the
// point D0 where its normal line first meets the fluid (two plane indices and a weight; the
// normal is fixed, so D0 is found once at set-up).
struct FillNode {
  int32_t dom, i, j, li;  // domain, coordinates, index within the domain's plane
  int32_t d0a, d0b;       // plane indices of the interpolation nodes of D0
  double d0w;             // C(D0) = C(d0a) + d0w (C(d0b) - C(d0a))
  double nx, ny;
  FluidMask mask;         // fluid indicator of the block around the node
};

// A characteristic line's crossing D for one of the angles Eq. (21) gives when at most two fluids
// are present at D0 (theta13 or theta12 for fluid 1, theta23 or theta21 for fluid 2, or the mean
// of the pair when neither of the other two is present): the two interpolation nodes as plane
// indices (a < 0: the line reaches no fluid) and the weight, C(D) = C(a) + w (C(b) - C(a)).
// Formed once in FP64 at set-up (and when the angles change) with the march of the fill.
// phi_lo..phi_hi: the line angles phi = |pi/2 - theta| around the candidate's over which the
// march crosses the same grid lines in the same order and classifies them alike up to its hit
// (bounded by the angles of rays through lattice nodes and of axis-parallel rays, with a margin;
// phi_lo > phi_hi: none), so a line whose angle lies there has its hit at the same crossing:
// the march may start there, at crossing counters kx, ky, and reach the same result.
struct FillCand {
  int32_t a, b;
  double w;
  double phi_lo, phi_hi;
  int32_t kx, ky;
};
constexpr int kFillCands = 3;  // candidate angles per fluid

// A fluid node with interpolated-bounce-back links: q[a-1] for direction a = 1..8 is the
// fraction of the link from the node towards x - e_a at which the wall lies (1/2 when the link
// is not cut by a circle).
struct IbbNode {
  int32_t li, dom;
  double q[8];
};

// A tile (x0, y0 and the context's tile shape) or a strip (columns x0..x1-1, rows y0..y1-1).
// kind: WK_INNER when the tile's three halo rings lie inside the grid (no index wraps or clamps),
// WK_PLAIN when the tile and its first ring are all fluid and touch no Zou-He or fluid-
// exchanging x boundary column (streaming is a plain pull).
enum : int32_t { WK_INNER = 1, WK_PLAIN = 2 };
// ibb_begin, ibb_count: the item's range of TileIbb entries (tiles of the step; zero otherwise).
// pitch, base, plane: the domain's row pitch, state offset and plane size (as in DomainDev),
// repeated here so that a tile's first loads need its work item only.
struct WorkItem {
  int32_t dom, x0, y0, x1, y1, kind, ibb_begin, ibb_count;
  int32_t pitch = 0, pad_ = 0;
  int64_t base = 0, plane = 0;
};

// An interpolated-bounce-back node of a step tile: its position q = lx + TX ly in the tile and the
// index of its IbbNode record.
struct TileIbb {
  int32_t q, idx;
};


__host__ __device__ inline int64_t plane_index(int i, int j, int pitch) {
  return (int64_t)i + (int64_t)pitch * (j + 2);
}

// Element (i, j) of a domain's extended plane in the adjoint's scratch: columns -1..nx, rows
// -2..ny+1.
__host__ __device__ inline int64_t adj_index(const DomainDev &D, int i, int j) {
  return D.abase + (i + 1) + (int64_t)(D.nx + 2) * (j + 2);
}

// ---- characteristic line (Sec. II B) ------------------------------------------------------
// From node (pi, pj) along (dx, dy), t > 0, visit the crossings with the vertical lines
// x = integer and the horizontal lines y = integer in increasing t.  At a horizontal line the
// two nodes left and right of the crossing are interpolated, at a vertical line the two nodes
// below and above; a crossing within 1e-9 of a node uses that node alone.  The first crossing
// whose nodes are all fluid is the intersection point D; beyond t = 24 the line fails.
constexpr double kEpsDir = 1e-12;
constexpr double kEpsNode = 1e-9;
constexpr double kTMax = 24.0;

struct LineHit {
  int ok;
  int i0, j0, i1, j1;  // interpolation nodes (equal for a node hit)
  double w;            // value = v(i0, j0) + w * (v(i1, j1) - v(i0, j0))
};

// kx, ky: the indices of the next vertical and horizontal crossings to visit (1, 1 from the
// node; a march that resumes another one's passes that march's state).
// hit_k (may be null): receives the counters kx, ky with which the hit crossing was reached.
template <class FluidAt>
__host__ __device__ inline LineHit march_line(int pi, int pj, double dx, double dy,
                                              const FluidAt &fluid, int kx = 1, int ky = 1, int *hit_k = nullptr) {
  LineHit h;
  h.ok = 0;
  h.i0 = h.j0 = h.i1 = h.j1 = 0;
  h.w = 0.0;
  const int sx = dx > kEpsDir ? 1 : (dx < -kEpsDir ? -1 : 0);
  const int sy = dy > kEpsDir ? 1 : (dy < -kEpsDir ? -1 : 0);
  const double ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
  const double iax = sx ? 1.0 / ax : 0.0, iay = sy ? 1.0 / ay : 0.0;
  for (int guard = 0; guard < 256; ++guard) {
    if (hit_k) { hit_k[0] = kx; hit_k[1] = ky; }
    const double tx = sx ? (double)kx * iax : 1e300;  // t of the next vertical line
    const double ty = sy ? (double)ky * iay : 1e300;  // t of the next horizontal line
    const double t = tx < ty ? tx : ty;
    if (t > kTMax) return h;
    if (tx <= ty) {
      const int i = pi + sx * kx;
      const double y = pj + tx * dy;
      const double yr = floor(y + 0.5);
      ++kx;
      if (fabs(y - yr) < kEpsNode) {
        const int j = (int)yr;
        if (sy && j == pj + sy * ky) ++ky;
        if (fluid(i, j)) {
          h.ok = 1; h.i0 = h.i1 = i; h.j0 = h.j1 = j; h.w = 0.0;
          return h;
        }
      } else {
        const int j0 = (int)floor(y);
        if (fluid(i, j0) && fluid(i, j0 + 1)) {
          h.ok = 1; h.i0 = h.i1 = i; h.j0 = j0; h.j1 = j0 + 1; h.w = y - j0;
          return h;
        }
      }
    } else {
      const int j = pj + sy * ky;
      const double x = pi + ty * dx;
      const double xr = floor(x + 0.5);
      ++ky;
      if (fabs(x - xr) < kEpsNode) {
        const int i = (int)xr;
        if (sx && i == pi + sx * kx) ++kx;
        if (fluid(i, j)) {
          h.ok = 1; h.i0 = h.i1 = i; h.j0 = h.j1 = j; h.w = 0.0;
          return h;
        }
      } else {
        const int i0 = (int)floor(x);
        if (fluid(i0, j) && fluid(i0 + 1, j)) {
          h.ok = 1; h.i0 = i0; h.i1 = i0 + 1; h.j0 = h.j1 = j; h.w = x - i0;
          return h;
        }
      }
    }
  }
  return h;
}

// march_line with the fluid tests of a (2R + 1)^2 block around the node answered by test(dx, dy)
// (a bit mask, no memory access): the same crossings in the same order with the same arithmetic,
// so its hit is march_line's.  A line that needs a node outside the block (or more crossings than
// the block can hold) before it hits is handed to fallback(kx, ky) at that crossing: every
// crossing before it failed the block's test, which agrees with the fallback's on the block, so
// the fallback's first hit from there is the line's.  kx, ky: as for march_line.
template <int R, class BlockTest, class Fallback>
__host__ __device__ inline LineHit march_line_block(int pi, int pj, double dx, double dy, const BlockTest &test,
                                                    const Fallback &fallback, int kx = 1, int ky = 1) {
  LineHit h;
  h.ok = 0;
  h.i0 = h.j0 = h.i1 = h.j1 = 0;
  h.w = 0.0;
  const int sx = dx > kEpsDir ? 1 : (dx < -kEpsDir ? -1 : 0);
  const int sy = dy > kEpsDir ? 1 : (dy < -kEpsDir ? -1 : 0);
  const double ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy;
  const double iax = sx ? 1.0 / ax : 0.0, iay = sy ? 1.0 / ay : 0.0;
  for (int it = 0; it < 4 * R + 2; ++it) {
    const double tx = sx ? (double)kx * iax : 1e300;  // t of the next vertical line
    const double ty = sy ? (double)ky * iay : 1e300;  // t of the next horizontal line
    const bool vert = tx <= ty;
    if ((vert ? tx : ty) > kTMax) return h;
    const int line = vert ? pi + sx * kx : pj + sy * ky;  // the column or row crossed
    const double c = vert ? pj + tx * dy : pi + ty * dx;  // the other coordinate there
    const double cr = floor(c + 0.5);
    const bool node = fabs(c - cr) < kEpsNode;
    const int c0 = node ? (int)cr : (int)floor(c);
    // block offsets of the crossing's node (node) or of its two interpolation nodes; a crossing
    // outside the block goes to the fallback before the indices move past it
    const int a0 = vert ? line - pi : c0 - pi, b0 = vert ? c0 - pj : line - pj;
    const int a1 = (vert || node) ? a0 : a0 + 1, b1 = (vert && !node) ? b0 + 1 : b0;
    if (a0 < -R || a1 > R || b0 < -R || b1 > R) break;
    if (vert) {
      ++kx;
      if (node && sy && c0 == pj + sy * ky) ++ky;
    } else {
      ++ky;
      if (node && sx && c0 == pi + sx * kx) ++kx;
    }
    if (test(a0, b0) && test(a1, b1)) {
      h.ok = 1;
      h.i0 = pi + a0; h.j0 = pj + b0; h.i1 = pi + a1; h.j1 = pj + b1;
      h.w = node ? 0.0 : c - c0;
      return h;
    }
  }
  return fallback(kx, ky);
}

// The wetting fill's march: the 11 x 11 mask of the fill record first; a line leaving it
// continues, from the crossing where it left, over the 25 x 25 block of the node's far mask (rows
// of 25 bits, offsets -12..12, bit dx + 12 of row dy + 12); beyond that march_line continues over
// the flags.
constexpr int kFarR = 12, kFarW = 2 * kFarR + 1;

template <class FluidAt>
__host__ __device__ inline LineHit march_line_masked(int pi, int pj, double dx, double dy, const FluidMask &mask,
                                                     const uint32_t *far_rows, const FluidAt &fluid, int kx = 1,
                                                     int ky = 1) {
  auto near_test = [&](int a, int b) { return mask.fluid(a, b); };
  auto far_test = [&](int a, int b) { return ((far_rows[b + kFarR] >> (a + kFarR)) & 1u) != 0; };
  auto general = [&](int kx, int ky) { return march_line(pi, pj, dx, dy, fluid, kx, ky); };
  auto far = [&](int kx, int ky) { return march_line_block<kFarR>(pi, pj, dx, dy, far_test, general, kx, ky); };
  return march_line_block<kMaskR>(pi, pj, dx, dy, near_test, far, kx, ky);
}

// sin and cos of an angle in [0, pi/2] in FP64 (the wetting fill's line angle phi), to a few
// ulp: Taylor series of degree 19 (sine) and 20 (cosine), evaluated by Horner's rule in x^2, on
// [0, pi/4]; above pi/4 the series run on the complementary angle pi/2 - phi (pi/2 split in two
// doubles so that the difference is exact) and the results swap.  A short straight-line
// sequence, unlike a general-argument sine with its range reduction.
constexpr double taylor_coef(int n) {  // (-1)^m / n!, n = 2m or 2m + 1
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f *= k;
  return ((n / 2) % 2 ? -1.0 : 1.0) / f;
}

__host__ __device__ inline void sincos_quadrant(double phi, double &sn, double &cs) {
  const double kPio2Hi = 1.5707963267948966, kPio2Lo = 6.123233995736766e-17;
  const bool comp = phi > 0.78539816339744831;
  const double x = comp ? (kPio2Hi - phi) + kPio2Lo : phi;
  const double x2 = x * x;
  double ps = taylor_coef(19);
  ps = ps * x2 + taylor_coef(17);
  ps = ps * x2 + taylor_coef(15);
  ps = ps * x2 + taylor_coef(13);
  ps = ps * x2 + taylor_coef(11);
  ps = ps * x2 + taylor_coef(9);
  ps = ps * x2 + taylor_coef(7);
  ps = ps * x2 + taylor_coef(5);
  ps = ps * x2 + taylor_coef(3);
  const double s = x + x * x2 * ps;
  double pc = taylor_coef(20);
  pc = pc * x2 + taylor_coef(18);
  pc = pc * x2 + taylor_coef(16);
  pc = pc * x2 + taylor_coef(14);
  pc = pc * x2 + taylor_coef(12);
  pc = pc * x2 + taylor_coef(10);
  pc = pc * x2 + taylor_coef(8);
  pc = pc * x2 + taylor_coef(6);
  pc = pc * x2 + taylor_coef(4);
  pc = pc * x2 + taylor_coef(2);
  const double c = 1.0 + x2 * pc;
  sn = comp ? c : s;
  cs = comp ? s : c;
}

// Host: the radius of lattice nodes whose rays can change a line's march up to its hit h.
inline int line_reach(int pi, int pj, const LineHit &h) {
  return (int)std::ceil(std::hypot(0.5 * (h.i0 + h.i1) - pi, 0.5 * (h.j0 + h.j1) - pj) + 2.0);
}

// Host: the angles in [0, pi/2] at which the fill's line on side s (direction cos(phi) n +
// s sin(phi) t, t = (-n_y, n_x)) is parallel to an axis or passes through a lattice node within
// distance R of its node, sorted.  The march's crossings, their order and their node / segment
// classification change only near these angles (for a hit within distance R - 2).
inline std::vector<double> line_breakpoints(double nx, double ny, double s, int R) {
  const double half_pi = 1.5707963267948966, pi2 = 6.283185307179586, tx = -ny, ty = nx;
  // The ray to node offset q is at angle s (alpha_q - alpha_n) from the normal; the offsets' own
  // angles alpha_q (within radius 8) are formed once.
  constexpr int kTableR = 8;
  struct Offset { double alpha; int r2; };
  static const std::vector<Offset> table = [] {
    std::vector<Offset> t;
    for (int v = -kTableR; v <= kTableR; ++v)
      for (int u = -kTableR; u <= kTableR; ++u)
        if ((u || v) && u * u + v * v <= kTableR * kTableR) t.push_back({std::atan2((double)v, (double)u), u * u + v * v});
    return t;
  }();
  std::vector<double> brk;
  if (R <= kTableR) {
    const double an = std::atan2(ny, nx);
    for (const Offset &o : table) {
      if (o.r2 > R * R) continue;
      double a = s * (o.alpha - an);
      if (a > 3.141592653589793) a -= pi2;
      if (a <= -3.141592653589793) a += pi2;
      if (a >= -1e-6 && a <= half_pi + 1e-6) brk.push_back(a);
    }
  } else {
    for (int v = -R; v <= R; ++v)
      for (int u = -R; u <= R; ++u) {
        if ((u == 0 && v == 0) || u * u + v * v > R * R) continue;
        const double a = std::atan2(s * (u * tx + v * ty), u * nx + v * ny);
        if (a >= -1e-6 && a <= half_pi + 1e-6) brk.push_back(a);
      }
  }
  for (const double a : {std::atan2(-nx, s * tx), std::atan2(-ny, s * ty), std::atan2(nx, -s * tx), std::atan2(ny, -s * ty)})
    if (a >= -1e-6 && a <= half_pi + 1e-6) brk.push_back(a);
  std::sort(brk.begin(), brk.end());
  return brk;
}

// Host: the fill line's march at angle phi on side s, and the range lo..hi of angles around phi
// over which the march meets its hit at the same crossing, reached with counters hk (lo > hi: none;
// also when the line has no hit).  Between two breakpoints (line_breakpoints, for a radius of at
// least the hit's distance + 2), farther from both than the node tolerance's angular width
// (below 1e-9 for nodes at distance 1 or more), the crossings up to the hit are fixed; when phi
// itself is at a breakpoint (a ray through a node), the range is the +-2e-11 over which every
// crossing keeps its class.  The range is kept only if the march at both its ends agrees.
// brk: sorted breakpoints of this side for a radius R_brk (formed here when null or too small).
template <class FluidAt>
inline LineHit line_angle_range(int pi, int pj, double nx, double ny, double s, double phi, const FluidAt &fluid,
                                double &lo, double &hi, int hk[2], const std::vector<double> *brk = nullptr,
                                int R_brk = 0) {
  const double half_pi = 1.5707963267948966, tx = -ny, ty = nx;
  auto march_at = [&](double a, int *k) {
    double sp, cp;
    sincos_quadrant(a, sp, cp);
    sp *= s;
    return march_line(pi, pj, cp * nx + sp * tx, cp * ny + sp * ty, fluid, 1, 1, k);
  };
  hk[0] = hk[1] = 1;
  lo = 1.0;
  hi = 0.0;
  const LineHit h = march_at(phi, hk);
  if (!h.ok) return h;
  const int R = line_reach(pi, pj, h);
  std::vector<double> own;
  if (!brk || R_brk < R) {
    own = line_breakpoints(nx, ny, s, R);
    brk = &own;
  }
  const double m = 1e-9;
  // the nearest breakpoints below phi - m and above phi + m, and whether one lies within m
  const auto b_lo = std::lower_bound(brk->begin(), brk->end(), phi - m);
  const auto b_hi = std::upper_bound(brk->begin(), brk->end(), phi + m);
  double l = b_lo == brk->begin() ? -1.0 : *(b_lo - 1) + m;
  double u = b_hi == brk->end() ? 10.0 : *b_hi - m;
  if (b_lo != b_hi) {  // a ray through a node
    l = phi - 2e-11;
    u = phi + 2e-11;
  }
  l = std::fmax(l, 0.0);
  u = std::fmin(u, half_pi);
  if (!(l <= phi && phi <= u)) return h;
  for (const double a : {l, u}) {
    int k2[2];
    const LineHit g = march_at(a, k2);
    if (!(g.ok && g.i0 == h.i0 && g.j0 == h.j0 && g.i1 == h.i1 && g.j1 == h.j1 && k2[0] == hk[0] && k2[1] == hk[1]))
      return h;
  }
  lo = l;
  hi = u;
  return h;
}

}  // namespace lbm3
