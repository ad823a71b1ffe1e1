// lbm3_api.cpp -- host side of liblbm3: validation, the one-time boundary set-up and the C ABI
// declared in include/lbm3.h.
//
// One-time set-up per domain (Sec. II B of arXiv:2102.04709):
//   - theta12 from the Young relations, Eq. (17)-(18), and g(X_kl) of Eq. (15);
//   - node categories: a solid node touching a fluid node in the D2Q9 8-neighbourhood is a
//     boundary node (C_SB); solid nodes touching C_SB form a second filled layer, because the
//     stress divergence of Eq. (10) at a boundary fluid node reads the stress of its C_SB
//     neighbours, whose own gradient reaches one node further into the solid;
//   - fluid-pointing unit normals by Eq. (19)-(20) (integer weights 960, 448, 84, 32, 1 in units
//     of 1/5040, summed exactly), and a check that every normal line reaches the fluid;
//   - link fractions q of the interpolated bounce-back on the exact circles (FP64);
//   - the (domain, tile) work list of the fused kernel.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lbm3.h"
#include "lbm3_adjoint.h"
#include "lbm3_internal.h"
#include "lbm3_kernels.h"

using namespace lbm3;

namespace {

const int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double kPI = 3.14159265358979323846;

struct Candidate {
  int kernel, tx, ty;
};
// Candidate configurations of the fused kernel (the autotuner picks among them).
const Candidate kCands[] = {{MODE_TILE, 32, 8},      {MODE_TILE, 16, 16},     {MODE_TILE, 64, 4},
                            {MODE_TILE, 64, 8},      {MODE_TILE512, 16, 16},  {MODE_TILE512, 32, 16},
                            {MODE_TILE512, 64, 8},   {MODE_STRIP128, 0, 32},  {MODE_STRIP256, 0, 32},
                            {MODE_STRIP256, 0, 64}};
const int kMinTileArea = 256;
const int kMinStripRows = 8;
const int kFieldTileX = 32, kFieldTileY = 8;  // tile of the field export
// |G_kl| at or below which n_kl := 0 and the pair adds no stress, in every precision (|G|^2 =
// 1e-24 is still a normal FP32 number; a larger FP32 threshold switches normals on and off where
// FP64 keeps them and lets the FP32 path drift from the FP64 one near walls).
const double kEpsG = 1e-12;
// The FP32 adjoint treats n_kl as constant where |G_kl| < 1e-8: below that |G| is smaller than
// the FP32 rounding of the two products it is formed from, and the 1/|G| of the normal's
// derivative feeds rounding noise into a mode of the adjoint that then grows without bound
// (overflow within ~700 steps on the 512 x 256 inverse problem at a cutoff of 1e-10).  The FP64
// adjoint is exact.
const double kEpsNormalAdjF32 = 1e-8;
const int kAdjTileX = 32, kAdjTileY = 8;      // tile of the adjoint kernels

int round_up(int v, int m) { return (v + m - 1) / m * m; }

struct DomHost {
  DomainDev dd;
  std::vector<uint8_t> flags;   // [(ny+4) * pitch]
  std::vector<FillNode> fill;
  std::vector<FillCand> cand;   // [fill][4 lines][kFillCands]
  std::vector<uint32_t> far;    // kFarW rows per fill node: its far fluid mask
  std::vector<IbbNode> ibb;
};

struct Layout {
  size_t off_F[2], off_R[2], off_flags, off_fill, off_fillC, off_ibb, off_doms, off_work, off_fwork, off_partial,
      off_chunk_dom, off_chunk_first, off_mass, off_bad, off_aX, off_awork, off_raw, off_tibb, off_fblk, off_ibbof,
      off_links, off_far, off_lpart, off_lfirst, off_cand, total;
  int64_t total_plane;
  int64_t aplane;  // elements of one adjoint scratch plane (all domains' extended grids)
  int n_fill, n_ibb, n_chunks, max_work, n_fwork, n_awork, n_fblk;
};

size_t s_size(int precision) { return precision == LBM3_F64 ? 8 : (precision == LBM3_F32 ? 4 : 2); }
size_t t_size(int precision) { return precision == LBM3_F64 ? 8 : 4; }

double g_of_X(double X) {
  if (X < -1.0) return 1.0;
  if (X < 0.0) return 1.0 - std::sqrt(1.0 - X * X);
  if (X <= 1.0) return std::sqrt(1.0 - X * X) - 1.0;
  return -1.0;
}

// X_kl of Eq. (15) for the pair whose own tension is c, the other two being a and b:
// X = (a^2 + b^2 - c^2) / (2ab), with its partials.
double pair_X(double c, double a, double b, double *dc = nullptr, double *da = nullptr, double *db = nullptr) {
  if (dc) *dc = -c / (a * b);
  if (da) *da = (a * a - b * b + c * c) / (2.0 * a * a * b);
  if (db) *db = (b * b - a * a + c * c) / (2.0 * a * b * b);
  return (a * a + b * b - c * c) / (2.0 * a * b);
}

double g_of_X_prime(double X) {
  if (X <= -1.0 || X >= 1.0) return 0.0;
  const double r = std::sqrt(1.0 - X * X);
  return X < 0.0 ? X / r : -X / r;
}

// The parameters a domain derives from (theta13, theta23) and the tensions: theta12 by Eq. (18)
// (with theta31 = pi - theta13) and g(X_kl) of Eq. (15).  Returns an error message or null.
const char *derive_params(const double *theta_deg, const double *sigma, DomainDev &D) {
  for (int k = 0; k < 3; ++k)
    if (!(sigma[k] > 0.0)) return "every interfacial tension must be > 0";
  for (int k = 0; k < 2; ++k)
    if (!(theta_deg[k] > 0.0 && theta_deg[k] < 180.0)) return "contact angles must lie in (0, 180) degrees";
  const double th13 = theta_deg[0] * kPI / 180.0, th23 = theta_deg[1] * kPI / 180.0;
  double c12 = (sigma[1] * std::cos(th13) - sigma[2] * std::cos(th23)) / sigma[0];
  if (std::fabs(c12) > 1.0 + 1e-12) return "contact angles and tensions violate Eq. (18): |cos theta12| > 1";
  c12 = std::min(1.0, std::max(-1.0, c12));
  const double s12 = sigma[0], s13 = sigma[1], s23 = sigma[2];
  for (int k = 0; k < 3; ++k) D.sig[k] = sigma[k];
  D.gX[0] = g_of_X(pair_X(s12, s13, s23));
  D.gX[1] = g_of_X(pair_X(s13, s12, s23));
  D.gX[2] = g_of_X(pair_X(s23, s12, s13));
  D.th13 = th13;
  D.th23 = th23;
  D.th12 = std::acos(c12);
  return nullptr;
}

// J[r][p]: derivative of the raw parameter r of the adjoint kernels (sigma12, sigma13, sigma23,
// g(X_12), g(X_13), g(X_23), theta13, theta23, theta12 in radians) with respect to the public
// parameter p (theta13, theta23 in degrees, sigma12, sigma13, sigma23).
void param_jacobian(const double *theta_deg, const double *sigma, double J[9][5]) {
  for (int r = 0; r < 9; ++r)
    for (int p = 0; p < 5; ++p) J[r][p] = 0.0;
  const double deg = kPI / 180.0;
  for (int k = 0; k < 3; ++k) J[k][2 + k] = 1.0;
  const double s12 = sigma[0], s13 = sigma[1], s23 = sigma[2];
  double dc, da, db;
  // pair 12: own s12, others s13, s23
  double X = pair_X(s12, s13, s23, &dc, &da, &db), g = g_of_X_prime(X);
  J[3][2] = g * dc; J[3][3] = g * da; J[3][4] = g * db;
  X = pair_X(s13, s12, s23, &dc, &da, &db); g = g_of_X_prime(X);
  J[4][3] = g * dc; J[4][2] = g * da; J[4][4] = g * db;
  X = pair_X(s23, s12, s13, &dc, &da, &db); g = g_of_X_prime(X);
  J[5][4] = g * dc; J[5][2] = g * da; J[5][3] = g * db;
  J[6][0] = deg;
  J[7][1] = deg;
  const double th13 = theta_deg[0] * deg, th23 = theta_deg[1] * deg;
  const double c12 = (s13 * std::cos(th13) - s23 * std::cos(th23)) / s12;
  if (std::fabs(c12) < 1.0) {
    const double dth = -1.0 / std::sqrt(1.0 - c12 * c12);  // d theta12 / d cos theta12
    J[8][0] = dth * (-s13 * std::sin(th13) / s12) * deg;
    J[8][1] = dth * (s23 * std::sin(th23) / s12) * deg;
    J[8][2] = dth * (-c12 / s12);
    J[8][3] = dth * (std::cos(th13) / s12);
    J[8][4] = dth * (-std::cos(th23) / s12);
  }
}

// The crossings of a fill node's four characteristic lines (fluid k = line / 2, side line % 2) for
// the angles Eq. (21) gives when at most two fluids are present at D0: fluid 1 theta13, theta12 or
// their mean, fluid 2 theta23, theta21 = pi - theta12 or their mean; with the fill's own angle
// clamp, sine and cosine and march, in FP64.  flags: the domain's flag plane.
// The angle ranges (and crossing counters) of a fill node's candidates depend only on its normal,
// the candidate angles and the fluid flags its marches test: when every candidate's march stays in
// the node's 11 x 11 block, on the node's fluid mask (FillNode::mask), so nodes with the same
// mask and normal (flat walls) share them.
constexpr int kRangeReach = 26;
struct CandRangeCache {
  struct Entry {
    int32_t rel[4 * kFillCands][4];  // the crossing's nodes relative to the fill node
    double lo[4 * kFillCands], hi[4 * kFillCands];
    int32_t kx[4 * kFillCands], ky[4 * kFillCands];
  };
  std::unordered_map<std::string, Entry> map;
};

void fill_candidates(const DomainDev &D, const uint8_t *flags, const FillNode &fn, FillCand *out,
                     CandRangeCache *cache) {
  const double PI = 3.14159265358979323846;
  const bool zh = D.bcx == BCX_ZOUHE;
  auto fluid_at = [&](int i, int j) -> bool {
    if (zh) {
      if (i < 0 || i >= D.nx) return false;
    } else {
      i = ((i % D.nx) + D.nx) % D.nx;
    }
    if (D.yper) j = ((j % D.ny) + D.ny) % D.ny;
    else if (j < 0 || j >= D.ny) return false;
    return !(flags[plane_index(i, j, D.pitch)] & FL_SOLID);
  };
  auto wrapped = [&](int i, int j) {
    if (!zh) i = ((i % D.nx) + D.nx) % D.nx;
    if (D.yper) j = ((j % D.ny) + D.ny) % D.ny;
    return (int32_t)plane_index(i, j, D.pitch);
  };
  const double th21 = PI - D.th12;
  const double ang[2][kFillCands] = {{D.th13, D.th12, 0.5 * (D.th13 + D.th12)}, {D.th23, th21, 0.5 * (D.th23 + th21)}};
  auto phi_of = [&](int line, int c) {
    const double tk = std::min(std::max(ang[line >> 1][c], 5.0 * PI / 180.0), 175.0 * PI / 180.0);
    return std::fabs(0.5 * PI - tk);
  };
  // Angle ranges only for crossings within a reach of kRangeReach (nearly all: the lines that go
  // farther are few, and their breakpoint sets large), from one sorted set of breakpoints per side
  // (lines 0, 2: +t; 1, 3: -t) for the farthest of those crossings.
  LineHit hit[4][kFillCands];
  int R[2] = {0, 0};
  bool in_block = true;
  for (int line = 0; line < 4; ++line)
    for (int c = 0; c < kFillCands; ++c) {
      double sp, cp;
      sincos_quadrant(phi_of(line, c), sp, cp);
      if (line & 1) sp = -sp;
      const double tx = -fn.ny, ty = fn.nx;
      // (the block march: the same hit as march_line's; it reports a line that leaves the block)
      auto leaves = [&](int kx, int ky) {
        in_block = false;
        return march_line(fn.i, fn.j, cp * fn.nx + sp * tx, cp * fn.ny + sp * ty, fluid_at, kx, ky);
      };
      auto near_test = [&](int a, int b) { return fn.mask.fluid(a, b); };
      hit[line][c] = march_line_block<kMaskR>(fn.i, fn.j, cp * fn.nx + sp * tx, cp * fn.ny + sp * ty, near_test, leaves);
      const int r = hit[line][c].ok ? line_reach(fn.i, fn.j, hit[line][c]) : kRangeReach + 1;
      if (r <= kRangeReach) R[line & 1] = std::max(R[line & 1], r);
    }
  for (int line = 0; line < 4; ++line)
    for (int c = 0; c < kFillCands; ++c) {
      const LineHit &h = hit[line][c];
      out[line * kFillCands + c] = h.ok ? FillCand{wrapped(h.i0, h.j0), wrapped(h.i1, h.j1), h.w, 1.0, 0.0, 1, 1}
                                        : FillCand{-1, -1, 0.0, 1.0, 0.0, 1, 1};
    }
  bool all_near = in_block;
  for (int line = 0; line < 4; ++line)
    for (int c = 0; c < kFillCands; ++c)
      all_near = all_near && hit[line][c].ok && line_reach(fn.i, fn.j, hit[line][c]) <= kRangeReach;
  std::string key;
  if (cache && all_near) {
    const double head[5] = {fn.nx, fn.ny, D.th13, D.th12, D.th23};
    key.assign(reinterpret_cast<const char *>(head), sizeof head);
    key.append(reinterpret_cast<const char *>(fn.mask.w), sizeof fn.mask.w);
    const auto it = cache->map.find(key);
    if (it != cache->map.end()) {
      const CandRangeCache::Entry &e = it->second;
      for (int q = 0; q < 4 * kFillCands; ++q) {
        const LineHit &h = hit[q / kFillCands][q % kFillCands];
        if (e.rel[q][0] != h.i0 - fn.i || e.rel[q][1] != h.j0 - fn.j || e.rel[q][2] != h.i1 - fn.i ||
            e.rel[q][3] != h.j1 - fn.j)
          continue;  // (cannot differ: the same surroundings give the same crossings)
        out[q].phi_lo = e.lo[q];
        out[q].phi_hi = e.hi[q];
        out[q].kx = e.kx[q];
        out[q].ky = e.ky[q];
      }
      return;
    }
  }
  const std::vector<double> brk[2] = {line_breakpoints(fn.nx, fn.ny, 1.0, R[0]), line_breakpoints(fn.nx, fn.ny, -1.0, R[1])};
  for (int line = 0; line < 4; ++line)
    for (int c = 0; c < kFillCands; ++c) {
      FillCand &o = out[line * kFillCands + c];
      const LineHit &h = hit[line][c];
      if (!h.ok || line_reach(fn.i, fn.j, h) > kRangeReach) continue;
      double lo, hi;
      int hk[2];
      const LineHit g = line_angle_range(fn.i, fn.j, fn.nx, fn.ny, (line & 1) ? -1.0 : 1.0, phi_of(line, c), fluid_at,
                                         lo, hi, hk, &brk[line & 1], R[line & 1]);
      if (g.ok && g.i0 == h.i0 && g.j0 == h.j0 && g.i1 == h.i1 && g.j1 == h.j1) {
        o.phi_lo = lo;
        o.phi_hi = hi;
        o.kx = hk[0];
        o.ky = hk[1];
      }
    }
  if (cache && all_near) {
    CandRangeCache::Entry e;
    for (int q = 0; q < 4 * kFillCands; ++q) {
      const LineHit &h = hit[q / kFillCands][q % kFillCands];
      e.rel[q][0] = h.i0 - fn.i; e.rel[q][1] = h.j0 - fn.j; e.rel[q][2] = h.i1 - fn.i; e.rel[q][3] = h.j1 - fn.j;
      e.lo[q] = out[q].phi_lo; e.hi[q] = out[q].phi_hi; e.kx[q] = out[q].kx; e.ky[q] = out[q].ky;
    }
    cache->map.emplace(std::move(key), e);
  }
}

bool validate_and_build(const lbm3_domain &d, int dom, double beta0, DomHost &H, std::string &err) {
  char buf[256];  // detail of a message; fail() formats into its own buffer (never from buf into buf)
  auto fail = [&](const char *m) {
    char out[320];
    snprintf(out, sizeof out, "domain %d: %s", dom, m);
    err = out;
    return false;
  };
  if (d.nx < 3 || d.ny < 3) return fail("nx and ny must be >= 3");
  if (d.bc_x < 0 || d.bc_x > 2) return fail("bc_x must be 0, 1 or 2");
  if (d.reserved != 0) return fail("reserved must be 0");
  if (d.bc_x == LBM3_X_ZOUHE && !d.y_periodic) return fail("the Zou-He x boundary requires y_periodic = 1");
  if (d.bc_x == LBM3_X_PERIODIC_SWAP13 && d.n_circles > 0) return fail("circles are not allowed with the fluid-exchanging periodic boundary");
  if (d.n_circles < 0 || (d.n_circles > 0 && !d.circles)) return fail("bad circle list");
  if (!d.solid || !d.rho_init) return fail("solid and rho_init are required");
  if (d.bc_x == LBM3_X_ZOUHE && !(std::fabs(d.u_in) < 0.5 && d.rho_out > 0.0)) return fail("bad Zou-He inlet velocity or outlet density");
  for (int k = 0; k < 3; ++k) {
    if (!(d.sigma[k] > 0.0)) return fail("every interfacial tension must be > 0");
    const double tau = 0.5 + 3.0 * d.nu[k];
    if (!(tau > 0.5 && tau <= 10.0)) return fail("viscosity gives tau outside (0.5, 10]");
  }
  {
    DomainDev tmp;
    const char *m = derive_params(d.theta_deg, d.sigma, tmp);
    if (m) return fail(m);
  }
  const int nx = d.nx, ny = d.ny;
  const int pitch = round_up(nx, 64);
  const int rows = ny + 4;
  DomainDev &D = H.dd;
  memset(&D, 0, sizeof D);
  D.nx = nx;
  D.ny = ny;
  D.pitch = pitch;
  D.yper = d.y_periodic ? 1 : 0;
  D.bcx = d.bc_x;
  D.plane = (int64_t)pitch * rows;
  D.u_in = d.u_in;
  D.rho_out = d.rho_out;
  for (int k = 0; k < 3; ++k) {
    D.nu[k] = d.nu[k];
    D.inu[k] = 1.0 / d.nu[k];
  }
  (void)derive_params(d.theta_deg, d.sigma, D);
  D.beta0 = beta0;
  D.g[0] = d.body_force[0];
  D.g[1] = d.body_force[1];

  if (d.bc_x == LBM3_X_ZOUHE)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < 3; ++i)
        if (d.solid[(size_t)j * nx + i] || d.solid[(size_t)j * nx + nx - 1 - i]) return fail("solid nodes within 3 columns of a Zou-He boundary");

  // Base solid indicator on rows -2..ny+1; padding columns and unused rows are solid.
  H.flags.assign((size_t)rows * pitch, FL_SOLID);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) H.flags[plane_index(i, j, pitch)] = d.solid[(size_t)j * nx + i] ? FL_SOLID : 0;
  const bool yper = D.yper;
  const bool zh = D.bcx == BCX_ZOUHE;
  const int jlo = yper ? 0 : -2, jhi = yper ? ny - 1 : ny + 1;
  // s(x) of Eq. (19): solid beyond a non-periodic y boundary, fluid beyond a Zou-He column.
  auto solid_at = [&](int i, int j) -> bool {
    if (zh) {
      if (i < 0 || i >= nx) return false;
    } else {
      i = ((i % nx) + nx) % nx;
    }
    if (yper) j = ((j % ny) + ny) % ny;
    else if (j < -2 || j > ny + 1) return true;
    return H.flags[plane_index(i, j, pitch)] & FL_SOLID;
  };
  auto fluid_at = [&](int i, int j) -> bool {
    if (zh) {
      if (i < 0 || i >= nx) return false;
    } else {
      i = ((i % nx) + nx) % nx;
    }
    if (yper) j = ((j % ny) + ny) % ny;
    else if (j < 0 || j >= ny) return false;
    return !(H.flags[plane_index(i, j, pitch)] & FL_SOLID);
  };
  // C_SB: solid nodes with a fluid node among their 8 neighbours.
  std::vector<uint8_t> cat((size_t)rows * pitch, 0);  // 1 = C_SB, 2 = second layer
  for (int j = jlo; j <= jhi; ++j)
    for (int i = 0; i < nx; ++i) {
      if (!solid_at(i, j)) continue;
      for (int a = 1; a < 9; ++a)
        if (fluid_at(i + kEX[a], j + kEY[a])) {
          cat[plane_index(i, j, pitch)] = 1;
          break;
        }
    }
  auto is_sb = [&](int i, int j) -> bool {
    if (zh) {
      if (i < 0 || i >= nx) return false;
    } else {
      i = ((i % nx) + nx) % nx;
    }
    if (yper) j = ((j % ny) + ny) % ny;
    else if (j < -2 || j > ny + 1) return false;
    return cat[plane_index(i, j, pitch)] == 1;
  };
  for (int j = jlo; j <= jhi; ++j)
    for (int i = 0; i < nx; ++i) {
      const int64_t p = plane_index(i, j, pitch);
      if (!solid_at(i, j) || cat[p] == 1) continue;
      for (int a = 1; a < 9; ++a)
        if (is_sb(i + kEX[a], j + kEY[a])) {
          cat[p] = 2;
          break;
        }
    }
  // Fill list with Eq. (19)-(20) normals.
  CandRangeCache ranges;  // (shared by the domain's fill nodes)
  for (int pass = 1; pass <= 2; ++pass)
    for (int j = jlo; j <= jhi; ++j)
      for (int i = 0; i < nx; ++i) {
        const int64_t p = plane_index(i, j, pitch);
        if (cat[p] != pass) continue;
        long sx = 0, sy = 0;
        for (int cy = -2; cy <= 2; ++cy)
          for (int cx = -2; cx <= 2; ++cx) {
            const int r2 = cx * cx + cy * cy;
            if (r2 == 0 || !solid_at(i + cx, j + cy)) continue;
            const long w = r2 == 1 ? 960 : r2 == 2 ? 448 : r2 == 4 ? 84 : r2 == 5 ? 32 : 1;
            sx += w * cx;
            sy += w * cy;
          }
        if (sx == 0 && sy == 0) {
          snprintf(buf, sizeof buf, "degenerate solid normal at node (%d,%d)", i, j);
          return fail(buf);
        }
        const double len = std::sqrt((double)sx * sx + (double)sy * sy);
        FillNode fn;
        fn.dom = dom;
        fn.i = i;
        fn.j = j;
        fn.li = (int32_t)p;
        fn.nx = -(double)sx / len;
        fn.ny = -(double)sy / len;
        const LineHit h0 = march_line(i, j, fn.nx, fn.ny, fluid_at);
        if (!h0.ok) {
          snprintf(buf, sizeof buf, "the normal line from solid node (%d,%d) reaches no fluid node", i, j);
          return fail(buf);
        }
        auto wrapped = [&](int ii, int jj) {
          if (!zh) ii = ((ii % nx) + nx) % nx;
          if (yper) jj = ((jj % ny) + ny) % ny;
          return (int32_t)plane_index(ii, jj, pitch);
        };
        fn.d0a = wrapped(h0.i0, h0.j0);
        fn.d0b = wrapped(h0.i1, h0.j1);
        fn.d0w = h0.w;
        fn.mask.w[0] = fn.mask.w[1] = 0;
        for (int dy = -kMaskR; dy <= kMaskR; ++dy)
          for (int dx = -kMaskR; dx <= kMaskR; ++dx)
            if (fluid_at(i + dx, j + dy)) fn.mask.set(dx, dy);
        for (int dy = -kFarR; dy <= kFarR; ++dy) {
          uint32_t row = 0;
          for (int dx = -kFarR; dx <= kFarR; ++dx)
            if (fluid_at(i + dx, j + dy)) row |= 1u << (dx + kFarR);
          H.far.push_back(row);
        }
        H.flags[p] |= FL_FILL;
        H.fill.push_back(fn);
        H.cand.resize(H.cand.size() + 4 * kFillCands);
        fill_candidates(D, H.flags.data(), fn, H.cand.data() + H.cand.size() - 4 * kFillCands, &ranges);
      }
  // Interpolated bounce-back link fractions.
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int64_t p = plane_index(i, j, pitch);
      if (H.flags[p] & FL_SOLID) continue;
      IbbNode node;
      node.li = (int32_t)p;
      node.dom = dom;
      bool any = false;
      for (int a = 1; a < 9; ++a) {
        node.q[a - 1] = 0.5;
        const int si = i - kEX[a], sj = j - kEY[a];
        if (zh && (si < 0 || si >= nx)) continue;
        if (fluid_at(si, sj)) continue;
        bool found = false;
        double q = 0.5;
        for (int c = 0; c < d.n_circles; ++c) {
          for (int ix = -1; ix <= 1; ++ix)
            for (int iy = -1; iy <= 1; ++iy) {
              if (ix && zh) continue;
              if (iy && !yper) continue;
              const double cx = d.circles[3 * c] + ix * nx, cy = d.circles[3 * c + 1] + iy * ny, R = d.circles[3 * c + 2];
              const double dxs = si - cx, dys = sj - cy, dxf = i - cx, dyf = j - cy;
              if (dxs * dxs + dys * dys > R * R) continue;
              if (dxf * dxf + dyf * dyf <= R * R) continue;
              const double a2 = kEX[a] * kEX[a] + kEY[a] * kEY[a];
              const double b = kEX[a] * dxf + kEY[a] * dyf;
              const double cc = dxf * dxf + dyf * dyf - R * R;
              const double disc = b * b - a2 * cc;
              const double qq = (b - std::sqrt(std::max(disc, 0.0))) / a2;
              if (!found || qq < q) q = qq;
              found = true;
            }
        }
        if (found) {
          node.q[a - 1] = std::min(std::max(q, 1e-6), 1.0);
          any = true;
          // a cut link with q < 1/2 reads the post-collision population of the fluid node behind
          if (node.q[a - 1] < 0.5 && fluid_at(i + kEX[a], j + kEY[a])) {
            int bi = i + kEX[a], bj = j + kEY[a];
            if (!zh) bi = ((bi % nx) + nx) % nx;
            if (yper) bj = ((bj % ny) + ny) % ny;
            H.flags[plane_index(bi, bj, pitch)] |= FL_IBBSRC;
          }
        }
      }
      if (any) {
        H.flags[p] |= FL_CURVED;
        H.ibb.push_back(node);
      }
    }
  return true;
}

int tiles_of(int nx, int ny, int tx, int ty) { return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty); }

bool plan(const lbm3_domain *d, int n, const lbm3_options *o, std::vector<DomHost> &H, Layout &L,
          std::string &err) {
  if (!d || n < 1) return err = "need at least one domain", false;
  if (!o) return err = "options are required", false;
  if (o->precision < 0 || o->precision > 2) return err = "bad precision", false;
  if (o->kernel < -1 || o->kernel > 3) return err = "kernel must be -1, 0, 1, 2 or 3", false;
  if (o->tile_x < 0 || o->tile_y < 0 || o->graph_block_steps < 0 || o->persistent_blocks < 0) return err = "negative option", false;
  const bool tiles = o->kernel <= 0 || o->kernel == MODE_TILE512;
  if (tiles && (o->tile_x > 0 || o->tile_y > 0)) {
    const int mode = o->kernel == MODE_TILE512 ? MODE_TILE512 : MODE_TILE;
    const int area = o->tile_x * o->tile_y;
    if (o->tile_x <= 0 || o->tile_y <= 0 || area < kMinTileArea || !tile_supported(mode, o->tile_x, o->tile_y) ||
        step_smem_bytes(o->precision, mode, o->tile_x, o->tile_y) > 160 * 1024)
      return err = "tile shape not supported (256 threads: 32x8, 16x16, 64x4, 64x8; 512 threads: 16x16, "
                   "32x16, 64x8; within 160 KiB of LDS)", false;
  }
  if (!tiles && o->tile_y > 0 && o->tile_y < kMinStripRows) return err = "strip segments need at least 8 rows", false;
  const double beta0 = o->beta0 > 0 ? o->beta0 : 0.7;
  // The step kernels address a plane as a base plus a 32-bit byte offset: a domain's padded plane
  // (nx rounded up to 64, rows -2..ny+1) of the arithmetic type stays below 4 GiB.
  const int64_t max_plane = (int64_t(1) << 32) / (o->precision == LBM3_F64 ? 8 : 4);
  for (int i = 0; i < n; ++i)
    if (d[i].nx >= 3 && d[i].ny >= 3 && ((int64_t)d[i].nx + 63) / 64 * 64 * ((int64_t)d[i].ny + 4) >= max_plane) {
      char m[160];
      snprintf(m, sizeof m, "domain %d: the padded plane (nx rounded up to 64, times ny + 4) must hold fewer than %lld nodes",
               i, (long long)max_plane);
      return err = m, false;
    }
  H.assign(n, DomHost());
  {  // the domains are independent: up to 16 host threads take them in turn; the first failing
     // domain (in index order) reports
    std::vector<std::string> errs(n);
    std::vector<char> ok(n, 0);
    std::atomic<int> next{0};
    auto work = [&]() {
      for (int i; (i = next.fetch_add(1)) < n;) ok[i] = validate_and_build(d[i], i, beta0, H[i], errs[i]);
    };
    const int nt = std::min(n, std::max(1, std::min(16, (int)std::thread::hardware_concurrency())));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (std::thread &t : pool) t.join();
    for (int i = 0; i < n; ++i)
      if (!ok[i]) return err = errs[i], false;
  }
  if (o->adjoint != 0 && o->adjoint != 1) return err = "adjoint must be 0 or 1", false;
  if (o->adjoint && o->precision == LBM3_F32_STORE_F16) return err = "the adjoint needs LBM3_F64 or LBM3_F32", false;
  int64_t base = 0, abase = 0, goff = 0;
  int nf = 0, ni = 0, nch = 0, maxw = 0, nfw = 0, naw = 0, nfb = 0;
  for (int i = 0; i < n; ++i) {
    H[i].dd.base = base;
    base += H[i].dd.plane;
    H[i].dd.abase = abase;
    abase += (int64_t)(d[i].nx + 2) * (d[i].ny + 4);
    H[i].dd.goff = goff;
    goff += 3 * (int64_t)d[i].nx * d[i].ny;
    naw += tiles_of(d[i].nx + 2, d[i].ny + 4, kAdjTileX, kAdjTileY);
    H[i].dd.fill_off = nf;
    H[i].dd.n_fill = (int)H[i].fill.size();
    nf += H[i].dd.n_fill;
    nfb += (H[i].dd.n_fill + kFillNodes - 1) / kFillNodes;
    H[i].dd.ibb_off = ni;
    H[i].dd.n_ibb = (int)H[i].ibb.size();
    ni += H[i].dd.n_ibb;
    nch += (d[i].ny + 15) / 16;
    int mw = 0;
    for (const Candidate &t : kCands)
      if (is_tile_mode(t.kernel)) mw = std::max(mw, tiles_of(d[i].nx, d[i].ny, t.tx, t.ty));
    mw = std::max(mw, tiles_of(d[i].nx, d[i].ny, 122, kMinStripRows));
    if (o->tile_x > 0 && o->tile_y > 0) mw = std::max(mw, tiles_of(d[i].nx, d[i].ny, o->tile_x, o->tile_y));
    maxw += mw;
    nfw += tiles_of(d[i].nx, d[i].ny, kFieldTileX, kFieldTileY);
  }
  const int prec = o->precision;
  L.total_plane = base;
  L.n_fill = nf;
  L.n_fblk = nfb;
  L.n_ibb = ni;
  L.n_chunks = nch;
  L.max_work = maxw;
  L.n_fwork = nfw;
  L.aplane = abase;
  L.n_awork = o->adjoint ? naw : 0;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += (bytes + 255) / 256 * 256;
    return r;
  };
  for (int b = 0; b < 2; ++b) {
    L.off_F[b] = take(9 * (size_t)base * s_size(prec));
    L.off_R[b] = take(3 * (size_t)base * t_size(prec));
  }
  L.off_flags = take((size_t)base);
  L.off_fill = take(sizeof(FillNode) * std::max(nf, 1));
  L.off_fillC = take(3 * t_size(prec) * std::max(nf, 1));
  L.off_tibb = take(sizeof(TileIbb) * std::max(ni, 1));
  L.off_fblk = take(sizeof(FillBlock) * std::max(nfb, 1));
  L.off_far = take(sizeof(uint32_t) * kFarW * (size_t)std::max(nf, 1));
  L.off_cand = take(sizeof(FillCand) * 4 * kFillCands * (size_t)std::max(nf, 1));
  L.off_ibb = take(sizeof(IbbNode) * std::max(ni, 1));
  L.off_doms = take(sizeof(DomainDev) * n);
  L.off_work = take(sizeof(WorkItem) * maxw);
  L.off_fwork = take(sizeof(WorkItem) * nfw);
  L.off_partial = take(sizeof(double) * 3 * nch);
  L.off_chunk_dom = take(sizeof(int) * nch);
  L.off_chunk_first = take(sizeof(int) * (n + 1));
  L.off_mass = take(sizeof(double) * 3 * n);
  L.off_bad = take(sizeof(int));
  L.off_aX = L.off_awork = L.off_raw = L.off_ibbof = L.off_links = L.off_lpart = L.off_lfirst = 0;
  if (o->adjoint) {
    L.off_aX = take((size_t)A_PLANES * (size_t)abase * t_size(prec));
    L.off_awork = take(sizeof(WorkItem) * naw);
    L.off_raw = take(sizeof(double) * 9 * n);
    L.off_ibbof = take(sizeof(int32_t) * (size_t)base);
    L.off_links = take(sizeof(uint32_t) * (size_t)base);
    L.off_lpart = take(sizeof(double) * (size_t)std::max(nfw, 1));
    L.off_lfirst = take(sizeof(int) * (size_t)(n + 1));
  }
  L.total = off;
  return true;
}

}  // namespace

struct lbm3_ctx {
  int n = 0;
  int device = 0;               // the GPU current at creation
  double *mass_scratch = nullptr;  // that GPU's fixed scratch of lbm3_mass_device
  std::string tune_cache;       // lbm3_options.tune_cache ("" = none)
  int precision = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<DomainDev> doms;
  Layout L;
  char *ws = nullptr;
  int cur = 0;
  long steps = 0;
  int tx = 32, ty = 8;
  int mode = MODE_TILE;
  int persistent = 0;
  int graph_block = 0;
  std::vector<WorkItem> work;
  std::vector<WorkItem> fwork;  // tiles of the field export
  std::vector<int> fwork_off, fwork_n;
  std::vector<WorkItem> awork;  // tiles of the adjoint over the extended grids
  std::vector<FillNode> hfill;  // host copy of the fill records (all domains)
  std::vector<IbbNode> hibb;    // host copy of the interpolated-bounce-back records
  std::vector<TileIbb> tibb;    // their tile entries for the current work list (tiles only)
  std::vector<uint8_t> hflags;  // host copy of the flag planes
  struct Params {
    double theta_deg[2], sigma[3];
  };
  std::vector<Params> params;  // the public wetting/tension parameters of each domain
  bool adjoint = false;
  hipGraphExec_t graph = nullptr;
  bool graph_valid = false;
  long graph_launches = 0;  // hipGraph replays so far
  std::string err;

  template <typename P>
  P *at(size_t off) const { return reinterpret_cast<P *>(ws + off); }
  CandRangeCache cand_ranges;  // lbm3_set_params: fill candidates' angle ranges, by surroundings and angles
};

namespace {

lbm3_status hip_fail(lbm3_ctx *c, hipError_t e, const char *what) {
  if (c) {
    char b[256];
    snprintf(b, sizeof b, "%s: %s", what, hipGetErrorString(e));
    c->err = b;
  }
  return LBM3_EHIP;
}

#define HIPC(c, call)                                      \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return hip_fail(c, e_, #call);   \
  } while (0)

// The kind bits of a work item (see WorkItem): whether its 3-ring halo needs no index mapping and
// whether its tile + 1 ring streams by plain pulls.
int32_t work_kind(const lbm3_ctx *c, const WorkItem &w) {
  const DomainDev &D = c->doms[w.dom];
  int32_t k = 0;
  if (w.x0 - 3 >= 0 && w.x1 + 3 <= D.nx && w.y0 - 3 >= 0 && w.y1 + 3 <= D.ny) k |= WK_INNER;
  bool plain = !(D.bcx != BCX_PERIODIC && (w.x0 == 0 || w.x1 == D.nx));
  const uint8_t *fl = c->hflags.data() + D.base;
  for (int y = w.y0 - 1; plain && y < w.y1 + 1; ++y)
    for (int x = w.x0 - 1; plain && x < w.x1 + 1; ++x) {
      int i = x, j = y;
      if (D.bcx == BCX_ZOUHE) i = std::min(std::max(i, 0), D.nx - 1);
      else i = ((i % D.nx) + D.nx) % D.nx;
      if (D.yper) j = ((j % D.ny) + D.ny) % D.ny;
      else j = std::min(std::max(j, -2), D.ny + 1);
      if (fl[plane_index(i, j, D.pitch)] & FL_SOLID) plain = false;
    }
  if (plain) k |= WK_PLAIN;
  return k;
}

void build_work_for(lbm3_ctx *c, int mode, int tx, int ty, std::vector<WorkItem> &work,
                    std::vector<int> *offs, std::vector<int> *counts) {
  work.clear();
  if (offs) offs->assign(c->n, 0);
  if (counts) counts->assign(c->n, 0);
  for (int d = 0; d < c->n; ++d) {
    DomainDev &D = c->doms[d];
    const int off = (int)work.size();
    if (is_tile_mode(mode)) {
      for (int y = 0; y < D.ny; y += ty)
        for (int x = 0; x < D.nx; x += tx)
          work.push_back(WorkItem{d, x, y, std::min(x + tx, D.nx), std::min(y + ty, D.ny), 0, 0, 0});
    } else {
      const int W = (mode == MODE_STRIP128 ? 128 : 256) - 6;
      const int ns = (D.nx + W - 1) / W;
      const int wd = (D.nx + ns - 1) / ns;
      for (int y = 0; y < D.ny; y += ty)
        for (int x = 0; x < D.nx; x += wd)
          work.push_back(WorkItem{d, x, y, std::min(x + wd, D.nx), std::min(y + ty, D.ny), 0, 0, 0});
    }
    if (offs) (*offs)[d] = off;
    if (counts) (*counts)[d] = (int)work.size() - off;
  }
  for (WorkItem &w : work) w.kind = work_kind(c, w);
}

// Work list of the fused step kernel (tiles or strips), with the curved-node entries of tiles.
// The field export always uses the tile kernel with its own tile list (built once at creation).
void build_work(lbm3_ctx *c) {
  std::vector<int> offs, counts;
  build_work_for(c, c->mode, c->tx, c->ty, c->work, &offs, &counts);
  c->tibb.clear();
  if (is_tile_mode(c->mode)) {  // each curved node in the list of the tile that contains it
    std::vector<std::vector<TileIbb>> per(c->work.size());
    for (int d = 0; d < c->n; ++d) {
      const DomainDev &D = c->doms[d];
      const int nbx = (D.nx + c->tx - 1) / c->tx;
      for (int r = D.ibb_off; r < D.ibb_off + D.n_ibb; ++r) {
        const int i = c->hibb[r].li % D.pitch, j = c->hibb[r].li / D.pitch - 2;
        const int t = offs[d] + (j / c->ty) * nbx + i / c->tx;
        const WorkItem &w = c->work[t];
        per[t].push_back(TileIbb{(i - w.x0) + (j - w.y0) * c->tx, r});
      }
    }
    for (size_t t = 0; t < per.size(); ++t) {
      c->work[t].ibb_begin = (int32_t)c->tibb.size();
      c->work[t].ibb_count = (int32_t)per[t].size();
      c->tibb.insert(c->tibb.end(), per[t].begin(), per[t].end());
    }
  }
}

// Tiles of the adjoint kernels over each domain's extended range: columns -1..nx with a Zou-He
// x boundary (its ghost columns carry a stress), rows -2..ny+1 with a non-periodic y axis.
void build_adjoint_work(lbm3_ctx *c) {
  c->awork.clear();
  for (int d = 0; d < c->n; ++d) {
    const DomainDev &D = c->doms[d];
    const int x0 = D.bcx == BCX_ZOUHE ? -1 : 0, x1 = D.bcx == BCX_ZOUHE ? D.nx + 1 : D.nx;
    const int y0 = D.yper ? 0 : -2, y1 = D.yper ? D.ny : D.ny + 2;
    for (int y = y0; y < y1; y += kAdjTileY)
      for (int x = x0; x < x1; x += kAdjTileX)
        c->awork.push_back(WorkItem{d, x, y, std::min(x + kAdjTileX, x1), std::min(y + kAdjTileY, y1), 0, 0, 0});
  }
}

lbm3_status upload_tables(lbm3_ctx *c) {
  for (std::vector<WorkItem> *v : {&c->work, &c->fwork, &c->awork})
    for (WorkItem &w : *v) {
      const DomainDev &D = c->doms[w.dom];
      w.pitch = D.pitch;
      w.base = D.base;
      w.plane = D.plane;
    }
  if (!c->tibb.empty())
    HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_tibb), c->tibb.data(), sizeof(TileIbb) * c->tibb.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_doms), c->doms.data(), sizeof(DomainDev) * c->n, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_work), c->work.data(), sizeof(WorkItem) * c->work.size(), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_fwork), c->fwork.data(), sizeof(WorkItem) * c->fwork.size(), hipMemcpyHostToDevice, c->stream));
  if (c->adjoint && !c->awork.empty())
    HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_awork), c->awork.data(), sizeof(WorkItem) * c->awork.size(), hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return LBM3_OK;
}

template <typename S, typename T>
StepArgs<S, T> step_args(lbm3_ctx *c, int from) {
  StepArgs<S, T> a;
  a.doms = c->at<DomainDev>(c->L.off_doms);
  a.work = c->at<WorkItem>(c->L.off_work);
  a.work_begin = 0;
  a.work_end = (int)c->work.size();
  a.flags = c->at<uint8_t>(c->L.off_flags);
  a.ibb = c->at<IbbNode>(c->L.off_ibb);
  a.fillC = c->at<T>(c->L.off_fillC);
  a.tibb = c->at<TileIbb>(c->L.off_tibb);
  a.remap = 0;
  a.fin = c->at<S>(c->L.off_F[from]);
  a.rin = c->at<T>(c->L.off_R[from]);
  a.fout = c->at<S>(c->L.off_F[1 - from]);
  a.rout = c->at<T>(c->L.off_R[1 - from]);
  a.tile_x = c->tx;
  a.tile_y = c->ty;
  a.eps_g = T(kEpsG);
  a.out_rho = a.out_u = a.out_force = nullptr;
  a.adj_X = nullptr;
  a.adj_plane = 0;
  return a;
}

template <typename T>
FillArgs<T> fill_args(lbm3_ctx *c, int which) {
  FillArgs<T> f;
  f.fill = c->at<FillNode>(c->L.off_fill);
  f.n_fill = c->L.n_fill;
  f.blocks = c->at<FillBlock>(c->L.off_fblk);
  f.n_blocks = c->L.n_fblk;
  f.far = c->at<uint32_t>(c->L.off_far);
  f.cand = c->at<FillCand>(c->L.off_cand);
  f.doms = c->at<DomainDev>(c->L.off_doms);
  f.flags = c->at<uint8_t>(c->L.off_flags);
  f.rho = c->at<T>(c->L.off_R[which]);
  f.fillC = c->at<T>(c->L.off_fillC);
  return f;
}

// ev (optional): 3 events per step around the fill and the fused kernel.
template <typename S, typename T>
lbm3_status enqueue_steps_t(lbm3_ctx *c, int nsteps, hipStream_t s, hipEvent_t *ev) {
  const int nw = (int)c->work.size();
  const bool persistent = c->persistent > 0;
  const int grid = persistent ? std::min(c->persistent, nw) : round_up(nw, 8);
  for (int k = 0; k < nsteps; ++k) {
    StepArgs<S, T> a = step_args<S, T>(c, c->cur);
    a.remap = persistent ? 0 : 1;
    if (ev) HIPC(c, hipEventRecord(ev[3 * k], s));
    HIPC(c, launch_fill<T>(fill_args<T>(c, c->cur), s));
    if (ev) HIPC(c, hipEventRecord(ev[3 * k + 1], s));
    HIPC(c, (launch_step<S, T>(a, grid, c->mode, OUT_STEP, s)));
    if (ev) HIPC(c, hipEventRecord(ev[3 * k + 2], s));
    c->cur = 1 - c->cur;
  }
  return LBM3_OK;
}

lbm3_status enqueue_steps(lbm3_ctx *c, int nsteps, hipStream_t s, hipEvent_t *ev = nullptr) {
  switch (c->precision) {
    case LBM3_F64: return enqueue_steps_t<double, double>(c, nsteps, s, ev);
    case LBM3_F32: return enqueue_steps_t<float, float>(c, nsteps, s, ev);
    default: return enqueue_steps_t<__half, float>(c, nsteps, s, ev);
  }
}

lbm3_status build_graph(lbm3_ctx *c) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  const int saved = c->cur;
  hipGraph_t g = nullptr;
  HIPC(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  lbm3_status st = enqueue_steps(c, c->graph_block, c->cap_stream);
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  c->cur = saved;
  if (st != LBM3_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  c->graph_valid = true;
  return LBM3_OK;
}

template <typename S, typename T>
void init_state(const lbm3_domain *d, int n, const std::vector<DomHost> &H, int64_t total,
                std::vector<unsigned char> &Fh, std::vector<unsigned char> &Rh) {
  Fh.assign(9 * (size_t)total * sizeof(S), 0);
  Rh.assign(3 * (size_t)total * sizeof(T), 0);
  S *F = reinterpret_cast<S *>(Fh.data());
  T *R = reinterpret_cast<T *>(Rh.data());
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  for (int dd = 0; dd < n; ++dd) {
    const DomainDev &D = H[dd].dd;
    const size_t np = (size_t)d[dd].nx * d[dd].ny;
    for (int j = 0; j < D.ny; ++j)
      for (int i = 0; i < D.nx; ++i) {
        const int64_t li = plane_index(i, j, D.pitch);
        if (H[dd].flags[li] & FL_SOLID) continue;
        const size_t src = (size_t)j * D.nx + i;
        const double r0 = d[dd].rho_init[src], r1 = d[dd].rho_init[np + src], r2 = d[dd].rho_init[2 * np + src];
        const double rho = r0 + r1 + r2;
        for (int a = 0; a < 9; ++a) {
          const double v = (rho - 1.0) * w[a];  // shifted f = rho w_a - w_a at rest
          if constexpr (sizeof(S) == 2) F[9 * D.base + a * D.plane + li] = __float2half_rn((float)v);
          else F[9 * D.base + a * D.plane + li] = (S)v;
        }
        R[3 * D.base + li] = (T)r0;
        R[3 * D.base + D.plane + li] = (T)r1;
        R[3 * D.base + 2 * D.plane + li] = (T)r2;
      }
    // The first density slot of a fill node holds the index of its FillNode record; the filled
    // C of each step lives in the compact fillC array.
    for (size_t p = 0; p < H[dd].fill.size(); ++p) {
      const int idx = D.fill_off + (int)p;
      T v;
      if constexpr (sizeof(T) == 4) {
        int32_t bits = idx;
        memcpy(&v, &bits, 4);
      } else {
        int64_t bits = idx;
        memcpy(&v, &bits, 8);
      }
      R[3 * D.base + H[dd].fill[p].li] = v;
    }
  }
}

template <typename S, typename T>
lbm3_status fields_t(lbm3_ctx *c, int dom, void *rho, void *u, void *force) {
  HIPC(c, launch_fill<T>(fill_args<T>(c, c->cur), c->stream));
  StepArgs<S, T> a = step_args<S, T>(c, c->cur);
  a.work = c->at<WorkItem>(c->L.off_fwork);
  a.work_begin = c->fwork_off[dom];
  a.work_end = c->fwork_off[dom] + c->fwork_n[dom];
  a.tile_x = kFieldTileX;
  a.tile_y = kFieldTileY;
  a.out_rho = reinterpret_cast<T *>(rho);
  a.out_u = reinterpret_cast<T *>(u);
  a.out_force = reinterpret_cast<T *>(force);
  HIPC(c, (launch_step<S, T>(a, c->fwork_n[dom], MODE_TILE, OUT_FIELDS, c->stream)));
  return LBM3_OK;
}

template <typename S, typename T>
lbm3_status adjoint_step_t(lbm3_ctx *c, const void *state, const void *lin, void *lout) {
  const size_t fb = 9 * (size_t)c->L.total_plane * sizeof(S);
  const S *fin = reinterpret_cast<const S *>(state);
  const T *rin = reinterpret_cast<const T *>(reinterpret_cast<const char *>(state) + fb);
  FillArgs<T> f = fill_args<T>(c, 0);
  f.rho = rin;
  HIPC(c, launch_fill<T>(f, c->stream));
  {  // forward intermediates of s_t on the adjoint's tiles
    StepArgs<S, T> sa = step_args<S, T>(c, 0);
    sa.work = c->at<WorkItem>(c->L.off_awork);
    sa.work_begin = 0;
    sa.work_end = (int)c->awork.size();
    sa.remap = 1;
    sa.fin = fin;
    sa.rin = rin;
    sa.fout = nullptr;
    sa.rout = nullptr;
    sa.tile_x = kAdjTileX;
    sa.tile_y = kAdjTileY;
    sa.adj_X = c->at<T>(c->L.off_aX);
    sa.adj_plane = c->L.aplane;
    HIPC(c, (launch_step<S, T>(sa, round_up(sa.work_end, 8), MODE_TILE, OUT_ADJ, c->stream)));
  }
  AdjArgs<S, T> a;
  a.doms = c->at<DomainDev>(c->L.off_doms);
  a.work = c->at<WorkItem>(c->L.off_awork);
  a.n_work = (int)c->awork.size();
  a.flags = c->at<uint8_t>(c->L.off_flags);
  a.ibb = c->at<IbbNode>(c->L.off_ibb);
  a.ibb_of = c->at<int32_t>(c->L.off_ibbof);
  a.far = c->at<uint32_t>(c->L.off_far);
  a.links = c->at<uint32_t>(c->L.off_links);
  a.fill = c->at<FillNode>(c->L.off_fill);
  a.n_fill = c->L.n_fill;
  a.fillC = c->at<T>(c->L.off_fillC);
  a.fin = fin;
  a.rin = rin;
  a.X = c->at<T>(c->L.off_aX);
  a.aplane = c->L.aplane;
  a.lin = reinterpret_cast<const T *>(lin);
  a.lout = reinterpret_cast<T *>(lout);
  a.raw = c->at<double>(c->L.off_raw);
  a.eps_g = T(kEpsG);
  a.eps_n = sizeof(T) == 8 ? T(kEpsG) : T(kEpsNormalAdjF32);
  HIPC(c, (launch_adjoint<S, T>(a, c->L.total_plane, c->stream)));
  return LBM3_OK;
}

// Back-to-back launches on the current state: n wetting fills, then n fused steps that all
// compute the same next state into the other buffer (the state does not advance).
template <typename S, typename T>
lbm3_status time_kernels_t(lbm3_ctx *c, int n, hipEvent_t ev[3]) {
  hipStream_t s = c->stream;
  const int nw = (int)c->work.size();
  const bool persistent = c->persistent > 0;
  const int grid = persistent ? std::min(c->persistent, nw) : round_up(nw, 8);
  StepArgs<S, T> a = step_args<S, T>(c, c->cur);
  a.remap = persistent ? 0 : 1;
  const FillArgs<T> f = fill_args<T>(c, c->cur);
  HIPC(c, launch_fill<T>(f, s));
  HIPC(c, hipEventRecord(ev[0], s));
  for (int k = 0; k < n; ++k) HIPC(c, launch_fill<T>(f, s));
  HIPC(c, hipEventRecord(ev[1], s));
  for (int k = 0; k < n; ++k) HIPC(c, (launch_step<S, T>(a, grid, c->mode, OUT_STEP, s)));
  HIPC(c, hipEventRecord(ev[2], s));
  return LBM3_OK;
}

// ---- autotuner cache --------------------------------------------------------------------
// A JSON object with one line per entry,
//   "<key>": {"kernel": K, "tile_x": X, "tile_y": Y, "ms_per_step": T},
// keyed by the device architecture, the precision and the domains' shapes and boundary types
// (their count, total nodes and an FNV-1a hash of nx, ny, y_periodic, bc_x, fill and curved-node
// counts of every domain).  The configurations compute identical results, so a stale entry can
// only cost time.
struct TuneEntry {
  std::string key;
  int kernel, tx, ty;
  double ms;
};

std::string tune_key(const lbm3_ctx *c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  int64_t nodes = 0;
  for (const DomainDev &D : c->doms) {
    mix(D.nx); mix(D.ny); mix(D.yper); mix(D.bcx); mix(D.n_fill); mix(D.n_ibb);
    nodes += (int64_t)D.nx * D.ny;
  }
  hipDeviceProp_t prop;
  const char *arch = hipGetDeviceProperties(&prop, c->device) == hipSuccess ? prop.gcnArchName : "unknown";
  std::string a(arch);
  const size_t colon = a.find(':');
  if (colon != std::string::npos) a = a.substr(0, colon);
  const char *prec = c->precision == LBM3_F64 ? "f64" : (c->precision == LBM3_F32 ? "f32" : "f32-f16store");
  char b[256];
  snprintf(b, sizeof b, "%s %s domains=%d nodes=%lld shapes=%016llx", a.c_str(), prec, c->n, (long long)nodes,
           (unsigned long long)h);
  return b;
}

std::vector<TuneEntry> read_tune_cache(const std::string &path) {
  std::vector<TuneEntry> out;
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return out;
  char line[1024];
  while (fgets(line, sizeof line, f)) {
    const char *q0 = strchr(line, '"');
    if (!q0) continue;
    const char *q1 = strchr(q0 + 1, '"');
    if (!q1) continue;
    TuneEntry e;
    e.key.assign(q0 + 1, q1);
    if (sscanf(q1 + 1, ": {\"kernel\": %d, \"tile_x\": %d, \"tile_y\": %d, \"ms_per_step\": %lf", &e.kernel, &e.tx,
               &e.ty, &e.ms) == 4)
      out.push_back(e);
  }
  fclose(f);
  return out;
}

bool write_tune_cache(const std::string &path, const TuneEntry &add) {
  std::vector<TuneEntry> entries = read_tune_cache(path);
  bool found = false;
  for (TuneEntry &e : entries)
    if (e.key == add.key) {
      e = add;
      found = true;
    }
  if (!found) entries.push_back(add);
  const std::string tmp = path + ".tmp";
  FILE *f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i)
    fprintf(f, "  \"%s\": {\"kernel\": %d, \"tile_x\": %d, \"tile_y\": %d, \"ms_per_step\": %.6g}%s\n",
            entries[i].key.c_str(), entries[i].kernel, entries[i].tx, entries[i].ty, entries[i].ms,
            i + 1 < entries.size() ? "," : "");
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

extern "C" {

const char *lbm3_status_string(int32_t code) {
  switch (code) {
    case LBM3_OK: return "ok";
    case LBM3_EINVAL: return "invalid argument";
    case LBM3_ENOMEM: return "out of memory / workspace too small";
    case LBM3_EHIP: return "HIP runtime error";
    case LBM3_ESTATE: return "invalid state";
    case LBM3_ENUMERIC: return "non-finite density";
    case LBM3_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char *lbm3_last_error(const lbm3_ctx *c) { return c ? c->err.c_str() : "null context"; }

static thread_local std::string g_plan_err;

lbm3_status lbm3_workspace_bytes(const lbm3_domain *d, int32_t n, const lbm3_options *o, size_t *bytes) {
  if (!bytes) return LBM3_EINVAL;
  std::vector<DomHost> H;
  Layout L;
  if (!plan(d, n, o, H, L, g_plan_err)) return LBM3_EINVAL;
  *bytes = L.total;
  return LBM3_OK;
}

lbm3_status lbm3_create(const lbm3_domain *d, int32_t n, const lbm3_options *o, void *dev_workspace,
                        size_t bytes, void *hip_stream, lbm3_ctx **out) {
  if (!out) return LBM3_EINVAL;
  *out = nullptr;
  std::vector<DomHost> H;
  Layout L;
  if (!plan(d, n, o, H, L, g_plan_err)) return LBM3_EINVAL;
  if (!dev_workspace || bytes < L.total) {
    g_plan_err = "workspace missing or smaller than lbm3_workspace_bytes";
    return LBM3_ENOMEM;
  }
  if ((reinterpret_cast<uintptr_t>(dev_workspace) & 255) != 0) {
    g_plan_err = "workspace must be 256-byte aligned";
    return LBM3_EINVAL;
  }
  lbm3_ctx *c = new lbm3_ctx();
  c->n = n;
  c->precision = o->precision;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->L = L;
  c->ws = reinterpret_cast<char *>(dev_workspace);
  c->graph_block = o->graph_block_steps > 0 ? round_up(o->graph_block_steps, 2) : 0;
  c->persistent = o->persistent_blocks;
  c->mode = o->kernel > 0 ? o->kernel : MODE_TILE;
  if (is_tile_mode(c->mode)) {  // default shapes: 32x8 (256 threads), 64x8 (512 threads)
    c->tx = o->tile_x > 0 ? o->tile_x : (c->mode == MODE_TILE512 ? 64 : 32);
    c->ty = o->tile_y > 0 ? o->tile_y : 8;
  } else {
    c->tx = 0;
    c->ty = o->tile_y > 0 ? o->tile_y : 64;
  }
  for (auto &h : H) c->doms.push_back(h.dd);
  for (int i = 0; i < n; ++i)
    c->params.push_back({{d[i].theta_deg[0], d[i].theta_deg[1]}, {d[i].sigma[0], d[i].sigma[1], d[i].sigma[2]}});
  c->adjoint = o->adjoint == 1;
  if (c->adjoint) build_adjoint_work(c);
  auto bail = [&](lbm3_status s) {
    g_plan_err = c->err;
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return s;
  };
  hipError_t e = init_kernel_attributes();
  if (e != hipSuccess) return bail(hip_fail(c, e, "hipFuncSetAttribute"));
  e = hipGetDevice(&c->device);
  if (e != hipSuccess) return bail(hip_fail(c, e, "hipGetDevice"));
  e = mass_scratch_init(c->device, &c->mass_scratch);  // once per device, with it current
  if (e != hipSuccess) return bail(hip_fail(c, e, "hipGetSymbolAddress(scratch)"));
  if (o->tune_cache) c->tune_cache = o->tune_cache;
  e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(hip_fail(c, e, "hipStreamCreateWithFlags"));
  c->hflags.assign((size_t)L.total_plane, 0);
  for (int i = 0; i < n; ++i) memcpy(c->hflags.data() + H[i].dd.base, H[i].flags.data(), H[i].flags.size());
  for (int i = 0; i < n; ++i) c->hfill.insert(c->hfill.end(), H[i].fill.begin(), H[i].fill.end());
  for (int i = 0; i < n; ++i) c->hibb.insert(c->hibb.end(), H[i].ibb.begin(), H[i].ibb.end());
  build_work(c);
  build_work_for(c, MODE_TILE, kFieldTileX, kFieldTileY, c->fwork, &c->fwork_off, &c->fwork_n);
  // chunk tables of the mass reduction
  std::vector<int> chunk_dom, chunk_first;
  for (int i = 0; i < n; ++i) {
    chunk_first.push_back((int)chunk_dom.size());
    for (int j = 0; j < d[i].ny; j += 16) chunk_dom.push_back(i);
  }
  chunk_first.push_back((int)chunk_dom.size());
  const std::vector<FillNode> &fill = c->hfill;
  const std::vector<IbbNode> &ibb = c->hibb;
  const std::vector<uint8_t> &flags = c->hflags;
  std::vector<unsigned char> Fh, Rh;
  if (c->precision == LBM3_F64) init_state<double, double>(d, n, H, L.total_plane, Fh, Rh);
  else if (c->precision == LBM3_F32) init_state<float, float>(d, n, H, L.total_plane, Fh, Rh);
  else init_state<__half, float>(d, n, H, L.total_plane, Fh, Rh);
  hipStream_t s = c->stream;
#define CK(call)                                              \
  do {                                                        \
    hipError_t e2 = (call);                                   \
    if (e2 != hipSuccess) return bail(hip_fail(c, e2, #call)); \
  } while (0)
  for (int b = 0; b < 2; ++b) {  // both buffers: solid slots are never written by the step
    CK(hipMemcpyAsync(c->at<void>(L.off_F[b]), Fh.data(), Fh.size(), hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(c->at<void>(L.off_R[b]), Rh.data(), Rh.size(), hipMemcpyHostToDevice, s));
  }
  CK(hipMemcpyAsync(c->at<void>(L.off_flags), flags.data(), flags.size(), hipMemcpyHostToDevice, s));
  if (!fill.empty()) CK(hipMemcpyAsync(c->at<void>(L.off_fill), fill.data(), sizeof(FillNode) * fill.size(), hipMemcpyHostToDevice, s));
  if (!ibb.empty()) CK(hipMemcpyAsync(c->at<void>(L.off_ibb), ibb.data(), sizeof(IbbNode) * ibb.size(), hipMemcpyHostToDevice, s));
  {
    std::vector<uint32_t> far;  // far fluid masks of all fill nodes, in fill order
    for (int i = 0; i < n; ++i) far.insert(far.end(), H[i].far.begin(), H[i].far.end());
    if (!far.empty())
      CK(hipMemcpyAsync(c->at<void>(L.off_far), far.data(), sizeof(uint32_t) * far.size(), hipMemcpyHostToDevice, s));
    std::vector<FillCand> cand;  // candidate crossings of all fill nodes, in fill order
    for (int i = 0; i < n; ++i) cand.insert(cand.end(), H[i].cand.begin(), H[i].cand.end());
    if (!cand.empty())
      CK(hipMemcpyAsync(c->at<void>(L.off_cand), cand.data(), sizeof(FillCand) * cand.size(), hipMemcpyHostToDevice, s));
    CK(hipStreamSynchronize(s));
  }
  std::vector<FillBlock> fblk;  // work-groups of the fill kernel: up to kFillNodes nodes of one domain
  for (int i = 0; i < n; ++i)
    for (int f0 = 0; f0 < H[i].dd.n_fill; f0 += kFillNodes)
      fblk.push_back(FillBlock{i, H[i].dd.fill_off + f0, std::min(kFillNodes, H[i].dd.n_fill - f0), 0});
  if (!fblk.empty())
    CK(hipMemcpyAsync(c->at<void>(L.off_fblk), fblk.data(), sizeof(FillBlock) * fblk.size(), hipMemcpyHostToDevice, s));
  std::vector<int32_t> ibb_of;  // adjoint only: index of each node's link record (-1: none)
  if (c->adjoint) {
    ibb_of.assign((size_t)L.total_plane, -1);
    for (int i = 0; i < n; ++i)
      for (int r = 0; r < H[i].dd.n_ibb; ++r) ibb_of[(size_t)(H[i].dd.base + ibb[H[i].dd.ibb_off + r].li)] = H[i].dd.ibb_off + r;
    CK(hipMemcpyAsync(c->at<void>(L.off_ibbof), ibb_of.data(), sizeof(int32_t) * ibb_of.size(), hipMemcpyHostToDevice, s));
  }
  std::vector<uint32_t> links;  // adjoint only: the link bits of every fluid node (AdjArgs::links)
  if (c->adjoint) {
    links.assign((size_t)L.total_plane, 0u);
    for (int dd = 0; dd < n; ++dd) {
      const DomainDev &D = H[dd].dd;
      const uint8_t *fl = H[dd].flags.data();
      auto mapped = [&](int i, int j) -> uint8_t {  // flags of the node a read at (i, j) sees
        i = D.bcx == BCX_ZOUHE ? std::min(std::max(i, 0), D.nx - 1) : ((i % D.nx) + D.nx) % D.nx;
        j = D.yper ? ((j % D.ny) + D.ny) % D.ny : std::min(std::max(j, -2), D.ny + 1);
        return fl[plane_index(i, j, D.pitch)];
      };
      for (int j = 0; j < D.ny; ++j)
        for (int i = 0; i < D.nx; ++i) {
          const int64_t li = plane_index(i, j, D.pitch);
          if (fl[li] & FL_SOLID) continue;
          uint32_t b = (fl[li] & FL_CURVED) ? (1u << 27) : 0u;
          for (int d = 0; d < 9; ++d) {
            const uint8_t f1 = mapped(i + kEX[d], j + kEY[d]), f2 = mapped(i + 2 * kEX[d], j + 2 * kEY[d]);
            if (f1 & FL_SOLID) b |= 1u << d;
            if (f1 & FL_CURVED) b |= 1u << (9 + d);
            if (f2 & FL_SOLID) b |= 1u << (18 + d);
          }
          links[(size_t)(D.base + li)] = b;
        }
    }
    CK(hipMemcpyAsync(c->at<void>(L.off_links), links.data(), sizeof(uint32_t) * links.size(), hipMemcpyHostToDevice, s));
  }
  CK(hipMemcpyAsync(c->at<void>(L.off_chunk_dom), chunk_dom.data(), sizeof(int) * chunk_dom.size(), hipMemcpyHostToDevice, s));
  CK(hipMemcpyAsync(c->at<void>(L.off_chunk_first), chunk_first.data(), sizeof(int) * chunk_first.size(), hipMemcpyHostToDevice, s));
  std::vector<int> lfirst;  // adjoint only: first field tile of each domain (loss partials)
  if (c->adjoint) {
    for (int i = 0; i < n; ++i) lfirst.push_back(c->fwork_off[i]);
    lfirst.push_back((int)c->fwork.size());
    CK(hipMemcpyAsync(c->at<void>(L.off_lfirst), lfirst.data(), sizeof(int) * lfirst.size(), hipMemcpyHostToDevice, s));
  }
  CK(hipMemsetAsync(c->at<void>(L.off_bad), 0, sizeof(int), s));
#undef CK
  lbm3_status st = upload_tables(c);  // synchronises the stream
  if (st != LBM3_OK) return bail(st);
  *out = c;
  return LBM3_OK;
}

lbm3_status lbm3_step(lbm3_ctx *c, int32_t nsteps) {
  if (!c) return LBM3_EINVAL;
  if (nsteps < 0) {
    c->err = "nsteps must be >= 0";
    return LBM3_EINVAL;
  }
  int left = nsteps;
  if (c->graph_block > 0 && left >= c->graph_block) {
    if (c->cur == 1) {
      lbm3_status st = enqueue_steps(c, 1, c->stream);
      if (st != LBM3_OK) return st;
      --left;
    }
    if (!c->graph_valid) {
      lbm3_status st = build_graph(c);
      if (st != LBM3_OK) return st;
    }
    while (left >= c->graph_block) {
      HIPC(c, hipGraphLaunch(c->graph, c->stream));
      left -= c->graph_block;
      ++c->graph_launches;
    }
  }
  lbm3_status st = enqueue_steps(c, left, c->stream);
  if (st != LBM3_OK) return st;
  c->steps += nsteps;
  return LBM3_OK;
}

lbm3_status lbm3_fields(lbm3_ctx *c, int32_t domain, void *dev_rho, void *dev_u, void *dev_force, int32_t dtype) {
  if (!c) return LBM3_EINVAL;
  if (domain < 0 || domain >= c->n || !dev_rho) {
    c->err = "bad domain index or missing density buffer";
    return LBM3_EINVAL;
  }
  const int want = c->precision == LBM3_F64 ? LBM3_F64 : LBM3_F32;
  if (dtype != want) {
    c->err = "fields are written in the compute type (LBM3_F64 for FP64 contexts, LBM3_F32 otherwise)";
    return LBM3_EUNSUPPORTED;
  }
  switch (c->precision) {
    case LBM3_F64: return fields_t<double, double>(c, domain, dev_rho, dev_u, dev_force);
    case LBM3_F32: return fields_t<float, float>(c, domain, dev_rho, dev_u, dev_force);
    default: return fields_t<__half, float>(c, domain, dev_rho, dev_u, dev_force);
  }
}

lbm3_status lbm3_mass(lbm3_ctx *c, double *host_out) {
  if (!c || !host_out) return LBM3_EINVAL;
  HIPC(c, hipMemsetAsync(c->at<void>(c->L.off_bad), 0, sizeof(int), c->stream));
  double *out = c->at<double>(c->L.off_mass);
  if (c->precision == LBM3_F64) {
    MassArgs<double> a{c->at<DomainDev>(c->L.off_doms), c->at<uint8_t>(c->L.off_flags), c->at<double>(c->L.off_R[c->cur]),
                       c->at<int>(c->L.off_chunk_dom), c->at<int>(c->L.off_chunk_first), c->at<double>(c->L.off_partial),
                       c->at<int>(c->L.off_bad)};
    HIPC(c, launch_mass<double>(a, c->L.n_chunks, c->n, out, c->stream));
  } else {
    MassArgs<float> a{c->at<DomainDev>(c->L.off_doms), c->at<uint8_t>(c->L.off_flags), c->at<float>(c->L.off_R[c->cur]),
                      c->at<int>(c->L.off_chunk_dom), c->at<int>(c->L.off_chunk_first), c->at<double>(c->L.off_partial),
                      c->at<int>(c->L.off_bad)};
    HIPC(c, launch_mass<float>(a, c->L.n_chunks, c->n, out, c->stream));
  }
  int bad = 0;
  HIPC(c, hipMemcpyAsync(host_out, out, sizeof(double) * 3 * c->n, hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipMemcpyAsync(&bad, c->at<void>(c->L.off_bad), sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  if (bad) {
    c->err = "non-finite partial density found";
    return LBM3_ENUMERIC;
  }
  return LBM3_OK;
}

lbm3_status lbm3_mass_device(lbm3_ctx *c, double *dev_out) {
  if (!c || !dev_out) return LBM3_EINVAL;
  if (c->L.n_chunks > kMassScratchChunks) {
    char b[200];
    snprintf(b, sizeof b, "lbm3_mass_device: %d row chunks exceed the fixed scratch of %d (sum over domains of "
             "ceil(ny / 16)); use lbm3_mass", c->L.n_chunks, kMassScratchChunks);
    c->err = b;
    return LBM3_EINVAL;
  }
  if (c->precision == LBM3_F64) {
    MassArgs<double> a{c->at<DomainDev>(c->L.off_doms), c->at<uint8_t>(c->L.off_flags), c->at<double>(c->L.off_R[c->cur]),
                       c->at<int>(c->L.off_chunk_dom), c->at<int>(c->L.off_chunk_first), c->mass_scratch, nullptr};
    HIPC(c, launch_mass<double>(a, c->L.n_chunks, c->n, dev_out, c->stream));
  } else {
    MassArgs<float> a{c->at<DomainDev>(c->L.off_doms), c->at<uint8_t>(c->L.off_flags), c->at<float>(c->L.off_R[c->cur]),
                      c->at<int>(c->L.off_chunk_dom), c->at<int>(c->L.off_chunk_first), c->mass_scratch, nullptr};
    HIPC(c, launch_mass<float>(a, c->L.n_chunks, c->n, dev_out, c->stream));
  }
  return LBM3_OK;
}

lbm3_status lbm3_state_bytes(const lbm3_ctx *c, size_t *bytes) {
  if (!c || !bytes) return LBM3_EINVAL;
  *bytes = 9 * (size_t)c->L.total_plane * s_size(c->precision) + 3 * (size_t)c->L.total_plane * t_size(c->precision);
  return LBM3_OK;
}

lbm3_status lbm3_get_state(lbm3_ctx *c, void *dev_dst) {
  if (!c || !dev_dst) return LBM3_EINVAL;
  const size_t fb = 9 * (size_t)c->L.total_plane * s_size(c->precision);
  const size_t rb = 3 * (size_t)c->L.total_plane * t_size(c->precision);
  char *d = reinterpret_cast<char *>(dev_dst);
  HIPC(c, hipMemcpyAsync(d, c->at<void>(c->L.off_F[c->cur]), fb, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(d + fb, c->at<void>(c->L.off_R[c->cur]), rb, hipMemcpyDeviceToDevice, c->stream));
  return LBM3_OK;
}

lbm3_status lbm3_set_state(lbm3_ctx *c, const void *dev_src) {
  if (!c || !dev_src) return LBM3_EINVAL;
  const size_t fb = 9 * (size_t)c->L.total_plane * s_size(c->precision);
  const size_t rb = 3 * (size_t)c->L.total_plane * t_size(c->precision);
  const char *s = reinterpret_cast<const char *>(dev_src);
  HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_F[c->cur]), s, fb, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(c->at<void>(c->L.off_R[c->cur]), s + fb, rb, hipMemcpyDeviceToDevice, c->stream));
  return LBM3_OK;
}

lbm3_status lbm3_set_params(lbm3_ctx *c, int32_t domain, const double *theta_deg, const double *sigma) {
  if (!c) return LBM3_EINVAL;
  if (domain < 0 || domain >= c->n || !theta_deg || !sigma) {
    c->err = "bad domain index or missing parameters";
    return LBM3_EINVAL;
  }
  DomainDev D = c->doms[domain];
  const char *m = derive_params(theta_deg, sigma, D);
  if (m) {
    c->err = m;
    return LBM3_EINVAL;
  }
  c->doms[domain] = D;
  c->params[domain] = {{theta_deg[0], theta_deg[1]}, {sigma[0], sigma[1], sigma[2]}};
  HIPC(c, hipMemcpyAsync(c->at<DomainDev>(c->L.off_doms) + domain, &c->doms[domain], sizeof(DomainDev),
                         hipMemcpyHostToDevice, c->stream));
  // the fill's candidate crossings follow the angles
  std::vector<FillCand> cand(4 * kFillCands * (size_t)std::max(D.n_fill, 1));
  // (kept across calls: a set of angles seen before finds its ranges; bounded at ~30 MB)
  if (c->cand_ranges.map.size() > 65536) c->cand_ranges.map.clear();
  for (int p = 0; p < D.n_fill; ++p)
    fill_candidates(D, c->hflags.data() + D.base, c->hfill[D.fill_off + p], cand.data() + 4 * kFillCands * (size_t)p,
                    &c->cand_ranges);
  if (D.n_fill > 0)
    HIPC(c, hipMemcpyAsync(c->at<FillCand>(c->L.off_cand) + 4 * kFillCands * (size_t)D.fill_off, cand.data(),
                           sizeof(FillCand) * 4 * kFillCands * D.n_fill, hipMemcpyHostToDevice, c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  return LBM3_OK;
}

static lbm3_status adjoint_ready(lbm3_ctx *c) {
  if (!c) return LBM3_EINVAL;
  if (!c->adjoint) {
    c->err = "the context was created without options.adjoint = 1";
    return LBM3_ESTATE;
  }
  return LBM3_OK;
}

lbm3_status lbm3_adjoint_seed(lbm3_ctx *c, const double *dev_grad_rho, void *dev_lambda) {
  lbm3_status st = adjoint_ready(c);
  if (st != LBM3_OK) return st;
  if (!dev_grad_rho || !dev_lambda) {
    c->err = "missing buffer";
    return LBM3_EINVAL;
  }
  size_t bytes = 0;
  (void)lbm3_state_bytes(c, &bytes);
  HIPC(c, hipMemsetAsync(dev_lambda, 0, bytes, c->stream));
  HIPC(c, hipMemsetAsync(c->at<void>(c->L.off_raw), 0, sizeof(double) * 9 * c->n, c->stream));
  const DomainDev *doms = c->at<DomainDev>(c->L.off_doms);
  const WorkItem *w = c->at<WorkItem>(c->L.off_fwork);
  const uint8_t *fl = c->at<uint8_t>(c->L.off_flags);
  const int nw = (int)c->fwork.size();
  if (c->precision == LBM3_F64)
    HIPC(c, launch_adjoint_seed<double>(doms, w, nw, fl, dev_grad_rho, reinterpret_cast<double *>(dev_lambda),
                                        c->L.total_plane, c->stream));
  else
    HIPC(c, launch_adjoint_seed<float>(doms, w, nw, fl, dev_grad_rho, reinterpret_cast<float *>(dev_lambda),
                                       c->L.total_plane, c->stream));
  return LBM3_OK;
}

lbm3_status lbm3_loss_seed(lbm3_ctx *c, const double *dev_target_C, void *dev_adj, double *dev_loss) {
  lbm3_status st = adjoint_ready(c);
  if (st != LBM3_OK) return st;
  if (!dev_target_C || !dev_adj || !dev_loss) {
    c->err = "missing buffer";
    return LBM3_EINVAL;
  }
  size_t bytes = 0;
  (void)lbm3_state_bytes(c, &bytes);
  HIPC(c, hipMemsetAsync(dev_adj, 0, bytes, c->stream));
  HIPC(c, hipMemsetAsync(c->at<void>(c->L.off_raw), 0, sizeof(double) * 9 * c->n, c->stream));
  const DomainDev *doms = c->at<DomainDev>(c->L.off_doms);
  const WorkItem *w = c->at<WorkItem>(c->L.off_fwork);
  const uint8_t *fl = c->at<uint8_t>(c->L.off_flags);
  const int *first = c->at<int>(c->L.off_lfirst);
  double *part = c->at<double>(c->L.off_lpart);
  const int nw = (int)c->fwork.size();
  if (c->precision == LBM3_F64)
    HIPC(c, launch_loss_seed<double>(doms, w, nw, first, c->n, fl, c->at<double>(c->L.off_R[c->cur]), c->L.total_plane,
                                     dev_target_C, reinterpret_cast<double *>(dev_adj), part, dev_loss, c->stream));
  else
    HIPC(c, launch_loss_seed<float>(doms, w, nw, first, c->n, fl, c->at<float>(c->L.off_R[c->cur]), c->L.total_plane,
                                    dev_target_C, reinterpret_cast<float *>(dev_adj), part, dev_loss, c->stream));
  return LBM3_OK;
}

lbm3_status lbm3_adjoint_step(lbm3_ctx *c, const void *dev_state, const void *dev_lambda_in, void *dev_lambda_out) {
  lbm3_status st = adjoint_ready(c);
  if (st != LBM3_OK) return st;
  if (!dev_state || !dev_lambda_in || !dev_lambda_out || dev_lambda_in == dev_lambda_out) {
    c->err = "missing buffer, or lambda_in and lambda_out are the same buffer";
    return LBM3_EINVAL;
  }
  if (c->precision == LBM3_F64) return adjoint_step_t<double, double>(c, dev_state, dev_lambda_in, dev_lambda_out);
  return adjoint_step_t<float, float>(c, dev_state, dev_lambda_in, dev_lambda_out);
}

lbm3_status lbm3_adjoint_grad(lbm3_ctx *c, double *host_grad) {
  lbm3_status st = adjoint_ready(c);
  if (st != LBM3_OK) return st;
  if (!host_grad) return LBM3_EINVAL;
  std::vector<double> raw(9 * (size_t)c->n);
  HIPC(c, hipMemcpyAsync(raw.data(), c->at<void>(c->L.off_raw), sizeof(double) * raw.size(), hipMemcpyDeviceToHost,
                         c->stream));
  HIPC(c, hipStreamSynchronize(c->stream));
  for (int d = 0; d < c->n; ++d) {
    double J[9][5];
    param_jacobian(c->params[d].theta_deg, c->params[d].sigma, J);
    for (int p = 0; p < 5; ++p) {
      double g = 0.0;
      for (int r = 0; r < 9; ++r) g += raw[9 * d + r] * J[r][p];
      host_grad[5 * d + p] = g;
    }
  }
  return LBM3_OK;
}

lbm3_status lbm3_kernel_times(lbm3_ctx *c, int32_t nsteps, double *ms_fill, double *ms_step) {
  if (!c || nsteps < 1 || !ms_step || !ms_fill) return LBM3_EINVAL;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (auto &e : ev) HIPC(c, hipEventCreate(&e));
  lbm3_status st;
  switch (c->precision) {
    case LBM3_F64: st = time_kernels_t<double, double>(c, nsteps, ev); break;
    case LBM3_F32: st = time_kernels_t<float, float>(c, nsteps, ev); break;
    default: st = time_kernels_t<__half, float>(c, nsteps, ev); break;
  }
  float a = 0, b = 0;
  if (st == LBM3_OK) {
    hipError_t e = hipEventSynchronize(ev[2]);
    if (e != hipSuccess) st = hip_fail(c, e, "hipEventSynchronize");
    (void)hipEventElapsedTime(&a, ev[0], ev[1]);
    (void)hipEventElapsedTime(&b, ev[1], ev[2]);
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  *ms_fill = a / nsteps;
  *ms_step = b / nsteps;
  return st;
}

lbm3_status lbm3_autotune(lbm3_ctx *c, int32_t steps_per_candidate, int32_t *choice) {
  if (!c || steps_per_candidate < 1) return LBM3_EINVAL;
  double best = 1e300;
  Candidate bc{c->mode, c->tx, c->ty};
  const std::string key = c->tune_cache.empty() ? std::string() : tune_key(c);
  bool cached = false;
  if (!key.empty()) {
    const std::vector<TuneEntry> entries = read_tune_cache(c->tune_cache);
    for (const TuneEntry &e : entries)
      if (e.key == key)
        for (const Candidate &t : kCands)
          if (t.kernel == e.kernel && t.tx == e.tx && t.ty == e.ty) {
            bc = t;
            cached = true;
          }
  }
  // Two rounds over the candidates, each candidate's best round counting: close configurations
  // (at small sizes within a few per cent) are then not picked by one noisy timing.
  constexpr int kRounds = 2;
  double cand_best[sizeof(kCands) / sizeof(kCands[0])];
  for (double &b : cand_best) b = 1e300;
  for (int round = 0; round < kRounds && !cached; ++round)
    for (size_t ci = 0; ci < sizeof(kCands) / sizeof(kCands[0]); ++ci) {
      const Candidate &t = kCands[ci];
      if (is_tile_mode(t.kernel) && step_smem_bytes(c->precision, t.kernel, t.tx, t.ty) > 160 * 1024) continue;
      if (!is_tile_mode(t.kernel) && step_smem_bytes(c->precision, t.kernel, 0, 0) > 160 * 1024) continue;
      c->mode = t.kernel;
      c->tx = t.tx;
      c->ty = t.ty;
      build_work(c);
      lbm3_status st = upload_tables(c);
      if (st != LBM3_OK) return st;
      st = enqueue_steps(c, 2, c->stream);  // warm-up
      if (st != LBM3_OK) return st;
      c->steps += 2;
      double mf, ms;
      st = lbm3_kernel_times(c, steps_per_candidate, &mf, &ms);
      if (st != LBM3_OK) return st;
      cand_best[ci] = std::min(cand_best[ci], mf + ms);  // the whole step: a separate fill kernel counts too
    }
  for (size_t ci = 0; ci < sizeof(kCands) / sizeof(kCands[0]) && !cached; ++ci)
    if (cand_best[ci] < best) {
      best = cand_best[ci];
      bc = kCands[ci];
    }
  c->mode = bc.kernel;
  c->tx = bc.tx;
  c->ty = bc.ty;
  build_work(c);
  c->graph_valid = false;
  lbm3_status st = upload_tables(c);
  if (st != LBM3_OK) return st;
  if (!key.empty() && !cached && !write_tune_cache(c->tune_cache, TuneEntry{key, bc.kernel, bc.tx, bc.ty, best})) {
    c->err = "lbm3_autotune: cannot write the tune cache " + c->tune_cache;
    return LBM3_EINVAL;
  }
  if (choice) {
    choice[0] = bc.kernel;
    choice[1] = bc.tx;
    choice[2] = bc.ty;
  }
  return LBM3_OK;
}

lbm3_status lbm3_query(const lbm3_ctx *c, int32_t key, double *value) {
  if (!c || !value) return LBM3_EINVAL;
  int64_t nodes = 0;
  for (const auto &D : c->doms) nodes += (int64_t)D.nx * D.ny;
  switch (key) {
    case 0: *value = 2.0 * (9.0 * s_size(c->precision) + 3.0 * t_size(c->precision)); break;
    case 1: *value = (double)nodes; break;
    case 2: *value = c->L.n_fill; break;
    case 3: *value = c->L.n_ibb; break;
    case 4: *value = c->tx; break;
    case 5: *value = c->ty; break;
    case 6: *value = (double)c->work.size(); break;
    case 7: *value = (double)c->steps; break;
    case 8: *value = c->mode; break;
    case 9: *value = (double)c->graph_launches; break;
    case 10: *value = c->graph_block; break;
    default: return LBM3_EINVAL;
  }
  return LBM3_OK;
}

const char *lbm3_plan_error(void) { return g_plan_err.c_str(); }

void lbm3_destroy(lbm3_ctx *c) {
  if (!c) return;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // extern "C"
