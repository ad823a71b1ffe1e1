// Host check of two device helpers of the wetting fill (compiled for the CPU from the product
// header): march_line_masked (11 x 11 near mask, then the 25 x 25 far mask, then the general march)
// must give exactly march_line's hit (same nodes, bit-identical weight)
// for random fluid fields and directions, including lattice and rational-slope directions that
// pass through nodes; sincos_quadrant must agree with long-double sin/cos to 1 ulp on the angle
// range of Eq. (22)'s lines, [0, 85] degrees; and a candidate's angle range (line_angle_range) must
// hold only angles at which the march started at the candidate's crossing counters gives the full
// march's hit.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "lbm3_internal.h"

using namespace lbm3;

static double ulps(double a, double b) { return std::fabs(a - b) / (std::nextafter(std::fabs(b), 1e300) - std::fabs(b)); }

int main(int argc, char **argv) {
  const long trials = argc > 1 ? std::atol(argv[1]) : 200000;
  std::mt19937_64 g(2102);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  static int fl[41][41];
  long bad = 0, hits = 0, ranges = 0, bad_range = 0;
  for (long trial = 0; trial < trials; ++trial) {
    const double p = 0.2 + 0.75 * U(g);
    const int shape = trial % 4;
    for (int y = 0; y < 41; ++y)
      for (int x = 0; x < 41; ++x) {
        const int dx = x - 20, dy = y - 20;
        const double r = U(g);
        if (shape == 0) fl[y][x] = r < p;                                   // scattered solid
        else if (shape == 1) fl[y][x] = dy > 0 || r < 0.1;                  // wall below
        else if (shape == 2) fl[y][x] = dx * dx + dy * dy > 9 + 20 * U(g);  // rough disk
        else fl[y][x] = (dx + 2 * dy) > 0 && r < 0.95;                      // inclined wall
      }
    fl[20][20] = 0;
    const int pi = 7, pj = 11;  // the node, at the centre of the field
    auto field = [&](int i, int j) -> bool {
      const int x = i - pi + 20, y = j - pj + 20;
      return x >= 0 && x <= 40 && y >= 0 && y <= 40 && fl[y][x];
    };
    FluidMask mask;
    mask.w[0] = mask.w[1] = 0;
    for (int dy = -kMaskR; dy <= kMaskR; ++dy)
      for (int dx = -kMaskR; dx <= kMaskR; ++dx)
        if (field(pi + dx, pj + dy)) mask.set(dx, dy);
    uint32_t far[kFarW];
    for (int dy = -kFarR; dy <= kFarR; ++dy) {
      far[dy + kFarR] = 0;
      for (int dx = -kFarR; dx <= kFarR; ++dx)
        if (field(pi + dx, pj + dy)) far[dy + kFarR] |= 1u << (dx + kFarR);
    }
    auto fluid = [&](int i, int j) -> bool {  // as the fill's test: the mask inside the block
      const int dx = i - pi, dy = j - pj;
      if (FluidMask::inside(dx, dy)) return mask.fluid(dx, dy);
      return field(i, j);
    };
    double ang = U(g) * 6.283185307179586;
    if (trial % 7 == 0) ang = (int)(U(g) * 8) * 0.7853981633974483;
    if (trial % 7 == 1) ang = std::atan2((double)((int)(U(g) * 7) - 3), (double)((int)(U(g) * 7) - 3));
    const double dx = std::cos(ang), dy = std::sin(ang);
    const LineHit a = march_line(pi, pj, dx, dy, fluid);
    const LineHit b = march_line_masked(pi, pj, dx, dy, mask, far, fluid);
    hits += a.ok;
    if (a.ok != b.ok || (a.ok && (a.i0 != b.i0 || a.j0 != b.j0 || a.i1 != b.i1 || a.j1 != b.j1 || a.w != b.w))) {
      if (++bad <= 5) std::printf("march mismatch, trial %ld angle %.17g\n", trial, ang);
    }
    // A candidate's angle range: at any angle in it, the masked march started at the candidate's
    // counters gives exactly the full march's hit.  Normals at random and lattice angles, the
    // candidate at a random angle, at 0 (along the normal) or on a ray through a node.
    if (trial % 4 == 0) {
      double al = U(g) * 6.283185307179586;
      if (trial % 3 == 0) al = (int)(U(g) * 8) * 0.7853981633974483;
      const double nx = std::cos(al), ny = std::sin(al), s = U(g) < 0.5 ? 1.0 : -1.0;
      double phi = U(g) * 1.4835298641951802;
      if (trial % 5 == 0) phi = 0.0;
      if (trial % 5 == 1) {  // a ray through a nearby node, when one lies in the angle range
        const int u = (int)(U(g) * 9) - 4, v = (int)(U(g) * 9) - 4;
        const double t = std::atan2(s * (u * -ny + v * nx), u * nx + v * ny);
        if ((u || v) && t >= 0.0 && t <= 1.4835298641951802) phi = t;
      }
      double lo, hi;
      int hk[2];
      const LineHit c = line_angle_range(pi, pj, nx, ny, s, phi, fluid, lo, hi, hk);
      // breakpoints shared at a larger radius (as the set-up forms them, one set per side): the
      // same hit and counters, and a range checked below as this one is
      double lo2, hi2;
      int hk2[2];
      const int Rb = c.ok ? line_reach(pi, pj, c) + (int)(U(g) * 6) : 3;
      const std::vector<double> brk = line_breakpoints(nx, ny, s, Rb);
      const LineHit c2 = line_angle_range(pi, pj, nx, ny, s, phi, fluid, lo2, hi2, hk2, &brk, Rb);
      if (!(c2.ok == c.ok && (!c.ok || (c2.i0 == c.i0 && c2.j0 == c.j0 && c2.i1 == c.i1 && c2.j1 == c.j1 &&
                                        hk2[0] == hk[0] && hk2[1] == hk[1]))) && ++bad_range <= 5)
        std::printf("shared breakpoints: another hit, trial %ld phi %.17g\n", trial, phi);
      for (int pass = 0; pass < 2; ++pass) {
        const double lo_ = pass ? lo2 : lo, hi_ = pass ? hi2 : hi;
        const int kx_ = pass ? hk2[0] : hk[0], ky_ = pass ? hk2[1] : hk[1];
        if (lo_ <= hi_) {
          ++ranges;
          for (int q = 0; q < 8; ++q) {
            const double f = q == 0 ? lo_ : (q == 1 ? hi_ : (q == 2 ? phi : lo_ + (hi_ - lo_) * U(g)));
            double sp, cp;
            sincos_quadrant(f, sp, cp);
            sp *= s;
            const double ex = cp * nx + sp * -ny, ey = cp * ny + sp * nx;
            const LineHit full = march_line(pi, pj, ex, ey, fluid);
            const LineHit from = march_line_masked(pi, pj, ex, ey, mask, far, fluid, kx_, ky_);
            const bool same = full.ok == from.ok && full.ok && full.i0 == from.i0 && full.j0 == from.j0 &&
                              full.i1 == from.i1 && full.j1 == from.j1 && full.w == from.w && full.i0 == c.i0 &&
                              full.j0 == c.j0 && full.i1 == c.i1 && full.j1 == c.j1;
            if (!same && ++bad_range <= 5)
              std::printf("range mismatch, trial %ld phi %.17g in [%.17g, %.17g] at %.17g\n", trial, phi, lo_, hi_, f);
          }
        }
      }
    }
  }
  double es = 0.0, ec = 0.0;
  const long n = 1000000;
  for (long k = 0; k <= n; ++k) {
    const double phi = 1.4835298641951802 * k / n;
    double s, c;
    sincos_quadrant(phi, s, c);
    es = std::fmax(es, ulps(s, (double)sinl((long double)phi)));
    ec = std::fmax(ec, ulps(c, (double)cosl((long double)phi)));
  }
  std::printf("trials %ld hits %ld march mismatches %ld; angle ranges %ld, mismatches %ld; sincos max ulp %.2f %.2f\n",
              trials, hits, bad, ranges, bad_range, es, ec);
  return (bad != 0 || bad_range != 0 || ranges < trials / 20 || es > 1.0 || ec > 1.0) ? 1 : 0;
}
