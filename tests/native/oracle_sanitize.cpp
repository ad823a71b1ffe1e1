// Drives the FP64 oracle (linked from oracle/lbm3_oracle.cpp) through every boundary type for a
// few steps, and through its rejected inputs, for an AddressSanitizer / UndefinedBehaviorSanitizer
// build: walls with a curved solid, fully periodic, fluid-exchanging periodic, Zou-He with a
// curved solid, and a one-node slot whose characteristic lines fail.  Exit status 0 when every
// run stays finite and every bad input is rejected.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

extern "C" {
typedef struct {
  int32_t nx, ny, y_periodic, bc_x;
  double u_in, rho_out, nu[3], sigma[3], theta_deg[2], beta0, body_force[2];
  int32_t n_circles, force_half_q;
  const double *circles;
  const uint8_t *solid;
  const double *rho_init;
} orc_domain;
void *orc_create(const orc_domain *d, char *errbuf, int errlen);
void orc_destroy(void *h);
void orc_step(void *h, int n);
void orc_mass(void *h, double *out);
void orc_get_rho(void *h, double *out);
void orc_set_threads(int n);
}

struct Case {
  const char *name;
  int nx, ny, yper, bcx;
  std::vector<double> circ;
  bool walls, slot;
};

static bool run(const Case &c, bool expect_ok, double theta13 = 60.0) {
  const int nx = c.nx, ny = c.ny;
  std::vector<uint8_t> solid((size_t)nx * ny, 0);
  std::vector<double> rho(3 * (size_t)nx * ny, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      bool s = c.walls && (j == 0 || j == ny - 1);
      for (size_t k = 0; k + 2 < c.circ.size(); k += 3) {
        const double dx = i - c.circ[k], dy = j - c.circ[k + 1];
        if (dx * dx + dy * dy <= c.circ[k + 2] * c.circ[k + 2]) s = true;
      }
      if (c.slot) s = !(i == nx / 2 && j > 0 && j < ny - 1) && !(i > nx / 2 && i < nx / 2 + 8 && j > 2 && j < ny - 1);
      solid[(size_t)j * nx + i] = s;
      if (s) continue;
      const double a = 0.5 + 0.4 * std::sin(0.3 * i + 0.2 * j), b = 0.3 + 0.2 * std::cos(0.25 * i - 0.1 * j);
      const double t = a + b + 0.4;
      rho[(size_t)j * nx + i] = a / t;
      rho[(size_t)nx * ny + (size_t)j * nx + i] = b / t;
      rho[2 * (size_t)nx * ny + (size_t)j * nx + i] = 0.4 / t;
    }
  orc_domain d;
  std::memset(&d, 0, sizeof d);
  d.nx = nx;
  d.ny = ny;
  d.y_periodic = c.yper;
  d.bc_x = c.bcx;
  d.u_in = c.bcx == 2 ? 0.004 : 0.0;
  d.rho_out = 1.0;
  d.nu[0] = 0.1; d.nu[1] = 0.07; d.nu[2] = 0.13;
  d.sigma[0] = 0.01; d.sigma[1] = 0.012; d.sigma[2] = 0.011;
  d.theta_deg[0] = theta13;
  d.theta_deg[1] = 100.0;
  d.beta0 = 0.7;
  d.n_circles = (int32_t)(c.circ.size() / 3);
  d.circles = c.circ.empty() ? nullptr : c.circ.data();
  d.solid = solid.data();
  d.rho_init = rho.data();
  char err[256] = {0};
  void *h = orc_create(&d, err, sizeof err);
  if (!h) {
    std::printf("%s: rejected (%s)\n", c.name, err);
    return !expect_ok;
  }
  if (!expect_ok) {
    std::printf("%s: accepted but should be rejected\n", c.name);
    orc_destroy(h);
    return false;
  }
  orc_step(h, 6);
  double m[3];
  orc_mass(h, m);
  std::vector<double> r(3 * (size_t)nx * ny);
  orc_get_rho(h, r.data());
  orc_destroy(h);
  bool ok = std::isfinite(m[0]) && std::isfinite(m[1]) && std::isfinite(m[2]);
  for (double v : r) ok = ok && std::isfinite(v);
  std::printf("%s: masses %.12f %.12f %.12f %s\n", c.name, m[0], m[1], m[2], ok ? "ok" : "NON-FINITE");
  return ok;
}

int main() {
  orc_set_threads(2);
  bool ok = true;
  ok &= run({"walls+circle", 48, 30, 0, 0, {20.3, 14.6, 5.2}, true, false}, true);
  ok &= run({"periodic", 24, 20, 1, 0, {}, false, false}, true);
  ok &= run({"swap13", 40, 16, 0, 1, {}, true, false}, true);
  ok &= run({"zouhe+circle", 48, 24, 1, 2, {24.5, 11.3, 5.0}, false, false}, true);
  ok &= run({"slot (a failed line)", 40, 30, 0, 0, {}, false, true}, true);
  ok &= run({"3x3 periodic", 3, 3, 1, 0, {}, false, false}, true);
  // rejected: Zou-He without periodic y; solid next to the Zou-He columns; an isolated solid node
  ok &= run({"zouhe, walls", 30, 20, 0, 2, {}, true, false}, false);
  ok &= run({"zouhe, solid at inlet", 30, 20, 1, 2, {1.0, 10.0, 3.0}, false, false}, false);
  ok &= run({"isolated solid node", 20, 20, 1, 0, {10.0, 10.0, 0.1}, false, false}, false);
  std::printf(ok ? "ALL OK\n" : "FAILED\n");
  return ok ? 0 : 1;
}
