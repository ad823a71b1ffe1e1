// Calls the library's host-only entry point lbm3_workspace_bytes (validation and the one-time
// boundary set-up: categories, Eq. 19-20 normals, the characteristic-line D0 march, link
// fractions, the layout) on valid and invalid domains, for an AddressSanitizer /
// UndefinedBehaviorSanitizer build of the host code.  No device call is made.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lbm3.h"

static int check(const char *name, int nx, int ny, int yper, int bcx, std::vector<double> circ, bool walls, bool ok_expected,
                 int precision, int adjoint) {
  std::vector<uint8_t> solid((size_t)nx * ny, 0);
  std::vector<double> rho(3 * (size_t)nx * ny, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      bool s = walls && (j == 0 || j == ny - 1);
      for (size_t k = 0; k + 2 < circ.size(); k += 3) {
        const double dx = i - circ[k], dy = j - circ[k + 1];
        if (dx * dx + dy * dy <= circ[k + 2] * circ[k + 2]) s = true;
      }
      solid[(size_t)j * nx + i] = s;
      if (!s) rho[2 * (size_t)nx * ny + (size_t)j * nx + i] = 1.0;
    }
  lbm3_domain d;
  std::memset(&d, 0, sizeof d);
  d.nx = nx; d.ny = ny; d.y_periodic = yper; d.bc_x = bcx;
  d.u_in = bcx == LBM3_X_ZOUHE ? 0.005 : 0.0;
  d.rho_out = 1.0;
  for (int k = 0; k < 3; ++k) { d.nu[k] = 0.1; d.sigma[k] = 0.01; }
  d.theta_deg[0] = 60.0; d.theta_deg[1] = 90.0;
  d.n_circles = (int32_t)(circ.size() / 3);
  d.circles = circ.empty() ? nullptr : circ.data();
  d.solid = solid.data();
  d.rho_init = rho.data();
  lbm3_options o;
  std::memset(&o, 0, sizeof o);
  o.precision = precision;
  o.kernel = 0;
  o.adjoint = adjoint;
  size_t bytes = 0;
  const lbm3_status st = lbm3_workspace_bytes(&d, 1, &o, &bytes);
  bool ok = (st == LBM3_OK) == ok_expected;
  // a rejection names its domain once and its cause
  if (st != LBM3_OK && std::strstr(lbm3_plan_error(), "domain 0: domain") != nullptr) ok = false;
  std::printf("%s: status %d (%s) bytes %zu %s\n", name, (int)st, st == LBM3_OK ? "ok" : lbm3_plan_error(), bytes,
              ok ? "as expected" : "UNEXPECTED");
  return ok ? 0 : 1;
}

int main() {
  int bad = 0;
  bad += check("walls+circle f64 adjoint", 64, 40, 0, LBM3_X_PERIODIC, {30.3, 19.6, 7.2}, true, true, LBM3_F64, 1);
  bad += check("walls+circle f32", 64, 40, 0, LBM3_X_PERIODIC, {30.3, 19.6, 7.2}, true, true, LBM3_F32, 0);
  bad += check("periodic f16", 40, 32, 1, LBM3_X_PERIODIC, {}, false, true, LBM3_F32_STORE_F16, 0);
  bad += check("swap13", 48, 32, 0, LBM3_X_PERIODIC_SWAP13, {}, true, true, LBM3_F32, 1);
  bad += check("zouhe+circles", 96, 48, 1, LBM3_X_ZOUHE, {30.5, 20.2, 8.0, 60.1, 30.3, 6.0}, false, true, LBM3_F32, 1);
  bad += check("3x3", 3, 3, 1, LBM3_X_PERIODIC, {}, false, true, LBM3_F64, 1);
  bad += check("zouhe without periodic y", 30, 20, 0, LBM3_X_ZOUHE, {}, true, false, LBM3_F32, 0);
  bad += check("isolated solid node", 20, 20, 1, LBM3_X_PERIODIC, {10.0, 10.0, 0.1}, false, false, LBM3_F32, 0);
  if (std::strstr(lbm3_plan_error(), "degenerate solid normal at node (10,10)") == nullptr) {
    std::printf("unexpected message: %s\n", lbm3_plan_error());
    ++bad;
  }
  bad += check("too small", 2, 20, 1, LBM3_X_PERIODIC, {}, false, false, LBM3_F32, 0);
  bad += check("f16 with adjoint", 40, 32, 1, LBM3_X_PERIODIC, {}, false, false, LBM3_F32_STORE_F16, 1);
  std::printf(bad ? "FAILED\n" : "ALL OK\n");
  return bad ? 1 : 0;
}
