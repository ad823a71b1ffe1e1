// lbm3_oracle.cpp -- plain FP64 CPU oracle for the three-phase colour-gradient D2Q9 step of
// Li, Lu, Jiang & Liu, "Lattice Boltzmann simulation of three-phase flows with moving contact
// lines on curved surfaces" (arXiv:2102.04709).
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
// benchmark load this library.  It shares no code, header, table or helper with the GPU library.
//
// It runs the paper's algorithm literally: nine populations for each of the three fluids
// (27 values per node), nested loops, a fixed summation order (alpha = 0..8, fluids 1..3) and
// double precision everywhere.  Each stage names the passage it follows:
//   Sec. II A, Eq. (1)-(9)   MRT collision with the forcing term
//   Eq. (10)-(12)            interfacial force from the colour gradients, velocity, gradients
//   Eq. (13)-(15)            recolouring with the pairwise segregation parameters
//   Eq. (16)                 streaming and the per-fluid densities
//   Sec. II B, Eq. (17)-(22) Young relations, node categories, solid normal, weighted contact
//                            angle and the characteristic-line wetting fill
//   Sec. III                 flow boundary conditions: halfway bounce-back (III A), modified
//                            periodic exchange of fluids 1 and 3 (III C), Zou-He velocity inlet
//                            and pressure outlet (III D)
// Where the paper is silent or ambiguous, the choice made is marked "reading:" below.
// Parity status: every stage is pinned by a CPU test (tests/test_oracle_*.py) against closed
// forms, invariants, brute force (the characteristic-line march and its fallbacks) or physics
// (Table I angles, the Neumann triangle, Eq. 23 on a cylinder, Laplace, Poiseuille, Zou-He).
// Parity unpinned: the numerical constants of the readings -- the |G| threshold of the normals,
// the 1e-9 node tolerance and the t = 24 end of the line march -- which the physics pins
// constrain only through the contact angles they produce.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
// Problem description (the oracle's own copy of the inputs; not the GPU library's struct).
typedef struct {
  int32_t nx, ny;
  int32_t y_periodic;       // 1: periodic in y; 0: everything outside 0 <= y < ny is solid
  int32_t bc_x;             // 0 periodic, 1 periodic with fluid-1/fluid-3 exchange, 2 Zou-He
  double u_in, rho_out;     // Zou-He inlet velocity and outlet density
  double nu[3];             // viscosities of the pure fluids (rho_k^0 = 1, so mu_k = nu_k)
  double sigma[3];          // sigma12, sigma13, sigma23
  double theta_deg[2];      // theta13, theta23 (degrees), measured inside fluids 1 and 2
  double beta0;             // reference segregation parameter (the paper fixes 0.7)
  double body_force[2];     // uniform acceleration (test hook), added as rho*g to F_s
  int32_t n_circles;
  int32_t force_half_q;     // test hook: every solid link uses q = 1/2
  const double *circles;    // [3*n_circles] (cx, cy, R): exact solid geometry for q
  const uint8_t *solid;     // [ny*nx], x fastest
  const double *rho_init;   // [3][ny*nx] initial partial densities
} orc_domain;
}

namespace {

// D2Q9 lattice, Sec. II A: e_0=(0,0), e_{1,3}=(+-1,0), e_{2,4}=(0,+-1), e_{5,6}=(+-1,1),
// e_{7,8}=(-+1,-1); weights 4/9, 1/9 and 1/36 (reading: the garbled index range of the last
// weight means directions 5..8, the only choice with weights summing to one).
const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double WT[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Transformation matrix, Eq. (4).
const double MM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

double MINV[9][9];

// M^{-1} by Gauss-Jordan elimination with partial pivoting (a generic inverse, so that the
// pinned identity M^{-1} M = I checks Eq. (4) rather than a hand-derived closed form).
struct MinvInit {
  MinvInit() {
    double a[9][18];
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 18; ++j) a[i][j] = j < 9 ? MM[i][j] : (j - 9 == i ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
      int p = c;
      for (int r = c + 1; r < 9; ++r)
        if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
      for (int j = 0; j < 18; ++j) std::swap(a[c][j], a[p][j]);
      double d = a[c][c];
      for (int j = 0; j < 18; ++j) a[c][j] /= d;
      for (int r = 0; r < 9; ++r) {
        if (r == c) continue;
        double m = a[r][c];
        if (m == 0.0) continue;
        for (int j = 0; j < 18; ++j) a[r][j] -= m * a[c][j];
      }
    }
    for (int i = 0; i < 9; ++i)
      for (int j = 0; j < 9; ++j) MINV[i][j] = a[i][j + 9];
  }
} minv_init;

const double PI = 3.14159265358979323846;
const double EPS_G = 1e-12;     // reading: |G_kl| at or below this gives n_kl = 0, no stress
const double EPS_DIR = 1e-12;   // reading: direction components below this are axis-parallel
const double EPS_NODE = 1e-9;   // reading: a crossing this close to a node is a node hit
const double T_MAX = 24.0;      // reading: a characteristic line is extended at most this far
const double THETA_LO = 5.0 * PI / 180.0, THETA_HI = 175.0 * PI / 180.0;  // line-angle clamp

enum { T_FLUID = 0, T_SB = 1, T_SB2 = 2, T_SOLID = 3, T_GHOST = 4 };

inline int pmod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Eq. (3).
void equilibrium(double rho, double ux, double uy, double *feq) {
  double uu = ux * ux + uy * uy;
  for (int a = 0; a < 9; ++a) {
    double eu = EX[a] * ux + EY[a] * uy;
    feq[a] = rho * WT[a] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

// Eq. (9) with c_s^2 = 1/3 and delta_t = 1.
void force_populations(double ux, double uy, double Fx, double Fy, double *ft) {
  for (int a = 0; a < 9; ++a) {
    double eu = EX[a] * ux + EY[a] * uy;
    double vx = 3.0 * (EX[a] - ux) + 9.0 * eu * EX[a];
    double vy = 3.0 * (EY[a] - uy) + 9.0 * eu * EY[a];
    ft[a] = WT[a] * (vx * Fx + vy * Fy);
  }
}

// Eq. (5)-(6).
void relaxation_rates(double tau, double *s) {
  double s1 = 1.0 / tau;
  double s4 = 8.0 * (2.0 - s1) / (8.0 - s1);
  double v[9] = {0.0, s1, s1, 0.0, s4, 0.0, s4, s1, s1};
  for (int i = 0; i < 9; ++i) s[i] = v[i];
}

// Eq. (7) with mu = (tau - 1/2) rho c_s^2 and rho_k^0 = 1 (so mu_k = nu_k):
// tau = 1/2 + 3 / sum_k (rho_k / mu_k).
double relaxation_time(const double *rk, const double *nu) {
  double s = 0.0;
  for (int k = 0; k < 3; ++k) s += rk[k] / nu[k];
  return 0.5 + 3.0 / s;
}

// Eq. (1), (2), (8) on one node: f_dag = f - M^-1 S M (f - feq) + M^-1 (I - S/2) M F~,
// with u from Eq. (11).  F is the total force density acting on the node.
void collide(const double *f, const double *rk, const double *nu, double Fx, double Fy,
             double *fdag, double *u_out) {
  double rho = rk[0] + rk[1] + rk[2];
  double jx = 0.0, jy = 0.0;
  for (int a = 0; a < 9; ++a) {
    jx += f[a] * EX[a];
    jy += f[a] * EY[a];
  }
  double ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
  if (u_out) {
    u_out[0] = ux;
    u_out[1] = uy;
  }
  double tau = relaxation_time(rk, nu);
  double S[9];
  relaxation_rates(tau, S);
  double feq[9], ft[9];
  equilibrium(rho, ux, uy, feq);
  force_populations(ux, uy, Fx, Fy, ft);
  double m[9], meq[9], mf[9], dm[9];
  for (int i = 0; i < 9; ++i) {
    m[i] = meq[i] = mf[i] = 0.0;
    for (int a = 0; a < 9; ++a) {
      m[i] += MM[i][a] * f[a];
      meq[i] += MM[i][a] * feq[a];
      mf[i] += MM[i][a] * ft[a];
    }
  }
  for (int i = 0; i < 9; ++i) dm[i] = -S[i] * (m[i] - meq[i]) + (1.0 - 0.5 * S[i]) * mf[i];
  for (int a = 0; a < 9; ++a) {
    double s = 0.0;
    for (int i = 0; i < 9; ++i) s += MINV[a][i] * dm[i];
    fdag[a] = f[a] + s;
  }
}

// Eq. (15): g(X).
double g_of_X(double X) {
  if (X < -1.0) return 1.0;
  if (X < 0.0) return 1.0 - std::sin(std::acos(X));
  if (X <= 1.0) return std::sin(std::acos(X)) - 1.0;
  return -1.0;
}

// sigma is (s12, s13, s23); pair index p(k,l) for unordered fluid pairs.
inline int pair_index(int k, int l) {
  if (k > l) std::swap(k, l);
  return k == 0 ? (l == 1 ? 0 : 1) : 2;
}

// X_kl of Eq. (15), m the third fluid.
void segregation_X(const double *sig, double *X) {
  for (int k = 0; k < 3; ++k)
    for (int l = k + 1; l < 3; ++l) {
      int m = 3 - k - l;
      double smk = sig[pair_index(m, k)], sml = sig[pair_index(m, l)], skl = sig[pair_index(k, l)];
      X[pair_index(k, l)] = (smk * smk + sml * sml - skl * skl) / (2.0 * smk * sml);
    }
}

// Eq. (13)-(14) on one node.  nk[k][l] is n_kl (ordered pairs, n_kk unused); gX per pair.
void recolour(const double *fdag, const double *rk, const double nk[3][3][2], const double *gX,
              double beta0, double *out /*[3][9]*/) {
  double rho = rk[0] + rk[1] + rk[2];
  double r3 = 35.0 * rk[0] * rk[1] * rk[2] / (rho * rho * rho);
  r3 = std::min(std::max(r3, 0.0), 1.0);  // reading: also clamped below at 0
  for (int k = 0; k < 3; ++k)
    for (int a = 0; a < 9; ++a) {
      double v = rk[k] / rho * fdag[a];
      for (int l = 0; l < 3; ++l) {
        if (l == k) continue;
        double beta = beta0 + beta0 * r3 * gX[pair_index(k, l)];
        double ne = nk[k][l][0] * EX[a] + nk[k][l][1] * EY[a];
        v += beta * WT[a] * rk[k] * rk[l] / rho * ne;
      }
      out[k * 9 + a] = v;
    }
}

// Eq. (19)-(20) numerator, sum_c w(|c|^2) s(x + c) c over the 24 points of the 5x5 block,
// in units of 1/5040: the weights 4/21, 4/45, 1/60, 2/315, 1/5040 are 960, 448, 84, 32, 1.
// block[(cy+2)*5 + cx+2] holds s(x + c).
void isotropic_sum(const long *block, long *out) {
  long sx = 0, sy = 0;
  for (int cy = -2; cy <= 2; ++cy)
    for (int cx = -2; cx <= 2; ++cx) {
      int c2 = cx * cx + cy * cy;
      if (c2 == 0) continue;
      long w = c2 == 1 ? 960 : c2 == 2 ? 448 : c2 == 4 ? 84 : c2 == 5 ? 32 : 1;
      long s = block[(cy + 2) * 5 + cx + 2];
      sx += w * s * cx;
      sy += w * s * cy;
    }
  out[0] = sx;
  out[1] = sy;
}

struct Cross {
  int ok;
  int n0, n1;  // ext indices of the two interpolation nodes (equal for a node hit)
  double w;    // C = C[n0] + w (C[n1] - C[n0])
};

struct Oracle {
  int nx, ny, yper, bcx, GX, PY, NXE, NYE, NE;
  double u_in, rho_out, nu[3], sig[3], beta0, gacc[2];
  double th13, th23, th12;
  double gX[3];
  std::vector<double> circ;
  std::vector<uint8_t> solid;  // base solid indicator per ext node
  std::vector<uint8_t> type;   // node category per ext node
  std::vector<int> nb;         // [9][NE] neighbour ext index (wrap / clamp)
  std::vector<int> fill;       // fill node ext indices (C_SB then C_SB2 in index order)
  std::vector<double> fnx, fny;
  std::vector<Cross> d0;
  std::vector<double> f, fpp, fnew;  // [27][NE]
  std::vector<double> C, rk, rho;    // [3][NE], [3][NE], [NE]
  std::vector<double> T;             // [3][NE]  Txx, Txy, Tyy
  std::vector<double> nvec;          // [3][3][2][NE] ordered-pair normals
  std::vector<double> Fs;            // [2][NE]
  std::vector<double> U;             // [2][NE] velocity of the last collision, Eq. (11)
  std::vector<double> qv;            // [9][NE]
  std::vector<int> fill_fail;        // per fill node: lines that failed at the last fill (bits)
  std::string err;
  long steps = 0;

  int ext(int i, int j) const {
    if (bcx != 2) i = pmod(i, nx);
    else i = std::min(std::max(i, -GX), nx + GX - 1);
    if (yper) j = pmod(j, ny);
    else j = std::min(std::max(j, -PY), ny + PY - 1);
    return (i + GX) + NXE * (j + PY);
  }
  int ei(int e) const { return e % NXE - GX; }
  int ej(int e) const { return e / NXE - PY; }
  bool fluid_at(int i, int j) const { return type[ext(i, j)] == T_FLUID; }

  bool setup(const orc_domain *d);
  Cross march(int pi, int pj, double dx, double dy) const;
  double interp(const Cross &c, int k) const {
    return C[k * NE + c.n0] + c.w * (C[k * NE + c.n1] - C[k * NE + c.n0]);
  }
  // Eq. (12): d(psi)/dx_i = (1/c_s^2) sum_a w_a psi(x + e_a) e_ai, on an extended-grid field.
  void gradient(const double *psi, int e, double *g) const {
    double gx = 0, gy = 0;
    for (int a = 0; a < 9; ++a) {
      double c = psi[nb[a * NE + e]];
      gx += WT[a] * c * EX[a];
      gy += WT[a] * c * EY[a];
    }
    g[0] = 3.0 * gx;
    g[1] = 3.0 * gy;
  }
  void densities();
  void fill_solid();
  void stresses();
  void forces();
  void prepare() {
    densities();
    fill_solid();
    stresses();
    forces();
  }
  void collide_recolour_stream();
  void step() {
    prepare();
    collide_recolour_stream();
    ++steps;
  }
};

bool Oracle::setup(const orc_domain *d) {
  nx = d->nx;
  ny = d->ny;
  yper = d->y_periodic;
  bcx = d->bc_x;
  if (nx < 3 || ny < 3) return err = "nx and ny must be >= 3", false;
  if (bcx < 0 || bcx > 2) return err = "bc_x must be 0, 1 or 2", false;
  if (bcx == 2 && !yper) return err = "the Zou-He x boundary requires y_periodic = 1", false;
  if (bcx == 1 && d->n_circles > 0) return err = "curved solids are not allowed with the fluid-exchange periodic boundary", false;
  GX = bcx == 2 ? 2 : 0;
  PY = yper ? 0 : 2;
  NXE = nx + 2 * GX;
  NYE = ny + 2 * PY;
  NE = NXE * NYE;
  u_in = d->u_in;
  rho_out = d->rho_out;
  beta0 = d->beta0;
  for (int k = 0; k < 3; ++k) {
    nu[k] = d->nu[k];
    sig[k] = d->sigma[k];
    if (!(sig[k] > 0.0)) return err = "every interfacial tension must be > 0", false;
    double tau = 0.5 + 3.0 * nu[k];
    if (!(tau > 0.5 && tau <= 10.0)) return err = "viscosity gives tau outside (0.5, 10]", false;
  }
  gacc[0] = d->body_force[0];
  gacc[1] = d->body_force[1];
  for (int k = 0; k < 2; ++k)
    if (!(d->theta_deg[k] > 0.0 && d->theta_deg[k] < 180.0)) return err = "contact angles must lie in (0, 180)", false;
  th13 = d->theta_deg[0] * PI / 180.0;
  th23 = d->theta_deg[1] * PI / 180.0;
  // Eq. (17)-(18): sigma12 cos th12 + sigma31 cos th31 + sigma23 cos th23 = 0 with
  // th31 = pi - th13, hence cos th12 = (sigma13 cos th13 - sigma23 cos th23) / sigma12.
  double c12 = (sig[1] * std::cos(th13) - sig[2] * std::cos(th23)) / sig[0];
  if (std::fabs(c12) > 1.0 + 1e-12) return err = "contact angles and tensions violate Eq. (18) (|cos theta12| > 1)", false;
  c12 = std::min(std::max(c12, -1.0), 1.0);
  th12 = std::acos(c12);
  double X[3];
  segregation_X(sig, X);
  for (int p = 0; p < 3; ++p) gX[p] = g_of_X(X[p]);
  if (d->n_circles > 0) circ.assign(d->circles, d->circles + 3 * d->n_circles);

  // Base solid indicator; rows outside a non-periodic y range are solid, Zou-He ghost columns
  // are not.
  solid.assign(NE, 0);
  type.assign(NE, T_GHOST);
  for (int j = -PY; j < ny + PY; ++j)
    for (int i = -GX; i < nx + GX; ++i) {
      int e = (i + GX) + NXE * (j + PY);
      if (j < 0 || j >= ny) solid[e] = 1;
      else if (i >= 0 && i < nx) solid[e] = d->solid[i + nx * j] ? 1 : 0;
    }
  if (bcx == 2)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < 3; ++i)
        if (d->solid[i + nx * j] || d->solid[(nx - 1 - i) + nx * j])
          return err = "solid nodes within 3 columns of a Zou-He boundary", false;
  nb.assign(9 * NE, 0);
  for (int e = 0; e < NE; ++e)
    for (int a = 0; a < 9; ++a) nb[a * NE + e] = ext(ei(e) + EX[a], ej(e) + EY[a]);
  // Node categories, Sec. II B.  Reading: "in contact with" is the 8-neighbourhood of D2Q9.
  for (int e = 0; e < NE; ++e) {
    int i = ei(e);
    bool ingrid_x = i >= 0 && i < nx;
    if (!solid[e]) type[e] = ingrid_x ? T_FLUID : T_GHOST;
    else type[e] = T_SOLID;
  }
  for (int e = 0; e < NE; ++e) {
    if (type[e] != T_SOLID) continue;
    for (int a = 1; a < 9; ++a)
      if (type[nb[a * NE + e]] == T_FLUID) {
        type[e] = T_SB;
        break;
      }
  }
  // Reading: a second layer of solid nodes (neighbours of C_SB that touch no fluid) is filled
  // as well, because the divergence in Eq. (10) at a boundary fluid node needs the stress at
  // C_SB nodes, whose own gradient reaches one more node into the solid.
  for (int e = 0; e < NE; ++e) {
    if (type[e] != T_SOLID) continue;
    for (int a = 1; a < 9; ++a)
      if (type[nb[a * NE + e]] == T_SB) {
        type[e] = T_SB2;
        break;
      }
  }
  for (int e = 0; e < NE; ++e)
    if (type[e] == T_SB) fill.push_back(e);
  for (int e = 0; e < NE; ++e)
    if (type[e] == T_SB2) fill.push_back(e);

  // Eq. (19)-(20) solid normal over the 24 points of the 5x5 block.  The weights 4/21, 4/45,
  // 1/60, 2/315, 1/5040 are 960, 448, 84, 32, 1 in units of 1/5040; the sum is formed in
  // integers (exact, so symmetric stencils cancel exactly) and then normalised.  Reading: the
  // sum points into the solid (s = 1 there); the fill uses the opposite, fluid-pointing vector.
  fnx.resize(fill.size());
  fny.resize(fill.size());
  d0.resize(fill.size());
  fill_fail.assign(fill.size(), 0);
  for (size_t p = 0; p < fill.size(); ++p) {
    int i = ei(fill[p]), j = ej(fill[p]);
    long block[25], sum[2];
    for (int cy = -2; cy <= 2; ++cy)
      for (int cx = -2; cx <= 2; ++cx) block[(cy + 2) * 5 + cx + 2] = solid[ext(i + cx, j + cy)];
    isotropic_sum(block, sum);
    long sx = sum[0], sy = sum[1];
    if (sx == 0 && sy == 0) {
      char b[160];
      snprintf(b, sizeof b, "degenerate solid normal at fill node (%d,%d)", i, j);
      return err = b, false;
    }
    double len = std::sqrt((double)sx * sx + (double)sy * sy);
    fnx[p] = -(double)sx / len;
    fny[p] = -(double)sy / len;
    d0[p] = march(i, j, fnx[p], fny[p]);
    if (!d0[p].ok) {
      char b[160];
      snprintf(b, sizeof b, "the normal line from fill node (%d,%d) reaches no fluid", i, j);
      return err = b, false;
    }
  }

  // Link fractions q for solid links (reading: Bouzidi linear interpolated bounce-back on the
  // exact circles, applied to the total distribution; links whose solid node lies in no circle use
  // q = 1/2, halfway bounce-back).
  qv.assign(9 * NE, 0.5);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int e = ext(i, j);
      if (type[e] != T_FLUID) continue;
      for (int a = 1; a < 9; ++a) {
        int si = i - EX[a], sj = j - EY[a];
        if (bcx == 2 && (si < 0 || si >= nx)) continue;
        if (type[ext(si, sj)] == T_FLUID) continue;
        double q = 0.5;
        bool found = false;
        if (!d->force_half_q) {
          for (size_t c = 0; c < circ.size() / 3; ++c) {
            for (int ix = -1; ix <= 1; ++ix)
              for (int iy = -1; iy <= 1; ++iy) {
                if (ix && bcx == 2) continue;
                if (iy && !yper) continue;
                double cx = circ[3 * c] + ix * nx, cy = circ[3 * c + 1] + iy * ny, R = circ[3 * c + 2];
                double dxs = si - cx, dys = sj - cy, dxf = i - cx, dyf = j - cy;
                if (dxs * dxs + dys * dys > R * R) continue;   // solid node not in this circle
                if (dxf * dxf + dyf * dyf <= R * R) continue;  // fluid node inside: ignore
                // |x - q e_a - c| = R, smallest root: a2 q^2 - 2 b q + cc = 0.
                double a2 = EX[a] * EX[a] + EY[a] * EY[a];
                double b = EX[a] * dxf + EY[a] * dyf;
                double cc = dxf * dxf + dyf * dyf - R * R;
                double disc = b * b - a2 * cc;
                double qq = (b - std::sqrt(std::max(disc, 0.0))) / a2;
                if (!found || qq < q) q = qq;
                found = true;
              }
          }
        }
        if (found) q = std::min(std::max(q, 1e-6), 1.0);
        qv[a * NE + e] = q;
      }
    }

  // Initial state (reading: u = 0, f_{a,k} = rho_k w_a from the given partial densities).
  f.assign(27 * NE, 0.0);
  fpp.assign(27 * NE, 0.0);
  fnew.assign(27 * NE, 0.0);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      int e = ext(i, j);
      if (type[e] != T_FLUID) continue;
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 9; ++a) f[(k * 9 + a) * NE + e] = d->rho_init[k * nx * ny + i + nx * j] * WT[a];
    }
  C.assign(3 * NE, 0.0);
  rk.assign(3 * NE, 0.0);
  rho.assign(NE, 1.0);
  T.assign(3 * NE, 0.0);
  nvec.assign(18 * NE, 0.0);
  Fs.assign(2 * NE, 0.0);
  U.assign(2 * NE, 0.0);
  return true;
}

// Characteristic line P + t d, t > 0 (Sec. II B): walk the crossings with the vertical and
// horizontal grid lines in order of increasing t; at a crossing with a horizontal line the
// left/right nodes are interpolated, at a vertical line the lower/upper nodes; a crossing that
// lands on a node uses that node alone.  The first crossing whose interpolation nodes are all
// fluid nodes is the intersection point D; the line is given up beyond t = T_MAX.
Cross Oracle::march(int pi, int pj, double dx, double dy) const {
  Cross r{0, 0, 0, 0.0};
  int sx = dx > EPS_DIR ? 1 : dx < -EPS_DIR ? -1 : 0;
  int sy = dy > EPS_DIR ? 1 : dy < -EPS_DIR ? -1 : 0;
  double ax = std::fabs(dx), ay = std::fabs(dy);
  int kx = 1, ky = 1;
  for (int guard = 0; guard < 256; ++guard) {
    double tx = sx ? (double)kx / ax : 1e300;
    double ty = sy ? (double)ky / ay : 1e300;
    double t = std::min(tx, ty);
    if (t > T_MAX) return r;
    if (tx <= ty) {
      int i = pi + sx * kx;
      double y = pj + tx * dy;
      double yr = std::floor(y + 0.5);
      ++kx;
      if (std::fabs(y - yr) < EPS_NODE) {
        int j = (int)yr;
        if (sy && j == pj + sy * ky) ++ky;
        if (fluid_at(i, j)) {
          int e = ext(i, j);
          return Cross{1, e, e, 0.0};
        }
      } else {
        int j0 = (int)std::floor(y);
        if (fluid_at(i, j0) && fluid_at(i, j0 + 1))
          return Cross{1, ext(i, j0), ext(i, j0 + 1), y - j0};
      }
    } else {
      int j = pj + sy * ky;
      double x = pi + ty * dx;
      double xr = std::floor(x + 0.5);
      ++ky;
      if (std::fabs(x - xr) < EPS_NODE) {
        int i = (int)xr;
        if (sx && i == pi + sx * kx) ++kx;
        if (fluid_at(i, j)) {
          int e = ext(i, j);
          return Cross{1, e, e, 0.0};
        }
      } else {
        int i0 = (int)std::floor(x);
        if (fluid_at(i0, j) && fluid_at(i0 + 1, j))
          return Cross{1, ext(i0, j), ext(i0 + 1, j), x - i0};
      }
    }
  }
  return r;
}

// Partial densities of Eq. (16) and C_k = rho_k / rho at fluid nodes.
void Oracle::densities() {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < NE; ++e) {
    if (type[e] == T_FLUID) {
      double r[3];
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int a = 0; a < 9; ++a) s += f[(k * 9 + a) * NE + e];
        r[k] = s;
      }
      double rt = r[0] + r[1] + r[2];
      for (int k = 0; k < 3; ++k) {
        rk[k * NE + e] = r[k];
        C[k * NE + e] = r[k] / rt;
      }
      rho[e] = rt;
    } else {
      for (int k = 0; k < 3; ++k) rk[k * NE + e] = C[k * NE + e] = 0.0;
      rho[e] = 1.0;
    }
  }
}

// Characteristic-line wetting fill, Eq. (21)-(22), at every C_SB and C_SB2 node.
void Oracle::fill_solid() {
  std::vector<double> out(3 * fill.size());
#pragma omp parallel for schedule(static)
  for (long p = 0; p < (long)fill.size(); ++p) {
    int e = fill[p];
    int i = ei(e), j = ej(e);
    double nxv = fnx[p], nyv = fny[p];
    double tx = -nyv, ty = nxv;  // tangent
    // Reading: the C used in Eq. (21) is the value at D0, where the normal line meets the
    // fluid (P's own value is the unknown).
    double Cb[3];
    for (int k = 0; k < 3; ++k) Cb[k] = interp(d0[p], k);
    // Eq. (21) with 1 - C_r written as C_g + C_b (reading: negative C's count as 0 and a
    // vanishing denominator gives the mean of the two pair angles).
    double th[2];
    {
      double a = std::max(Cb[1], 0.0), b = std::max(Cb[2], 0.0), den = a + b;
      th[0] = den > 1e-12 ? (b * th13 + a * th12) / den : 0.5 * (th13 + th12);
      double a2 = std::max(Cb[0], 0.0), den2 = a2 + b;
      double th21 = PI - th12;
      th[1] = den2 > 1e-12 ? (b * th23 + a2 * th21) / den2 : 0.5 * (th23 + th21);
    }
    int failbits = 0;
    double CP[3];
    for (int k = 0; k < 2; ++k) {
      double tk = std::min(std::max(th[k], THETA_LO), THETA_HI);
      double phi = std::fabs(0.5 * PI - tk);
      double c = std::cos(phi), s = std::sin(phi);
      Cross l1 = march(i, j, c * nxv + s * tx, c * nyv + s * ty);
      Cross l2 = march(i, j, c * nxv - s * tx, c * nyv - s * ty);
      double v;
      if (l1.ok && l2.ok) {
        double v1 = interp(l1, k), v2 = interp(l2, k);
        v = tk <= 0.5 * PI ? std::max(v1, v2) : std::min(v1, v2);  // Eq. (22)
      } else if (l1.ok) {
        v = interp(l1, k);
      } else if (l2.ok) {
        v = interp(l2, k);
      } else {
        v = Cb[k];
      }
      if (!l1.ok) failbits |= 1 << (2 * k);
      if (!l2.ok) failbits |= 2 << (2 * k);
      CP[k] = v;
    }
    CP[2] = 1.0 - CP[0] - CP[1];
    fill_fail[p] = failbits;
    for (int k = 0; k < 3; ++k) out[3 * p + k] = CP[k];
  }
  // Reading: at solid nodes rho = rho^0 = 1, so the partial densities equal the filled C.
  for (size_t p = 0; p < fill.size(); ++p) {
    int e = fill[p];
    for (int k = 0; k < 3; ++k) C[k * NE + e] = rk[k * NE + e] = out[3 * p + k];
    rho[e] = 1.0;
  }
  // Zou-He ghost columns take the values of the nearest boundary column (zero gradient).
  if (bcx == 2)
    for (int j = 0; j < ny; ++j)
      for (int g = 1; g <= GX; ++g) {
        int el = ext(-g, j), er = ext(nx - 1 + g, j), e0 = ext(0, j), e1 = ext(nx - 1, j);
        for (int k = 0; k < 3; ++k) {
          C[k * NE + el] = C[k * NE + e0];
          rk[k * NE + el] = rk[k * NE + e0];
          C[k * NE + er] = C[k * NE + e1];
          rk[k * NE + er] = rk[k * NE + e1];
        }
        rho[el] = rho[e0];
        rho[er] = rho[e1];
      }
}

// Eq. (10) stress and Eq. (12) colour gradients at every node whose stress is read by a fluid
// node: fluid nodes, C_SB nodes and the Zou-He ghost columns.  Reading: the double sum over
// ordered pairs with the factor 1/2 is taken literally; A_kl = min(max(1e6 rho_k rho_l, 0), 1)
// (equal densities, rho_k^0 = 1).
void Oracle::stresses() {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < NE; ++e) {
    int t = type[e];
    double txx = 0, txy = 0, tyy = 0;
    for (int q = 0; q < 18; ++q) nvec[q * NE + e] = 0.0;
    if (t == T_FLUID || t == T_SB || t == T_GHOST) {
      double gr[3][2];
      for (int k = 0; k < 3; ++k) gradient(&C[k * NE], e, gr[k]);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          if (l == k) continue;
          double Ck = C[k * NE + e], Cl = C[l * NE + e];
          double Gx = Cl * gr[k][0] - Ck * gr[l][0];
          double Gy = Cl * gr[k][1] - Ck * gr[l][1];
          double mag = std::sqrt(Gx * Gx + Gy * Gy);
          double A = std::min(std::max(1e6 * rk[k * NE + e] * rk[l * NE + e], 0.0), 1.0);
          if (mag > EPS_G) {
            double nxk = Gx / mag, nyk = Gy / mag;
            double coef = 0.5 * sig[pair_index(k, l)] * A * mag;
            txx += coef * (1.0 - nxk * nxk);
            txy += coef * (-nxk * nyk);
            tyy += coef * (1.0 - nyk * nyk);
            nvec[((k * 3 + l) * 2 + 0) * NE + e] = nxk;
            nvec[((k * 3 + l) * 2 + 1) * NE + e] = nyk;
          }
        }
    }
    T[0 * NE + e] = txx;
    T[1 * NE + e] = txy;
    T[2 * NE + e] = tyy;
  }
}

// F_s = div T with Eq. (12) applied to the stress components (Eq. 10), at fluid nodes.
void Oracle::forces() {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < NE; ++e) {
    if (type[e] != T_FLUID) {
      Fs[e] = Fs[NE + e] = 0.0;
      continue;
    }
    double fx = 0, fy = 0;
    for (int a = 0; a < 9; ++a) {
      int n = nb[a * NE + e];
      fx += WT[a] * (T[0 * NE + n] * EX[a] + T[1 * NE + n] * EY[a]);
      fy += WT[a] * (T[1 * NE + n] * EX[a] + T[2 * NE + n] * EY[a]);
    }
    Fs[e] = 3.0 * fx;
    Fs[NE + e] = 3.0 * fy;
  }
}

void Oracle::collide_recolour_stream() {
#pragma omp parallel for schedule(static)
  for (int e = 0; e < NE; ++e) {
    if (type[e] != T_FLUID) continue;
    double ftot[9];
    for (int a = 0; a < 9; ++a) ftot[a] = f[a * NE + e] + f[(9 + a) * NE + e] + f[(18 + a) * NE + e];
    double r[3] = {rk[e], rk[NE + e], rk[2 * NE + e]};
    double rt = r[0] + r[1] + r[2];
    double Fx = Fs[e] + rt * gacc[0], Fy = Fs[NE + e] + rt * gacc[1];
    double fdag[9], u[2];
    collide(ftot, r, nu, Fx, Fy, fdag, u);
    U[e] = u[0];
    U[NE + e] = u[1];
    double nk[3][3][2];
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l)
        for (int c = 0; c < 2; ++c) nk[k][l][c] = nvec[((k * 3 + l) * 2 + c) * NE + e];
    double out[27];
    recolour(fdag, r, nk, gX, beta0, out);
    for (int q = 0; q < 27; ++q) fpp[q * NE + e] = out[q];
  }
  // Streaming, Eq. (16), written as a pull: f_{a,k}(x, t+1) = f''_{a,k}(x - e_a, t).
#pragma omp parallel for schedule(static)
  for (int e = 0; e < NE; ++e) {
    if (type[e] != T_FLUID) continue;
    int i = ei(e), j = ej(e);
    bool zh_unknown[9] = {false};
    for (int a = 0; a < 9; ++a) {
      int si = i - EX[a], sj = j - EY[a];
      if (bcx == 2 && (si < 0 || si >= nx)) {
        zh_unknown[a] = true;
        continue;
      }
      bool crossed = bcx == 1 && (si < 0 || si >= nx);
      int s = ext(si, sj);
      if (type[s] == T_FLUID) {
        for (int k = 0; k < 3; ++k) {
          int ks = crossed ? (k == 0 ? 2 : k == 2 ? 0 : 1) : k;  // Sec. III C exchange
          fnew[(k * 9 + a) * NE + e] = fpp[(ks * 9 + a) * NE + s];
        }
        continue;
      }
      // The link x -> x - e_a ends in a solid node.  Reading: the flow condition on curved solids
      // (Bouzidi linear interpolated bounce-back) acts on the total distribution; each fluid's
      // reflected population is its halfway-reflected recoloured population plus its share C_k(x)
      // of the interpolation's change of the total, i.e. Eq. (13) applied at x to the
      // interpolated total.  (Interpolating each fluid's populations instead mixes in the
      // composition of the neighbour and the segregation term of the other direction, which
      // moves the contact line on curved walls off the prescribed angles.)
      double q = qv[a * NE + e];
      int ab = OPP[a];
      int nf = ext(i + EX[a], j + EY[a]);
      auto total = [&](int dir, int node) {
        return fpp[dir * NE + node] + fpp[(9 + dir) * NE + node] + fpp[(18 + dir) * NE + node];
      };
      double v;
      if (q < 0.5 && type[nf] == T_FLUID)
        v = 2.0 * q * total(ab, e) + (1.0 - 2.0 * q) * total(ab, nf);
      else if (q < 0.5)
        v = total(ab, e);
      else
        v = (1.0 / (2.0 * q)) * total(ab, e) + (1.0 - 1.0 / (2.0 * q)) * total(a, e);
      const double dv = v - total(ab, e);
      for (int k = 0; k < 3; ++k) fnew[(k * 9 + a) * NE + e] = fpp[(k * 9 + ab) * NE + e] + C[k * NE + e] * dv;
    }
    if (bcx == 2 && (i == 0 || i == nx - 1)) {
      // Zou-He non-equilibrium bounce-back on the total distribution (Sec. III D).
      double ft[9];
      for (int a = 0; a < 9; ++a)
        ft[a] = zh_unknown[a] ? 0.0 : fnew[a * NE + e] + fnew[(9 + a) * NE + e] + fnew[(18 + a) * NE + e];
      if (i == 0) {
        double ux = u_in;
        double rw = (ft[0] + ft[2] + ft[4] + 2.0 * (ft[3] + ft[6] + ft[7])) / (1.0 - ux);
        ft[1] = ft[3] + 2.0 / 3.0 * rw * ux;
        ft[5] = ft[7] - 0.5 * (ft[2] - ft[4]) + rw * ux / 6.0;
        ft[8] = ft[6] + 0.5 * (ft[2] - ft[4]) + rw * ux / 6.0;
        // Reading: the incoming populations at the inlet carry pure fluid 3.
        for (int a : {1, 5, 8}) {
          fnew[a * NE + e] = 0.0;
          fnew[(9 + a) * NE + e] = 0.0;
          fnew[(18 + a) * NE + e] = ft[a];
        }
      } else {
        double ro = rho_out;
        double ux = -1.0 + (ft[0] + ft[2] + ft[4] + 2.0 * (ft[1] + ft[5] + ft[8])) / ro;
        ft[3] = ft[1] - 2.0 / 3.0 * ro * ux;
        ft[7] = ft[5] + 0.5 * (ft[2] - ft[4]) - ro * ux / 6.0;
        ft[6] = ft[8] - 0.5 * (ft[2] - ft[4]) - ro * ux / 6.0;
        // Reading: the outlet's unknown populations carry the node's own composition.
        for (int a : {3, 6, 7})
          for (int k = 0; k < 3; ++k) fnew[(k * 9 + a) * NE + e] = C[k * NE + e] * ft[a];
      }
    }
  }
  f.swap(fnew);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// C interface used by oracle/pyoracle.py.
extern "C" {

void *orc_create(const orc_domain *d, char *errbuf, int errlen) {
  Oracle *o = new Oracle();
  if (!o->setup(d)) {
    if (errbuf && errlen > 0) snprintf(errbuf, errlen, "%s", o->err.c_str());
    delete o;
    return nullptr;
  }
  return o;
}

void orc_destroy(void *h) { delete static_cast<Oracle *>(h); }

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n < 1 ? 1 : n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_step(void *h, int n) {
  Oracle *o = static_cast<Oracle *>(h);
  for (int s = 0; s < n; ++s) o->step();
}

// Runs the stages that precede collision (densities, fill, stresses, force) on the current
// state without advancing it.
void orc_prepare(void *h) { static_cast<Oracle *>(h)->prepare(); }

// info: nx, ny, GX, PY, NXE, NYE, n_fill, n_sb
void orc_info(void *h, int *out) {
  Oracle *o = static_cast<Oracle *>(h);
  int nsb = 0;
  for (int e : o->fill) nsb += o->type[e] == T_SB;
  int v[8] = {o->nx, o->ny, o->GX, o->PY, o->NXE, o->NYE, (int)o->fill.size(), nsb};
  memcpy(out, v, sizeof v);
}

// Extended-grid fields (rows -PY..ny+PY-1, columns -GX..nx+GX-1):
// which: 0 = C [3], 1 = partial densities [3], 2 = node type [1], 3 = stress [3],
//        4 = F_s [2], 5 = velocity of the last collision [2]
void orc_get_ext(void *h, int which, double *out) {
  Oracle *o = static_cast<Oracle *>(h);
  int NE = o->NE;
  switch (which) {
    case 0: memcpy(out, o->C.data(), sizeof(double) * 3 * NE); break;
    case 1: memcpy(out, o->rk.data(), sizeof(double) * 3 * NE); break;
    case 2: for (int e = 0; e < NE; ++e) out[e] = o->type[e]; break;
    case 3: memcpy(out, o->T.data(), sizeof(double) * 3 * NE); break;
    case 4: memcpy(out, o->Fs.data(), sizeof(double) * 2 * NE); break;
    case 5: memcpy(out, o->U.data(), sizeof(double) * 2 * NE); break;
    default: break;
  }
}

// Per-fluid populations at the in-grid nodes: out[(k*9+a)*ny*nx + i + nx*j].
void orc_get_f(void *h, double *out) {
  Oracle *o = static_cast<Oracle *>(h);
  int n = o->nx * o->ny;
  for (int q = 0; q < 27; ++q)
    for (int j = 0; j < o->ny; ++j)
      for (int i = 0; i < o->nx; ++i) out[q * n + i + o->nx * j] = o->f[q * o->NE + o->ext(i, j)];
}

void orc_set_f(void *h, const double *in) {
  Oracle *o = static_cast<Oracle *>(h);
  int n = o->nx * o->ny;
  for (int q = 0; q < 27; ++q)
    for (int j = 0; j < o->ny; ++j)
      for (int i = 0; i < o->nx; ++i) {
        int e = o->ext(i, j);
        o->f[q * o->NE + e] = o->type[e] == T_FLUID ? in[q * n + i + o->nx * j] : 0.0;
      }
}

// Partial densities sum_a f_{a,k} at in-grid fluid nodes (0 at solid nodes): [3][ny*nx].
void orc_get_rho(void *h, double *out) {
  Oracle *o = static_cast<Oracle *>(h);
  int n = o->nx * o->ny;
  for (int j = 0; j < o->ny; ++j)
    for (int i = 0; i < o->nx; ++i) {
      int e = o->ext(i, j);
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        if (o->type[e] == T_FLUID)
          for (int a = 0; a < 9; ++a) s += o->f[(k * 9 + a) * o->NE + e];
        out[k * n + i + o->nx * j] = s;
      }
    }
}

// Per-fluid mass, summed over fluid nodes in index order.
void orc_mass(void *h, double *out) {
  Oracle *o = static_cast<Oracle *>(h);
  double m[3] = {0, 0, 0};
  for (int e = 0; e < o->NE; ++e) {
    if (o->type[e] != T_FLUID) continue;
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 9; ++a) m[k] += o->f[(k * 9 + a) * o->NE + e];
  }
  memcpy(out, m, sizeof m);
}

// Fill nodes: out[4*p] = i, j, type, fail bits of the last fill; normals in nrm[2*p].
void orc_fill_nodes(void *h, int *out, double *nrm) {
  Oracle *o = static_cast<Oracle *>(h);
  for (size_t p = 0; p < o->fill.size(); ++p) {
    int e = o->fill[p];
    out[4 * p] = o->ei(e);
    out[4 * p + 1] = o->ej(e);
    out[4 * p + 2] = o->type[e];
    out[4 * p + 3] = o->fill_fail[p];
    if (nrm) {
      nrm[2 * p] = o->fnx[p];
      nrm[2 * p + 1] = o->fny[p];
    }
  }
}

double orc_link_q(void *h, int i, int j, int a) {
  Oracle *o = static_cast<Oracle *>(h);
  return o->qv[a * o->NE + o->ext(i, j)];
}

double orc_theta12(void *h) { return static_cast<Oracle *>(h)->th12; }

// Characteristic line from node (i, j) in direction (dx, dy): out = ok, i0, j0, i1, j1; w.
void orc_march(void *h, int i, int j, double dx, double dy, int *out, double *w) {
  Oracle *o = static_cast<Oracle *>(h);
  Cross c = o->march(i, j, dx, dy);
  out[0] = c.ok;
  out[1] = o->ei(c.n0);
  out[2] = o->ej(c.n0);
  out[3] = o->ei(c.n1);
  out[4] = o->ej(c.n1);
  *w = c.w;
}

// Eq. (12) applied to an arbitrary extended-grid field: out[2][NE].
void orc_gradient(void *h, const double *field, double *out) {
  Oracle *o = static_cast<Oracle *>(h);
  for (int e = 0; e < o->NE; ++e) {
    double g[2];
    o->gradient(field, e, g);
    out[e] = g[0];
    out[o->NE + e] = g[1];
  }
}

// ---- single-node building blocks, exposed for the unit pins -------------------------------
void orc_isotropic_sum(const long *block, long *out) { isotropic_sum(block, out); }
void orc_lattice(int *ex, int *ey, double *w) {
  for (int a = 0; a < 9; ++a) {
    ex[a] = EX[a];
    ey[a] = EY[a];
    w[a] = WT[a];
  }
}
void orc_matrix(double *m, double *minv) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      m[9 * i + j] = MM[i][j];
      minv[9 * i + j] = MINV[i][j];
    }
}
void orc_equilibrium(double rho, double ux, double uy, double *out) { equilibrium(rho, ux, uy, out); }
void orc_force_populations(double ux, double uy, double Fx, double Fy, double *out) {
  force_populations(ux, uy, Fx, Fy, out);
}
void orc_relaxation_rates(double tau, double *s) { relaxation_rates(tau, s); }
double orc_relaxation_time(const double *rk, const double *nu) { return relaxation_time(rk, nu); }
void orc_collide(const double *f, const double *rk, const double *nu, double Fx, double Fy,
                 double *fdag, double *u) {
  collide(f, rk, nu, Fx, Fy, fdag, u);
}
double orc_g_of_X(double X) { return g_of_X(X); }
void orc_segregation_X(const double *sig, double *X) { segregation_X(sig, X); }
// n: ordered-pair normals [3][3][2]; gX per unordered pair (12, 13, 23).
void orc_recolour(const double *fdag, const double *rk, const double *n, const double *gX,
                  double beta0, double *out) {
  double nk[3][3][2];
  memcpy(nk, n, sizeof nk);
  recolour(fdag, rk, nk, gX, beta0, out);
}

}  // extern "C"
