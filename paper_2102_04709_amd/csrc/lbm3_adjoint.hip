// lbm3_adjoint.hip -- hand-written adjoint of one step of the three-phase update
// (arXiv:2102.04709, Sec. II).  Given the forward state s_t and the adjoint lambda_{t+1} of the
// state at t+1, it produces lambda_t = (d s_{t+1} / d s_t)^T lambda_{t+1} and accumulates the
// raw parameter partials (d s_{t+1} / d p)^T lambda_{t+1} for p = (sigma12, sigma13, sigma23,
// g(X_12), g(X_13), g(X_23), theta13, theta23, theta12).
//
// Forward intermediates of s_t (on an extended grid, see lbm3_adjoint.h): C_k and rho with the
// filled C at the solid boundary nodes (Eq. 21-22), stress and pair normals (Eq. 10, 12),
// interfacial force, post-collision f' and recolouring vectors R (Eq. 1-9, 11, 13-15).
// Transposes, in reverse order of the forward: streaming (Eq. 16 with every boundary rule, in
// gather form) with the per-node collision + recolouring, the stress divergence (gathered) with
// the per-position stress (reverse-mode products written out from the forward formulas), the
// colour-gradient stencil (atomic scatter), the mass fractions, and the wetting fill (its
// discrete choices -- which
// crossing, which line -- fixed at their forward values).  Non-smooth points (the max/min of
// Eq. 22, clamps, the |G| threshold) take the derivative of the branch the forward took: a
// clamp passes the derivative when its argument lies inside or on the bounds, max/min give it
// to the first operand on ties.
#include <hip/hip_runtime.h>

#include "lbm3_adjoint.h"
#include "lbm3_device.h"
#include "lbm3_internal.h"

namespace lbm3 {

// Hardware floating-point atomic add (the workspace is ordinary coarse-grained device memory).
template <typename T>
__device__ __forceinline__ void aadd(T *p, T v) { unsafeAtomicAdd(p, v); }

// ---- extended grid ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t aidx(const DomainDev &D, int i, int j) { return adj_index(D, i, j); }
// Node whose stored data a read at (i, j) sees (the forward's node_index): periodic axes wrap,
// the Zou-He x axis clamps to the boundary columns, a non-periodic y axis to the off-grid rows.
__device__ __forceinline__ void cmap(const DomainDev &D, int &i, int &j) {
  i = D.bcx == BCX_ZOUHE ? min(max(i, 0), D.nx - 1) : wrap_near(i, D.nx);
  j = D.yper ? wrap_near(j, D.ny) : min(max(j, -2), D.ny + 1);
}
// Position of the stress a divergence at (i, j) reads: periodic axes wrap; the stress at a
// Zou-He ghost column or an off-grid row is its own value (computed there from clamped C).
__device__ __forceinline__ void tmap(const DomainDev &D, int &i, int &j) {
  if (D.bcx != BCX_ZOUHE) i = wrap_near(i, D.nx);
  if (D.yper) j = wrap_near(j, D.ny);
}
// Solid test of a mapped node (rows -2..ny+1 of the flag plane exist).
__device__ __forceinline__ bool solid_at(const uint8_t *flags, const DomainDev &D, int i, int j) {
  return flags[D.base + plane_index(i, j, D.pitch)] & FL_SOLID;
}
__device__ __forceinline__ bool fluid_node(const uint8_t *flags, const DomainDev &D, int i, int j) {
  return i >= 0 && i < D.nx && j >= 0 && j < D.ny && !solid_at(flags, D, i, j);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Sums v[] over the work-group and adds the sums to dst[] (one atomic per value and
// work-group).  Called by every thread of the work-group.
template <int N>
__device__ __forceinline__ void block_add(const double (&v)[N], double *dst) {
  __shared__ double red[N][kThreads / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) s += red[threadIdx.x][q];
    if (s != 0.0) aadd(dst + threadIdx.x, s);
  }
}

// Node (i, j) of the 32 x 8 tile handled by this thread.
// Work item of this work-group: consecutive items go to the same XCD (gfx950 dispatches
// work-group b to XCD b mod 8), so the tiles an XCD processes are contiguous and share their halo
// rows in that XCD's L2.  The grid is a multiple of 8; the padding groups have no item (-1).
// per: the groups per XCD (grid / 8), given by the launch as a scalar argument, which the
// compiler preloads into registers with the kernel's other leading arguments (work, doms, n_work:
// the fields of AdjArgs that locate the first tile, whose copies in AdjArgs are not read).
__device__ __forceinline__ int adj_item(int n_work, int per) {
  const int wi = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  return wi < n_work ? wi : -1;
}

// The adjoint kernels' tiles are 32 x 8 nodes, one per thread of a 256-thread work-group; the
// node kernel stages lambda_{t+1} of the tile + 1 ring in LDS.
constexpr int kAdjTX = 32, kAdjTY = 8, kAdjW1 = kAdjTX + 2, kAdjN1 = kAdjW1 * (kAdjTY + 2);
static_assert(kAdjTX * kAdjTY == kThreads, "one adjoint tile node per thread");

__device__ __forceinline__ bool tile_node(const WorkItem &wk, int &i, int &j) {
  i = wk.x0 + (threadIdx.x & 31);
  j = wk.y0 + (threadIdx.x >> 5);
  return i < wk.x1 && j < wk.y1;
}

template <typename T>
__device__ __forceinline__ T &XP(T *X, int64_t AP, int plane, int64_t q) { return X[plane * AP + q]; }

// ---- helpers of the transposes -----------------------------------------------------------
template <typename T>
__device__ __forceinline__ void c9_at(const T *X, int64_t AP, const DomainDev &D, int i, int j, int k, T c9[9]) {
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    int ii = i + lat_ex(a), jj = j + lat_ey(a);
    cmap(D, ii, jj);
    c9[a] = X[(AX_C + k) * AP + aidx(D, ii, jj)];
  }
}

// ---- transposes ----------------------------------------------------------------------------
// Zou-He at a boundary node y (Eq. 16 with the Zou-He rule): the unknown totals are affine in
// the known ones, so the adjoint of a known population d of y gains a term from the adjoints of
// the unknown populations (and, at the outlet, of the partial densities they carry).
template <typename T>
__device__ __forceinline__ T zh_add(const DomainDev &D, bool inlet, int d, const T *Lf, const T *Lr, int64_t yli,
                                    const T Cy[3]) {
  const int64_t P = D.plane;
  if (inlet) {
    const T u = (T)D.u_in;
    const T ir = T(1) / (T(1) - u);
    const T l1 = Lf[1 * P + yli] + Lr[2 * P + yli];  // the inflow is fluid 3
    const T l5 = Lf[5 * P + yli] + Lr[2 * P + yli];
    const T l8 = Lf[8 * P + yli] + Lr[2 * P + yli];
    const T lw = (T(2.0 / 3.0) * l1 + (l5 + l8) / T(6)) * u;
    // d rho_w / d ft_d: ft0, ft2, ft4 once, ft3, ft6, ft7 twice
    T add = lw * ir * (d == 3 || d == 6 || d == 7 ? T(2) : (d == 0 || d == 2 || d == 4 ? T(1) : T(0)));
    if (d == 3) add += l1;
    if (d == 7) add += l5;
    if (d == 6) add += l8;
    if (d == 2) add += T(0.5) * (l8 - l5);
    if (d == 4) add += T(0.5) * (l5 - l8);
    return add;
  }
  const T mc = Lr[yli] * Cy[0] + Lr[P + yli] * Cy[1] + Lr[2 * P + yli] * Cy[2];
  const T l3 = Lf[3 * P + yli] + mc, l6 = Lf[6 * P + yli] + mc, l7 = Lf[7 * P + yli] + mc;
  const T lw = -(T(2.0 / 3.0) * l3 + (l7 + l6) / T(6));
  // d (rho_out u_x) / d ft_d: ft0, ft2, ft4 once, ft1, ft5, ft8 twice
  T add = lw * (d == 1 || d == 5 || d == 8 ? T(2) : (d == 0 || d == 2 || d == 4 ? T(1) : T(0)));
  if (d == 1) add += l3;
  if (d == 5) add += l7;
  if (d == 8) add += l6;
  if (d == 2) add += T(0.5) * (l7 - l6);
  if (d == 4) add += T(0.5) * (l6 - l7);
  return add;
}

// Adjoint of streaming in gather form: each fluid node x collects the adjoints of its own
// post-collision data f'_d(x) and R(x) (and of its C through the recoloured parts) from every
// read of them in the forward pull:
//   - the node y = x + e_d pulls f'_d(x) (populations crossing the fluid-exchanging boundary
//     swap the adjoints of fluids 1 and 3; a Zou-He node adds the unknowns' dependence);
//   - the same y, when its link opposite to d is cut with q < 1/2 and x + 2 e_d is solid, reads
//     f'_d(x) again with weight 1 - 2q (interpolated bounce-back);
//   - x itself, for each of its own solid links (halfway or interpolated bounce-back).
// No atomics: every adjoint of x's data is written by x's thread, which then applies the
// collision transpose to them at once (adj_node).
// Post-collision shifted population f'_dir of the fluid node (i, j) (mapped) that the interpolated
// bounce-back of a neighbour reads: the intermediates kernel stores the post-collision populations
// of such nodes (flag FL_IBBSRC), formed with the forward's own collision.
template <typename S, typename T>
__device__ __forceinline__ T nb_post_collision(const AdjArgs<S, T> &A, const DomainDev &D, int i, int j, int dir) {
  cmap(D, i, j);
  return A.X[(AX_P + dir) * A.aplane + aidx(D, i, j)];
}

template <typename S, typename T>
__device__ __forceinline__ void stream_gather(const AdjArgs<S, T> &A, const DomainDev &D, const KT<T> &K, int i, int j,
                                              int64_t tplane, const T fp[9], const T (*sL)[kAdjN1], T lP[13],
                                              T lC[3]) {
  // sL[c][p]: lambda_{t+1} (9 distributions, 3 densities) of the node read at tile position p of the
  // ring-1 block; the node itself is at p0
  const int p0 = (int)(threadIdx.x & (kAdjTX - 1)) + 1 + ((int)(threadIdx.x / kAdjTX) + 1) * kAdjW1;
  const int64_t AP = A.aplane;
  const int64_t li = plane_index(i, j, D.pitch);
  const int64_t q = aidx(D, i, j);
  const T *Lf = A.lin + 9 * D.base;
  const T *Lr = A.lin + 9 * tplane + 3 * D.base;
  const bool zh = D.bcx == BCX_ZOUHE;
  const T C[3] = {A.X[AX_C * AP + q], A.X[(AX_C + 1) * AP + q], A.X[(AX_C + 2) * AP + q]};
  const uint32_t lk = A.links[D.base + li];
#pragma unroll
  for (int c = 0; c < 13; ++c) lP[c] = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) lC[c] = T(0);
  // a read of f'_dir(x) with weight coef into a node whose total has adjoint lfv and whose
  // partial densities have adjoints m[3] (the recoloured part k is C_k (f' + w) + w R_k.e)
  auto take = [&](int dir, T coef, T lfv, T m0, T m1, T m2) {
    const T w = wgt<T>(dir);
    const int ex = lat_ex(dir), ey = lat_ey(dir);
    lP[dir] += coef * (lfv + m0 * C[0] + m1 * C[1] + m2 * C[2]);
    const T fw = coef * (fp[dir] + w);
    lC[0] += m0 * fw;
    lC[1] += m1 * fw;
    lC[2] += m2 * fw;
    const T a = coef * w * (m0 - m2), b = coef * w * (m1 - m2);
    if (ex) {
      lP[9] += a * T(ex);
      lP[11] += b * T(ex);
    }
    if (ey) {
      lP[10] += a * T(ey);
      lP[12] += b * T(ey);
    }
  };
#pragma unroll
  for (int d = 0; d < 9; ++d) {
    const int ex = lat_ex(d), ey = lat_ey(d);
    const int yx = i + ex;
    if (zh && (yx < 0 || yx >= D.nx)) continue;  // nothing is pulled out through a Zou-He boundary
    if ((lk >> d) & 1) continue;
    int yi = yx, yj = j + ey;
    cmap(D, yi, yj);
    const int64_t yli = plane_index(yi, yj, D.pitch);
    const int py = p0 + ex + ey * kAdjW1;
    T lfv = sL[d][py];
    const T m0 = sL[9][py], m1 = sL[10][py], m2 = sL[11][py];
    if (zh && (yi == 0 || yi == D.nx - 1)) {
      const int64_t yq = aidx(D, yi, yj);
      const T Cy[3] = {A.X[AX_C * AP + yq], A.X[(AX_C + 1) * AP + yq], A.X[(AX_C + 2) * AP + yq]};
      lfv += zh_add(D, yi == 0, d, Lf, Lr, yli, Cy);
    }
    const bool crossed = D.bcx == BCX_SWAP13 && (yx < 0 || yx >= D.nx);
    if (crossed) take(d, T(1), lfv, m2, m1, m0);
    else take(d, T(1), lfv, m0, m1, m2);
    if (d != 0 && ((lk >> (9 + d)) & 1) && D.n_ibb > 0) {
      if ((lk >> (18 + d)) & 1) {
        // y's link opposite to d is cut with the fluid node x behind it: y's interpolated total
        // reads f'_d(x) with weight 1 - 2q, and each fluid of y takes its share C_k(y) of it
        const int a = lat_opp(d);
        const T qa = (T)A.ibb[A.ibb_of[D.base + yli]].q[a - 1];
        if (qa < T(0.5)) {
          const int64_t yq = aidx(D, yi, yj);
          const T gy = sL[a][py] + m0 * A.X[AX_C * AP + yq] + m1 * A.X[(AX_C + 1) * AP + yq] +
                       m2 * A.X[(AX_C + 2) * AP + yq];
          lP[d] += (T(1) - T(2) * qa) * gy;
        }
      }
    }
  }
  // own solid links
  const IbbNode *ib = (((lk >> 27) & 1) && D.n_ibb > 0) ? A.ibb + A.ibb_of[D.base + li] : nullptr;
  const T mu0 = sL[9][p0], mu1 = sL[10][p0], mu2 = sL[11][p0];
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    const int sx = i - ex;
    if (zh && (sx < 0 || sx >= D.nx)) continue;
    const int ab = lat_opp(a);
    if (!((lk >> ab) & 1)) continue;  // the node read at x - e_a is fluid
    const T qd = ib ? (T)ib->q[a - 1] : T(0.5);
    // forward: f_a(x) = v (the interpolated total), rho_k(x) += [C_k (f'_ab + w) + w R_k.e_ab] +
    // C_k (v - f'_ab): v's adjoint gathers lambda_fa + sum_k mu_k C_k, C_k's gathers mu_k (v + w),
    // R's the halfway term's
    const T g = sL[a][p0] + mu0 * C[0] + mu1 * C[1] + mu2 * C[2];
    T v;
    if (qd < T(0.5) && !((lk >> a) & 1)) {
      const T c1 = T(2) * qd, c2 = T(1) - T(2) * qd;
      v = c1 * fp[ab] + c2 * nb_post_collision(A, D, i + ex, j + ey, ab);
      lP[ab] += c1 * g;  // (the neighbour's share is gathered there)
    } else if (qd < T(0.5)) {
      v = fp[ab];
      lP[ab] += g;
    } else {
      const T c1 = rcp(T(2) * qd), c2 = T(1) - c1;
      v = c1 * fp[ab] + c2 * fp[a];
      lP[ab] += c1 * g;
      lP[a] += c2 * g;
    }
    const T w = wgt<T>(ab);
    const T vw = v + w;
    lC[0] += mu0 * vw;
    lC[1] += mu1 * vw;
    lC[2] += mu2 * vw;
    const T ra_ = w * (mu0 - mu2), rb_ = w * (mu1 - mu2);
    const int bx = lat_ex(ab), by = lat_ey(ab);
    if (bx) {
      lP[9] += ra_ * T(bx);
      lP[11] += rb_ * T(bx);
    }
    if (by) {
      lP[10] += ra_ * T(by);
      lP[12] += rb_ * T(by);
    }
  }
  if (zh && i == D.nx - 1) {
    // the outflowing unknowns carry the node's own composition: d ra_k / d C_k = f3 + f6 + f7
    T ft[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const int sx = i - lat_ex(a);
      int ii = sx, jj = j - lat_ey(a);
      cmap(D, ii, jj);
      ft[a] = sx >= D.nx ? T(0) : A.X[(AX_P + a) * AP + aidx(D, ii, jj)] + wgt<T>(a);
    }
    const T ro = (T)D.rho_out;
    const T ux = -T(1) + (ft[0] + ft[2] + ft[4] + T(2) * (ft[1] + ft[5] + ft[8])) / ro;
    const T f3 = ft[1] - T(2.0 / 3.0) * ro * ux;
    const T f7 = ft[5] + T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
    const T f6 = ft[8] - T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
    const T su = f3 + f6 + f7;
    lC[0] += mu0 * su;
    lC[1] += mu1 * su;
    lC[2] += mu2 * su;
  }
}

// Reverse-mode product of collide_shifted (Eq. 1-9, 11) followed by recolour_R (Eq. 13-15):
// given the adjoints lfd[9] of the post-collision shifted populations and lR[4] of the
// recolouring vectors, returns the adjoints of the inputs f[9], the interfacial force (lFx, lFy),
// the mass fractions C[3] and total density rt (r_k = C_k rt), the pair normals n[6] and the
// factors g(X_kl)[3].  The forward intermediates are recomputed in the same order.
template <typename T>
__device__ __forceinline__ void collide_recolour_vjp(const T f[9], T Fxi, T Fyi, const T C[3], T rt, const T nrm[6],
                                                     const KT<T> &K, const T lfd[9], const T lR[4], T lf[9],
                                                     T &lFx, T &lFy, T lC[3], T &lrt, T ln[6], T lgX[3]) {
  const T r0 = C[0] * rt, r1 = C[1] * rt, r2 = C[2] * rt;
  // ---- forward of the collision
  const T s14 = f[1] + f[2] + f[3] + f[4], s58 = f[5] + f[6] + f[7] + f[8];
  const T drho = f[0] + s14 + s58;
  const T m1 = -T(4) * f[0] - s14 + T(2) * s58;
  const T m2 = T(4) * f[0] - T(2) * s14 + s58;
  const T jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  const T m4 = -T(2) * f[1] + T(2) * f[3] + f[5] - f[6] - f[7] + f[8];
  const T jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  const T m6 = -T(2) * f[2] + T(2) * f[4] + f[5] + f[6] - f[7] - f[8];
  const T m7 = f[1] - f[2] + f[3] - f[4];
  const T m8 = f[5] - f[6] + f[7] - f[8];
  const T rho = T(1) + drho;
  const T Fx = Fxi + rho * K.g0, Fy = Fyi + rho * K.g1;
  const T irho = rcp(rho);
  const T ux = (jx + T(0.5) * Fx) * irho, uy = (jy + T(0.5) * Fy) * irho;
  const T sum = r0 * K.inu[0] + r1 * K.inu[1] + r2 * K.inu[2];
  const T den1 = T(0.5) * sum + T(3);
  const T s1 = sum * rcp(den1);
  const T s4 = T(8) * (T(2) - s1) * rcp(T(8) - s1);
  const T ruu = rho * (ux * ux + uy * uy);
  const T uF = ux * Fx + uy * Fy;
  const T h1 = T(1) - T(0.5) * s1, h4 = T(1) - T(0.5) * s4;
  const T A1 = m1 + T(2) * drho - T(3) * ruu, A2 = m2 - drho + T(3) * ruu;
  const T A4 = m4 + rho * ux, A6 = m6 + rho * uy;
  const T Pxy = ux * ux - uy * uy, A7 = m7 - rho * Pxy;
  const T A8 = m8 - rho * ux * uy;
  const T Q7 = ux * Fx - uy * Fy, Q8 = ux * Fy + uy * Fx;
  // ---- adjoint: fd = f - M^T d, so ld_i = -(M lfd)_i
  const T L0 = lfd[0], L1 = lfd[1], L2 = lfd[2], L3 = lfd[3], L4 = lfd[4];
  const T L5 = lfd[5], L6 = lfd[6], L7 = lfd[7], L8 = lfd[8];
  const T q14 = L1 + L2 + L3 + L4, q58 = L5 + L6 + L7 + L8;
  const T ld1 = -(-T(4) * L0 - q14 + T(2) * q58);
  const T ld2 = -(T(4) * L0 - T(2) * q14 + q58);
  const T ld3 = -(L1 - L3 + L5 - L6 - L7 + L8);
  const T ld4 = -(-T(2) * L1 + T(2) * L3 + L5 - L6 - L7 + L8);
  const T ld5 = -(L2 - L4 + L5 + L6 - L7 - L8);
  const T ld6 = -(-T(2) * L2 + T(2) * L4 + L5 + L6 - L7 - L8);
  const T ld7 = -(L1 - L2 + L3 - L4);
  const T ld8 = -(L5 - L6 + L7 - L8);
  // d1 = (s1 A1 - 6 h1 uF)/36, d2 = (s1 A2 + 6 h1 uF)/36, d3 = -Fx/6, d4 = (s4 A4 + h4 Fx)/12,
  // d5 = -Fy/6, d6 = (s4 A6 + h4 Fy)/12, d7 = (s1 A7 - 2 h1 Q7)/4, d8 = (s1 A8 - h1 Q8)/4
  const T e1 = ld1 * T(1.0 / 36.0), e2 = ld2 * T(1.0 / 36.0), e4 = ld4 * T(1.0 / 12.0);
  const T e6 = ld6 * T(1.0 / 12.0), e7 = ld7 * T(0.25), e8 = ld8 * T(0.25);
  T ls1 = e1 * A1 + e2 * A2 + e7 * A7 + e8 * A8;
  T ls4 = e4 * A4 + e6 * A6;
  const T lh1 = T(6) * uF * (e2 - e1) - T(2) * Q7 * e7 - Q8 * e8;
  const T lh4 = Fx * e4 + Fy * e6;
  const T luF = T(6) * h1 * (e2 - e1);
  const T lA1 = s1 * e1, lA2 = s1 * e2, lA4 = s4 * e4, lA6 = s4 * e6, lA7 = s1 * e7, lA8 = s1 * e8;
  const T lQ7 = -T(2) * h1 * e7, lQ8 = -h1 * e8;
  T lFxt = -ld3 * T(1.0 / 6.0) + h4 * e4;
  T lFyt = -ld5 * T(1.0 / 6.0) + h4 * e6;
  const T lruu = T(3) * (lA2 - lA1);
  T ldrho = T(2) * lA1 - lA2;
  T lrho = ux * lA4 + uy * lA6 - Pxy * lA7 - ux * uy * lA8 + (ux * ux + uy * uy) * lruu;
  const T lPxy = -rho * lA7;
  T lux = rho * lA4 - rho * uy * lA8 + Fx * lQ7 + Fy * lQ8 + T(2) * ux * lPxy + Fx * luF + T(2) * rho * ux * lruu;
  T luy = rho * lA6 - rho * ux * lA8 - Fy * lQ7 + Fx * lQ8 - T(2) * uy * lPxy + Fy * luF + T(2) * rho * uy * lruu;
  lFxt += ux * lQ7 + uy * lQ8 + ux * luF;
  lFyt += -uy * lQ7 + ux * lQ8 + uy * luF;
  // h = 1 - s/2; s4 = 8 (2 - s1) / (8 - s1); s1 = sum / (sum/2 + 3)
  ls1 += -T(0.5) * lh1;
  ls4 += -T(0.5) * lh4;
  const T i8 = rcp(T(8) - s1);
  ls1 += ls4 * (-T(48) * i8 * i8);
  const T id1 = rcp(den1);
  const T lsum = ls1 * T(3) * id1 * id1;
  // u = (j + F/2) / rho
  const T ljx = lux * irho, ljy = luy * irho;
  lFxt += T(0.5) * lux * irho;
  lFyt += T(0.5) * luy * irho;
  const T lirho = lux * (jx + T(0.5) * Fx) + luy * (jy + T(0.5) * Fy);
  lrho += -lirho * irho * irho;
  // F = F_s + rho g
  lFx = lFxt;
  lFy = lFyt;
  lrho += K.g0 * lFxt + K.g1 * lFyt;
  ldrho += lrho;
  // moments back to the populations: lf = lfd + M^T (ldrho, lm1, lm2, ljx, lm4, ljy, lm6, lm7, lm8)
  const T lm1 = lA1, lm2 = lA2, lm4 = lA4, lm6 = lA6, lm7 = lA7, lm8 = lA8;
  lf[0] = L0 + ldrho - T(4) * lm1 + T(4) * lm2;
  lf[1] = L1 + ldrho - lm1 - T(2) * lm2 + ljx - T(2) * lm4 + lm7;
  lf[2] = L2 + ldrho - lm1 - T(2) * lm2 + ljy - T(2) * lm6 - lm7;
  lf[3] = L3 + ldrho - lm1 - T(2) * lm2 - ljx + T(2) * lm4 + lm7;
  lf[4] = L4 + ldrho - lm1 - T(2) * lm2 - ljy + T(2) * lm6 - lm7;
  lf[5] = L5 + ldrho + T(2) * lm1 + lm2 + ljx + lm4 + ljy + lm6 + lm8;
  lf[6] = L6 + ldrho + T(2) * lm1 + lm2 - ljx - lm4 + ljy + lm6 - lm8;
  lf[7] = L7 + ldrho + T(2) * lm1 + lm2 - ljx - lm4 - ljy - lm6 + lm8;
  lf[8] = L8 + ldrho + T(2) * lm1 + lm2 + ljx + lm4 - ljy - lm6 - lm8;
  // ---- recolouring vectors
  const T irt = rcp(rt);
  const T P = T(35) * r0 * r1 * r2 * irt * irt * irt;
  const T r3 = fmin(fmax(P, T(0)), T(1));
  const T b0 = K.b0;
  const T b12 = b0 + b0 * r3 * K.gX[0], b13 = b0 + b0 * r3 * K.gX[1], b23 = b0 + b0 * r3 * K.gX[2];
  const T a12 = b12 * r0 * r1 * irt, a13 = b13 * r0 * r2 * irt, a23 = b23 * r1 * r2 * irt;
  const T la12 = (lR[0] - lR[2]) * nrm[0] + (lR[1] - lR[3]) * nrm[1];
  const T la13 = lR[0] * nrm[2] + lR[1] * nrm[3];
  const T la23 = lR[2] * nrm[4] + lR[3] * nrm[5];
  ln[0] = (lR[0] - lR[2]) * a12;
  ln[1] = (lR[1] - lR[3]) * a12;
  ln[2] = lR[0] * a13;
  ln[3] = lR[1] * a13;
  ln[4] = lR[2] * a23;
  ln[5] = lR[3] * a23;
  const T lb12 = la12 * r0 * r1 * irt, lb13 = la13 * r0 * r2 * irt, lb23 = la23 * r1 * r2 * irt;
  T lr0 = lsum * K.inu[0] + (la12 * b12 * r1 + la13 * b13 * r2) * irt;
  T lr1 = lsum * K.inu[1] + (la12 * b12 * r0 + la23 * b23 * r2) * irt;
  T lr2 = lsum * K.inu[2] + (la13 * b13 * r0 + la23 * b23 * r1) * irt;
  T lirt = la12 * b12 * r0 * r1 + la13 * b13 * r0 * r2 + la23 * b23 * r1 * r2;
  lgX[0] = b0 * r3 * lb12;
  lgX[1] = b0 * r3 * lb13;
  lgX[2] = b0 * r3 * lb23;
  const T lr3 = b0 * (lb12 * K.gX[0] + lb13 * K.gX[1] + lb23 * K.gX[2]);
  const T lP = (P >= T(0) && P <= T(1)) ? lr3 : T(0);
  const T i3 = irt * irt * irt;
  lr0 += lP * T(35) * r1 * r2 * i3;
  lr1 += lP * T(35) * r0 * r2 * i3;
  lr2 += lP * T(35) * r0 * r1 * i3;
  lirt += lP * T(105) * r0 * r1 * r2 * irt * irt;
  // r_k = C_k rt
  lC[0] = lr0 * rt;
  lC[1] = lr1 * rt;
  lC[2] = lr2 * rt;
  lrt = lr0 * C[0] + lr1 * C[1] + lr2 * C[2] - lirt * irt * irt;
}

// Adjoint of streaming and of the per-node collision and recolouring, node by node.  At solid
// positions of the grid it clears the adjoint of C (the stress and stencil transposes add there).
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_node(const WorkItem *__restrict__ work, const DomainDev *__restrict__ doms, int n_work, int per, 
                                                     AdjArgs<S, T> A, int64_t tplane) {
  __shared__ T sL[12][kAdjN1];
  const int wi = adj_item(n_work, per);
  if (wi < 0) return;
  const WorkItem wk = work[wi];
  const DomainDev &D = doms[wk.dom];
  int i, j;
  double graw[3] = {0, 0, 0};
  const int64_t AP = A.aplane;
  {  // lambda_{t+1} of the tile + 1 ring, at the nodes the reads there see
    const T *Lf = A.lin + 9 * D.base;
    const T *Lr = A.lin + 9 * tplane + 3 * D.base;
    for (int p = threadIdx.x; p < kAdjN1; p += kThreads) {
      int gi = wk.x0 - 1 + p % kAdjW1, gj = wk.y0 - 1 + p / kAdjW1;
      if (gi > wk.x1 || gj > wk.y1) continue;  // beyond the ring of a partial tile (never read)
      cmap(D, gi, gj);
      const int64_t gl = plane_index(gi, gj, D.pitch);
#pragma unroll
      for (int c = 0; c < 9; ++c) sL[c][p] = Lf[c * D.plane + gl];
#pragma unroll
      for (int c = 0; c < 3; ++c) sL[9 + c][p] = Lr[c * D.plane + gl];
    }
  }
  __syncthreads();
  if (tile_node(wk, i, j) && i >= 0 && i < D.nx) {
    const int64_t q = aidx(D, i, j);
    if (!fluid_node(A.flags, D, i, j)) {  // (the output's distributions are zero at solid positions)
#pragma unroll
      for (int c = 0; c < 4; ++c) A.X[(AL_C + c) * AP + q] = T(0);
      const int64_t li = plane_index(i, j, D.pitch);
#pragma unroll
      for (int a = 0; a < 9; ++a) A.lout[9 * D.base + a * D.plane + li] = T(0);
    } else {
      const int64_t li = plane_index(i, j, D.pitch);
      const KT<T> K = make_kt<T>(D);
      T f[9], C[3], nrm[6];
#pragma unroll
      for (int a = 0; a < 9; ++a) f[a] = load_s<S, T>(A.fin + 9 * D.base + a * D.plane + li);
#pragma unroll
      for (int c = 0; c < 3; ++c) C[c] = A.X[(AX_C + c) * AP + q];
      const T rt = A.X[(AX_C + 3) * AP + q];
      T fd[9];  // the node's post-collision populations, recomputed as the forward step formed them
      {
        T Fx = A.X[AX_F * AP + q], Fy = A.X[(AX_F + 1) * AP + q], ux, uy;
        collide_shifted(f, Fx, Fy, C[0] * rt, C[1] * rt, C[2] * rt, K, fd, ux, uy);
      }
      T lP[13], lCs[3];
      stream_gather(A, D, K, i, j, tplane, fd, sL, lP, lCs);
#pragma unroll
      for (int c = 0; c < 6; ++c) nrm[c] = A.X[(AX_N + c) * AP + q];
      T lf[9], lFx, lFy, lC[3], lrt, ln[6], lgX[3];
      collide_recolour_vjp(f, A.X[AX_F * AP + q], A.X[(AX_F + 1) * AP + q], C, rt, nrm, K, lP, lP + 9, lf, lFx, lFy,
                           lC, lrt, ln, lgX);
#pragma unroll
      for (int a = 0; a < 9; ++a) A.lout[9 * D.base + a * D.plane + li] = lf[a];
      A.X[AL_F * AP + q] = lFx;
      A.X[(AL_F + 1) * AP + q] = lFy;
#pragma unroll
      for (int c = 0; c < 3; ++c) A.X[(AL_C + c) * AP + q] = lC[c] + lCs[c];
      A.X[(AL_C + 3) * AP + q] = lrt;
#pragma unroll
      for (int c = 0; c < 6; ++c) A.X[(AL_N + c) * AP + q] = ln[c];
#pragma unroll
      for (int c = 0; c < 3; ++c) graw[c] = (double)lgX[c];
    }
  }
  block_add(graw, A.raw + 9 * wk.dom + 3);
}

// Reverse-mode product of pair_stress (Eq. 10 with the normals of Eq. 13): given the adjoints of
// the stress (lt[3]) and of the pair normals (ln[6]), accumulates the adjoints of C[3], of the
// colour gradients g[3][2], of rho and of the tensions sigma[3].
// Where |G_kl| < eps_n the normal is treated as locally constant (its derivative dropped).
template <typename T>
__device__ __forceinline__ void pair_stress_vjp(const T cc[3], const T g[3][2], T rho, const T sig[3], T eps,
                                                T eps_n, const T lt[3], const T ln[6], T lc[3], T lg[3][2],
                                                T &lrho, T lsig[3]) {
  const int pk[3] = {0, 0, 1}, pl[3] = {1, 2, 2};
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int k = pk[pr], l = pl[pr];
    lsig[pr] = T(0);
    const T Gx = cc[l] * g[k][0] - cc[k] * g[l][0];
    const T Gy = cc[l] * g[k][1] - cc[k] * g[l][1];
    T mag, im;
    if (!pair_norm(Gx, Gy, eps, mag, im)) continue;  // stress and normal are zero there
    const T rk = cc[k] * rho, rl = cc[l] * rho;
    const T Q = T(1e6) * rk * rl;
    const T Akl = fmin(fmax(Q, T(0)), T(1));
    const T nx = Gx * im, ny = Gy * im;
    const T S = sig[pr] * Akl;
    // T_pair = S (Gy^2, -Gx Gy, Gx^2) / |G|
    const T X = lt[0] * Gy * Gy - lt[1] * Gx * Gy + lt[2] * Gx * Gx;
    const T lS = X * im;
    T lGx = S * (T(2) * lt[2] * Gx - lt[1] * Gy) * im;
    T lGy = S * (T(2) * lt[0] * Gy - lt[1] * Gx) * im;
    const T lmag = -S * lS * im;
    lGx += lmag * nx;
    lGy += lmag * ny;
    // n = G / |G|: lG += (ln - n (n . ln)) / |G|
    const T lnx = ln[2 * pr], lny = ln[2 * pr + 1];
    const T nl = nx * lnx + ny * lny;
    if (mag > eps_n) {
      lGx += (lnx - nx * nl) * im;
      lGy += (lny - ny * nl) * im;
    }
    lsig[pr] = lS * Akl;
    const T lQ = (Q >= T(0) && Q <= T(1)) ? lS * sig[pr] : T(0);
    const T lrk = T(1e6) * rl * lQ, lrl = T(1e6) * rk * lQ;
    lc[k] += lrk * rho;
    lc[l] += lrl * rho;
    lrho += lrk * cc[k] + lrl * cc[l];
    // G = C_l g_k - C_k g_l
    lc[l] += lGx * g[k][0] + lGy * g[k][1];
    lc[k] -= lGx * g[l][0] + lGy * g[l][1];
    lg[k][0] += lGx * cc[l];
    lg[k][1] += lGy * cc[l];
    lg[l][0] -= lGx * cc[k];
    lg[l][1] -= lGy * cc[k];
  }
}

// Adjoint of the stress divergence and of the per-position stress and normals.  The stress at
// position z is read by the divergence F(y) = 3 sum_a w_a T(y + e_a) . e_a (Eq. 12 on Eq. 10)
// of the fluid nodes y = z - e_a (periodic axes wrap, other axes do not), so the adjoint of the
// stress at z is gathered from their adjoint forces; the normals at z matter only at fluid nodes.
// The adjoint of the colour gradients at z then goes through the transpose of the Eq. (12)
// stencil: an atomic scatter to the adjoint of C at the (clamped / wrapped) nodes z + e_a.
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_stress(const WorkItem *__restrict__ work, const DomainDev *__restrict__ doms, int n_work, int per, 
                                                       AdjArgs<S, T> A) {
  __shared__ T sC[3][kAdjN1];       // C_k at the nodes the ring-1 block's reads see
  __shared__ T sF[2][kAdjN1];       // adjoint force at the block's (wrapped) positions, fluid only
  __shared__ uint8_t sFl[kAdjN1];   // whether that position is a fluid node
  const int wi = adj_item(n_work, per);
  if (wi < 0) return;
  const WorkItem wk = work[wi];
  const DomainDev &D = doms[wk.dom];
  const int64_t AP = A.aplane;
  for (int p = threadIdx.x; p < kAdjN1; p += kThreads) {
    const int gi = wk.x0 - 1 + p % kAdjW1, gj = wk.y0 - 1 + p / kAdjW1;
    if (gi > wk.x1 || gj > wk.y1) continue;  // beyond the ring of a partial tile (never read)
    int ci = gi, cj = gj;
    cmap(D, ci, cj);
    const int64_t qc = aidx(D, ci, cj);
#pragma unroll
    for (int k = 0; k < 3; ++k) sC[k][p] = A.X[(AX_C + k) * AP + qc];
    int yi = gi, yj = gj;
    if (D.bcx != BCX_ZOUHE) yi = wrap_near(yi, D.nx);
    if (D.yper) yj = wrap_near(yj, D.ny);
    const bool fl = fluid_node(A.flags, D, yi, yj);
    sFl[p] = fl;
    if (fl) {
      const int64_t y = aidx(D, yi, yj);
      sF[0][p] = A.X[AL_F * AP + y];
      sF[1][p] = A.X[(AL_F + 1) * AP + y];
    }
  }
  __syncthreads();
  const int p0 = (int)(threadIdx.x & (kAdjTX - 1)) + 1 + ((int)(threadIdx.x / kAdjTX) + 1) * kAdjW1;
  int i, j;
  double sraw[3] = {0, 0, 0};
  if (tile_node(wk, i, j)) {
    const int64_t q = aidx(D, i, j);
    T lt[3] = {T(0), T(0), T(0)}, ln[6];
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      const int ex = lat_ex(a), ey = lat_ey(a);
      const int py = p0 - ex - ey * kAdjW1;  // y = z - e_a
      if (!sFl[py]) continue;
      const T lx = sF[0][py], ly = sF[1][py];
      const T c = T(3) * wgt<T>(a);
      lt[0] += c * T(ex) * lx;
      lt[1] += c * (T(ey) * lx + T(ex) * ly);
      lt[2] += c * T(ey) * ly;
    }
    const bool fluid = fluid_node(A.flags, D, i, j);
#pragma unroll
    for (int c = 0; c < 6; ++c) ln[c] = fluid ? A.X[(AL_N + c) * AP + q] : T(0);
    bool any = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) any |= lt[c] != T(0);
#pragma unroll
    for (int c = 0; c < 6; ++c) any |= ln[c] != T(0);
    if (any) {
      int ci = i, cj = j;
      cmap(D, ci, cj);
      const int64_t qc = aidx(D, ci, cj);
      T cc[3], g[3][2];
#pragma unroll
      for (int c = 0; c < 3; ++c) cc[c] = sC[c][p0];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T c9[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) c9[a] = sC[k][p0 + lat_ex(a) + lat_ey(a) * kAdjW1];
        grad9(c9, g[k][0], g[k][1]);
      }
      const T rho = A.X[(AX_C + 3) * AP + qc];
      const T sig[3] = {(T)D.sig[0], (T)D.sig[1], (T)D.sig[2]};
      T lc[3] = {0, 0, 0}, lg[3][2] = {{0, 0}, {0, 0}, {0, 0}}, lrho = T(0), lsig[3];
      pair_stress_vjp(cc, g, rho, sig, A.eps_g, A.eps_n, lt, ln, lc, lg, lrho, lsig);
#pragma unroll
      for (int c = 0; c < 3; ++c) aadd(&A.X[(AL_C + c) * AP + qc], lc[c]);
      aadd(&A.X[(AL_C + 3) * AP + qc], lrho);
      bool anyg = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) anyg |= (lg[k][0] != T(0)) | (lg[k][1] != T(0));
      if (anyg) {
#pragma unroll
        for (int a = 1; a < 9; ++a) {
          const int ex = lat_ex(a), ey = lat_ey(a);
          int ii = i + ex, jj = j + ey;
          cmap(D, ii, jj);
          const int64_t w = aidx(D, ii, jj);
          const T c = T(3) * wgt<T>(a);
#pragma unroll
          for (int k = 0; k < 3; ++k) aadd(&A.X[(AL_C + k) * AP + w], c * (T(ex) * lg[k][0] + T(ey) * lg[k][1]));
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) sraw[c] = (double)lsig[c];
    }
  }
  block_add(sraw, A.raw + 9 * wk.dom);
}

// Adjoint of C_k = rho_k / rho, rho = sum_k rho_k at fluid nodes.
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_comp(const WorkItem *__restrict__ work, const DomainDev *__restrict__ doms, int n_work, int per, 
                                                     AdjArgs<S, T> A, int64_t tplane) {
  const int wi = adj_item(n_work, per);
  if (wi < 0) return;
  const WorkItem wk = work[wi];
  const DomainDev &D = doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || i < 0 || i >= D.nx) return;
  const int64_t li = plane_index(i, j, D.pitch);
  if (!fluid_node(A.flags, D, i, j)) {  // zero at solid positions (nothing else writes them)
    T *o = A.lout + 9 * tplane + 3 * D.base + li;
    o[0] = o[D.plane] = o[2 * D.plane] = T(0);
    return;
  }
  const int64_t AP = A.aplane;
  const int64_t q = aidx(D, i, j);
  const T C0 = A.X[AX_C * AP + q], C1 = A.X[(AX_C + 1) * AP + q], C2 = A.X[(AX_C + 2) * AP + q];
  const T rt = A.X[(AX_C + 3) * AP + q];
  const T l0 = A.X[AL_C * AP + q], l1 = A.X[(AL_C + 1) * AP + q], l2 = A.X[(AL_C + 2) * AP + q];
  const T lr = A.X[(AL_C + 3) * AP + q];
  const T m = l0 * C0 + l1 * C1 + l2 * C2;
  const T ir = T(1) / rt;
  T *o = A.lout + 9 * tplane + 3 * D.base + li;
  o[0] = (l0 - m) * ir + lr;
  o[D.plane] = (l1 - m) * ir + lr;
  o[2 * D.plane] = (l2 - m) * ir + lr;
}

// Adjoint of the wetting fill (Eq. 21-22), four lanes per fill node as in the forward fill: lane
// `line` marches line `line` of fluid k = line / 2.  The filled C_1, C_2 (C_3 = 1 - C_1 - C_2)
// depend on the partial densities at the interpolation nodes of D0 (through Eq. 21) and of the
// chosen crossing (through the interpolation and, via the angle, the crossing's weight), and
// on theta13, theta23, theta12.  The lane whose value Eq. 22 picked (the first lane of the
// fluid when no line reached the fluid) carries that fluid's reverse-mode chain; its partials
// are added atomically to the density adjoint and to the parameter partials.
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_fill(AdjArgs<S, T> A, int64_t tplane) {
  __shared__ uint32_t far[kThreads / 4][kFarW];  // the nodes' far fluid masks
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = gid >> 2, line = gid & 3, k = line >> 1;
  const bool active = idx < A.n_fill;
  const FillNode fn = A.fill[active ? idx : 0];
  constexpr int kFarPerLane = (kFarW + 3) / 4;
  uint32_t fr[kFarPerLane];  // loaded with the node, stored to LDS once the adjoint of C is in
#pragma unroll
  for (int c = 0; c < kFarPerLane; ++c) {
    const int e = line + 4 * c;
    fr[c] = e < kFarW ? A.far[(size_t)(active ? idx : 0) * kFarW + e] : 0u;
  }
  const DomainDev &D = A.doms[fn.dom];
  const int64_t AP = A.aplane;
  const int64_t P = D.plane;
  const uint8_t *flags = A.flags + D.base;
  const T *r = A.rin + 3 * D.base;
  T *lr = A.lout + 9 * tplane + 3 * D.base;
  double lam = 0.0;  // adjoint of the filled C of fluid k
  if (active) {
    const int64_t qa = aidx(D, fn.i, fn.j);
    lam = (double)A.X[(AL_C + k) * AP + qa] - (double)A.X[(AL_C + 2) * AP + qa];
  }
  const bool work = active && lam != 0.0;  // equal in the two lanes of a fluid
#pragma unroll
  for (int c = 0; c < kFarPerLane; ++c)
    if (line + 4 * c < kFarW) far[threadIdx.x >> 2][line + 4 * c] = fr[c];
  __syncthreads();
  auto fluid_at = [&](int i, int j) -> bool {
    const int dx = i - fn.i, dy = j - fn.j;
    if (FluidMask::inside(dx, dy)) return fn.mask.fluid(dx, dy);
    if (D.bcx == BCX_ZOUHE) {
      if (i < 0 || i >= D.nx) return false;
    } else {
      i = wrap_small(i, D.nx);
    }
    if (D.yper) j = wrap_small(j, D.ny);
    else if (j < 0 || j >= D.ny) return false;
    return (flags[plane_index(i, j, D.pitch)] & FL_SOLID) == 0;
  };
  auto node_q = [&](int i, int j) -> int64_t {
    if (D.bcx != BCX_ZOUHE) i = wrap_small(i, D.nx);
    if (D.yper) j = wrap_small(j, D.ny);
    return plane_index(i, j, D.pitch);
  };
  const double PI = 3.14159265358979323846, LO = 5.0 * PI / 180.0, HI = 175.0 * PI / 180.0;
  double Cb[3] = {0, 0, 0}, ra[3] = {0, 0, 0}, rb[3] = {0, 0, 0}, sa = 1, sb = 1;
  double th = 0, tk = 0, wa = 0, wb = 0, den = 0, thA = 0, thB = 0;
  double v = 0, w = 0, dw = 0, c0 = 0, c1 = 0, s0 = 1, s1 = 1;
  int64_t n0 = 0, n1 = 0;
  int ok = 0;
  if (work) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      ra[q] = (double)r[q * P + fn.d0a];
      rb[q] = (double)r[q * P + fn.d0b];
    }
    sa = ra[0] + ra[1] + ra[2];
    sb = rb[0] + rb[1] + rb[2];
#pragma unroll
    for (int q = 0; q < 3; ++q) Cb[q] = ra[q] / sa + fn.d0w * (rb[q] / sb - ra[q] / sa);
    // Eq. (21): theta_k = (b thA + a thB) / (a + b), a and b the clipped C of the other fluids
    thA = k == 0 ? D.th13 : D.th23;
    thB = k == 0 ? D.th12 : PI - D.th12;
    wa = fmax(Cb[k == 0 ? 1 : 0], 0.0);
    wb = fmax(Cb[2], 0.0);
    den = wa + wb;
    th = den > 1e-12 ? (wb * thA + wa * thB) / den : 0.5 * (thA + thB);
    tk = fmin(fmax(th, LO), HI);
    const double ang = 0.5 * PI - tk, phi = fabs(ang);
    double sn, cs;
    sincos_quadrant(phi, sn, cs);
    const double sg = (line & 1) ? -1.0 : 1.0;
    const double dx = cs * fn.nx - sg * sn * fn.ny, dy = cs * fn.ny + sg * sn * fn.nx;
    const LineHit h = march_line_masked(fn.i, fn.j, dx, dy, fn.mask, far[threadIdx.x >> 2], fluid_at);
    if (h.ok) {
      ok = 1;
      n0 = node_q(h.i0, h.j0);
      n1 = node_q(h.i1, h.j1);
      s0 = (double)r[n0] + (double)r[P + n0] + (double)r[2 * P + n0];
      s1 = (double)r[n1] + (double)r[P + n1] + (double)r[2 * P + n1];
      c0 = (double)r[k * P + n0] / s0;
      c1 = (double)r[k * P + n1] / s1;
      w = h.w;
      v = c0 + w * (c1 - c0);
      // d w / d tk through the line direction (phi = |pi/2 - tk|)
      const double ddx = -sn * fn.nx - sg * cs * fn.ny, ddy = -sn * fn.ny + sg * cs * fn.nx;
      double dwdphi = 0.0;
      if (h.i0 == h.i1 && h.j0 == h.j1) dwdphi = 0.0;  // through a node
      else if (h.j0 == h.j1) dwdphi = (double)(h.j0 - fn.j) * (ddx * dy - dx * ddy) / (dy * dy);
      else dwdphi = (double)(h.i0 - fn.i) * (ddy * dx - dy * ddx) / (dx * dx);
      dw = dwdphi * (ang >= 0.0 ? -1.0 : 1.0);
    }
  }
  const double vo = __shfl_xor(v, 1);
  const int oko = __shfl_xor(ok, 1);
  const bool even = (line & 1) == 0;
  bool chosen = ok != 0;
  if (ok && oko) {  // Eq. (22): max for tk <= 90 degrees, min above; ties go to the first line
    const double ve = even ? v : vo, vd = even ? vo : v;
    const bool pick_even = tk <= 0.5 * PI ? ve >= vd : ve <= vd;
    chosen = even == pick_even;
  }
  const bool fallback = !ok && !oko;
  if (!(work && (chosen || (fallback && even)))) return;
  double lCb[3] = {0, 0, 0}, ltk = 0.0;
  if (fallback) {
    lCb[k] = lam;
  } else {
    const double l0 = lam * (1.0 - w), l1 = lam * w;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const double g0 = l0 * ((q == k ? 1.0 : 0.0) - c0) / s0;
      if (g0 != 0.0) aadd(lr + q * P + n0, (T)g0);
      const double g1 = l1 * ((q == k ? 1.0 : 0.0) - c1) / s1;
      if (g1 != 0.0) aadd(lr + q * P + n1, (T)g1);
    }
    ltk = lam * (c1 - c0) * dw;
  }
  const double lth = (th >= LO && th <= HI) ? ltk : 0.0;
  double lA = 0.0, lB = 0.0;
  if (den > 1e-12) {
    lA = lth * wb / den;
    lB = lth * wa / den;
    const double la = lth * (thB - th) / den, lb = lth * (thA - th) / den;
    if (Cb[k == 0 ? 1 : 0] >= 0.0) lCb[k == 0 ? 1 : 0] += la;
    if (Cb[2] >= 0.0) lCb[2] += lb;
  } else {
    lA = 0.5 * lth;
    lB = 0.5 * lth;
  }
  // C at D0 = C(d0a) + d0w (C(d0b) - C(d0a)), C(x) = rho_k(x) / sum rho(x)
  double ma = 0.0, mb = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    ma += lCb[q] * (1.0 - fn.d0w) * ra[q] / sa;
    mb += lCb[q] * fn.d0w * rb[q] / sb;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double ga = (lCb[q] * (1.0 - fn.d0w) - ma) / sa, gb = (lCb[q] * fn.d0w - mb) / sb;
    if (ga != 0.0) aadd(lr + q * P + fn.d0a, (T)ga);
    if (gb != 0.0) aadd(lr + q * P + fn.d0b, (T)gb);
  }
  // theta12 enters fluid 2's angle as theta21 = pi - theta12
  if (lA != 0.0) aadd(&A.raw[9 * fn.dom + 6 + k], lA);
  if (lB != 0.0) aadd(&A.raw[9 * fn.dom + 8], k == 0 ? lB : -lB);
}

// Seed: lambda_rho_k = dL/drho_k of a loss of the partial densities at fluid nodes, read from a
// flat [3][ny][nx] array per domain (domains concatenated).
template <typename T>
__global__ __launch_bounds__(kThreads) void adj_seed(const DomainDev *doms, const WorkItem *work, const uint8_t *flags,
                                                     const double *g, T *lam, int64_t tplane) {
  const WorkItem wk = work[blockIdx.x];
  const DomainDev &D = doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || !fluid_node(flags, D, i, j)) return;
  const int64_t li = plane_index(i, j, D.pitch);
  const int64_t n = (int64_t)D.nx * D.ny, o = D.goff + (int64_t)j * D.nx + i;
#pragma unroll
  for (int k = 0; k < 3; ++k) lam[9 * tplane + 3 * D.base + k * D.plane + li] = (T)g[o + k * n];
}

// Phase-field mismatch loss L = sum over fluid nodes of sum_k (C_k - C*_k)^2 with C_k = rho_k /
// rho (the loss of the inverse problem), and its gradient with respect to the partial densities,
// dL/drho_k = (2 / rho) [(C_k - C*_k) - sum_l C_l (C_l - C*_l)], written into the density planes of
// lam at fluid nodes.  FP64 throughout; each work-group writes its loss partial (fixed order
// inside the group) to part[blockIdx.x], and loss_final sums a domain's partials in tile order,
// so the loss is reproducible bit for bit.
template <typename T>
__global__ __launch_bounds__(kThreads) void loss_seed_tiles(const DomainDev *doms, const WorkItem *work,
                                                            const uint8_t *flags, const T *rho, int64_t tplane,
                                                            const double *target, T *lam, double *part) {
  const WorkItem wk = work[blockIdx.x];
  const DomainDev &D = doms[wk.dom];
  int i, j;
  double l = 0.0;
  if (tile_node(wk, i, j) && fluid_node(flags, D, i, j)) {
    const int64_t li = plane_index(i, j, D.pitch);
    const T *R = rho + 3 * D.base;
    const int64_t n = (int64_t)D.nx * D.ny, o = D.goff + (int64_t)j * D.nx + i;
    double r[3], c[3], d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = (double)R[k * D.plane + li];
    const double rt = r[0] + r[1] + r[2];
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c[k] = r[k] / rt;
      d[k] = c[k] - target[o + k * n];
      l += d[k] * d[k];
      m += c[k] * d[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) lam[9 * tplane + 3 * D.base + k * D.plane + li] = (T)(2.0 * (d[k] - m) / rt);
  }
  __shared__ double red[kThreads / 64];
  const double s = wave_sum(l);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kThreads / 64; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

__global__ void loss_final(const double *part, const int *first, int n_dom, double *loss) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= n_dom) return;
  double s = 0.0;
  for (int b = first[d]; b < first[d + 1]; ++b) s += part[b];
  loss[d] = s;
}

// ---- launchers -----------------------------------------------------------------------------
template <typename S, typename T>
hipError_t launch_adjoint(const AdjArgs<S, T> &a, int64_t tplane, hipStream_t s) {
  const dim3 g((a.n_work + 7) / 8 * 8), b(kThreads);
  hipLaunchKernelGGL((adj_node<S, T>), g, b, 0, s, a.work, a.doms, a.n_work, (int)(g.x >> 3), a, tplane);
  hipLaunchKernelGGL((adj_stress<S, T>), g, b, 0, s, a.work, a.doms, a.n_work, (int)(g.x >> 3), a);
  hipLaunchKernelGGL((adj_comp<S, T>), g, b, 0, s, a.work, a.doms, a.n_work, (int)(g.x >> 3), a, tplane);
  if (a.n_fill > 0)
    hipLaunchKernelGGL((adj_fill<S, T>), dim3((4 * a.n_fill + kThreads - 1) / kThreads), b, 0, s, a, tplane);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_seed(const DomainDev *doms, const WorkItem *work, int n_work, const uint8_t *flags,
                               const double *g, T *lam, int64_t tplane, hipStream_t s) {
  if (n_work > 0)
    hipLaunchKernelGGL((adj_seed<T>), dim3(n_work), dim3(kThreads), 0, s, doms, work, flags, g, lam, tplane);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_loss_seed(const DomainDev *doms, const WorkItem *work, int n_work, const int *first, int n_dom,
                            const uint8_t *flags, const T *rho, int64_t tplane, const double *target, T *lam,
                            double *part, double *loss, hipStream_t s) {
  if (n_work > 0)
    hipLaunchKernelGGL((loss_seed_tiles<T>), dim3(n_work), dim3(kThreads), 0, s, doms, work, flags, rho, tplane, target,
                       lam, part);
  hipLaunchKernelGGL(loss_final, dim3((n_dom + 63) / 64), dim3(64), 0, s, part, first, n_dom, loss);
  return hipGetLastError();
}

template hipError_t launch_adjoint<double, double>(const AdjArgs<double, double> &, int64_t, hipStream_t);
template hipError_t launch_adjoint<float, float>(const AdjArgs<float, float> &, int64_t, hipStream_t);
template hipError_t launch_adjoint_seed<double>(const DomainDev *, const WorkItem *, int, const uint8_t *,
                                                const double *, double *, int64_t, hipStream_t);
template hipError_t launch_adjoint_seed<float>(const DomainDev *, const WorkItem *, int, const uint8_t *,
                                               const double *, float *, int64_t, hipStream_t);

template hipError_t launch_loss_seed<double>(const DomainDev *, const WorkItem *, int, const int *, int,
                                             const uint8_t *, const double *, int64_t, const double *, double *,
                                             double *, double *, hipStream_t);
template hipError_t launch_loss_seed<float>(const DomainDev *, const WorkItem *, int, const int *, int,
                                            const uint8_t *, const float *, int64_t, const double *, float *,
                                            double *, double *, hipStream_t);

}  // namespace lbm3
