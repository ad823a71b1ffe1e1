// lbm3_adjoint.hip -- hand-written adjoint of one step of the three-phase update
// (arXiv:2102.04709, Sec. II).  Given the forward state s_t and the adjoint lambda_{t+1} of the
// state at t+1, it produces lambda_t = (d s_{t+1} / d s_t)^T lambda_{t+1} and accumulates the
// raw parameter partials (d s_{t+1} / d p)^T lambda_{t+1} for p = (sigma12, sigma13, sigma23,
// g(X_12), g(X_13), g(X_23), theta13, theta23, theta12).
//
// Forward intermediates of s_t (on an extended grid, see lbm3_adjoint.h): C_k and rho with the
// filled C at the solid boundary nodes (Eq. 21-22), stress and pair normals (Eq. 10, 12),
// interfacial force, post-collision f' and recolouring vectors R (Eq. 1-9, 11, 13-15).
// Transposes, in reverse order of the forward: streaming (Eq. 16 with every boundary rule, as
// atomic scatters), the per-node collision + recolouring (Jacobian-transpose products from
// forward-mode dual numbers run through the same templated code as the forward kernels, one
// seed per input), the stress divergence, the per-node stress (dual numbers), the colour-gradient
// stencil, the mass fractions, and the wetting fill (dual numbers over the fill's arithmetic with
// its discrete choices -- which crossing, which line -- fixed at their forward values).
// Non-smooth points (the max/min of Eq. 22, clamps, the |G| threshold) take the derivative of the
// branch the forward took.
#include <hip/hip_runtime.h>

#include "lbm3_adjoint.h"
#include "lbm3_device.h"
#include "lbm3_internal.h"

namespace lbm3 {

// ---- dual numbers: a value and one directional derivative ------------------------------------
// The math overloads are hidden friends: found for Dual arguments by argument-dependent lookup
// only, so plain double/float calls in this namespace still reach the C library functions.
template <typename T>
struct Dual {
  T v, d;
  __host__ __device__ Dual() : v(0), d(0) {}
  __host__ __device__ Dual(double x) : v((T)x), d(0) {}
  __host__ __device__ Dual(T x, T dx, int) : v(x), d(dx) {}
  friend __device__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d, 0); }
  friend __device__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d, 0); }
  friend __device__ Dual operator-(Dual a) { return Dual(-a.v, -a.d, 0); }
  friend __device__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d, 0); }
  friend __device__ Dual operator/(Dual a, Dual b) {
    const T r = a.v / b.v;
    return Dual(r, (a.d - r * b.d) / b.v, 0);
  }
  __device__ Dual &operator+=(Dual b) { v += b.v; d += b.d; return *this; }
  __device__ Dual &operator-=(Dual b) { v -= b.v; d -= b.d; return *this; }
  friend __device__ bool operator>(Dual a, Dual b) { return a.v > b.v; }
  friend __device__ bool operator<(Dual a, Dual b) { return a.v < b.v; }
  friend __device__ bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
  friend __device__ bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
  friend __device__ Dual sqrt(Dual a) {
    const T s = sqrt(a.v);
    return Dual(s, s > T(0) ? a.d / (T(2) * s) : T(0), 0);
  }
  friend __device__ Dual fmin(Dual a, Dual b) { return a.v <= b.v ? a : b; }
  friend __device__ Dual fmax(Dual a, Dual b) { return a.v >= b.v ? a : b; }
  friend __device__ Dual fabs(Dual a) { return a.v < T(0) ? -a : a; }
};

template <>
__device__ __forceinline__ Dual<float> rcp<Dual<float>>(Dual<float> x) {
  const float r = __builtin_amdgcn_rcpf(x.v);
  return Dual<float>(r, -x.d * r * r, 0);
}
template <>
__device__ __forceinline__ Dual<double> rcp<Dual<double>>(Dual<double> x) {
  const double r = 1.0 / x.v;
  return Dual<double>(r, -x.d * r * r, 0);
}

__device__ __forceinline__ void sincos_dual(Dual<double> x, Dual<double> &s, Dual<double> &c) {
  double sv, cv;
  sincos(x.v, &sv, &cv);
  s = Dual<double>(sv, cv * x.d, 0);
  c = Dual<double>(cv, -sv * x.d, 0);
}

// Hardware floating-point atomic add (the workspace is ordinary coarse-grained device memory).
template <typename T>
__device__ __forceinline__ void aadd(T *p, T v) { unsafeAtomicAdd(p, v); }

// Input number idx of a dual evaluation seeded on input s.
template <typename T>
__device__ __forceinline__ Dual<T> seeded(T v, int s, int idx) { return Dual<T>(v, s == idx ? T(1) : T(0), 0); }

// ---- extended grid ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t aidx(const DomainDev &D, int i, int j) {
  return D.abase + (i + 1) + (int64_t)(D.nx + 2) * (j + 2);
}
// Node whose stored data a read at (i, j) sees (the forward's node_index): periodic axes wrap,
// the Zou-He x axis clamps to the boundary columns, a non-periodic y axis to the off-grid rows.
__device__ __forceinline__ void cmap(const DomainDev &D, int &i, int &j) {
  i = D.bcx == BCX_ZOUHE ? min(max(i, 0), D.nx - 1) : wrap_small(i, D.nx);
  j = D.yper ? wrap_small(j, D.ny) : min(max(j, -2), D.ny + 1);
}
// Position of the stress a divergence at (i, j) reads: periodic axes wrap; the stress at a
// Zou-He ghost column or an off-grid row is its own value (computed there from clamped C).
__device__ __forceinline__ void tmap(const DomainDev &D, int &i, int &j) {
  if (D.bcx != BCX_ZOUHE) i = wrap_small(i, D.nx);
  if (D.yper) j = wrap_small(j, D.ny);
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
__device__ __forceinline__ bool tile_node(const WorkItem &wk, int &i, int &j) {
  i = wk.x0 + (threadIdx.x & 31);
  j = wk.y0 + (threadIdx.x >> 5);
  return i < wk.x1 && j < wk.y1;
}

template <typename T>
__device__ __forceinline__ T &XP(T *X, int64_t AP, int plane, int64_t q) { return X[plane * AP + q]; }

// ---- forward intermediates -----------------------------------------------------------------
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_fwd_c(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || i < 0 || i >= D.nx) return;  // ghost columns hold no C
  const int64_t li = plane_index(i, j, D.pitch);
  const uint8_t fl = A.flags[D.base + li];
  const T *R = A.rin + 3 * D.base;
  T v[4];
  node_composition<T>(fl, R[li], R[D.plane + li], R[2 * D.plane + li], A.fillC, v);
  const int64_t q = aidx(D, i, j);
#pragma unroll
  for (int c = 0; c < 4; ++c) XP(A.X, A.aplane, AX_C + c, q) = v[c];
}

template <typename T>
__device__ __forceinline__ void c9_at(const T *X, int64_t AP, const DomainDev &D, int i, int j, int k, T c9[9]) {
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    int ii = i + lat_ex(a), jj = j + lat_ey(a);
    cmap(D, ii, jj);
    c9[a] = X[(AX_C + k) * AP + aidx(D, ii, jj)];
  }
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_fwd_t(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j)) return;
  const int64_t AP = A.aplane;
  const KT<T> K = make_kt<T>(D);
  T g[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T c9[9];
    c9_at(A.X, AP, D, i, j, k, c9);
    grad9(c9, g[k][0], g[k][1]);
  }
  int ci = i, cj = j;
  cmap(D, ci, cj);
  const int64_t qc = aidx(D, ci, cj);
  const T cc[3] = {A.X[AX_C * AP + qc], A.X[(AX_C + 1) * AP + qc], A.X[(AX_C + 2) * AP + qc]};
  T txx, txy, tyy, nrm[6];
  pair_stress(cc, g, A.X[(AX_C + 3) * AP + qc], K, A.eps_g, txx, txy, tyy, nrm);
  const int64_t q = aidx(D, i, j);
  XP(A.X, AP, AX_T, q) = txx;
  XP(A.X, AP, AX_T + 1, q) = txy;
  XP(A.X, AP, AX_T + 2, q) = tyy;
#pragma unroll
  for (int c = 0; c < 6; ++c) XP(A.X, AP, AX_N + c, q) = nrm[c];
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_fwd_p(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || !fluid_node(A.flags, D, i, j)) return;
  const int64_t AP = A.aplane;
  const KT<T> K = make_kt<T>(D);
  T xx[9], xy[9], yy[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    int ii = i + lat_ex(a), jj = j + lat_ey(a);
    tmap(D, ii, jj);
    const int64_t q = aidx(D, ii, jj);
    xx[a] = A.X[AX_T * AP + q];
    xy[a] = A.X[(AX_T + 1) * AP + q];
    yy[a] = A.X[(AX_T + 2) * AP + q];
  }
  T Fx, Fy;
  div_stress(xx, xy, yy, Fx, Fy);
  const int64_t q = aidx(D, i, j);
  XP(A.X, AP, AX_F, q) = Fx;
  XP(A.X, AP, AX_F + 1, q) = Fy;
  const int64_t li = plane_index(i, j, D.pitch);
  T f[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) f[a] = load_s<S, T>(A.fin + 9 * D.base + a * D.plane + li);
  const T rt = A.X[(AX_C + 3) * AP + q];
  const T r0 = A.X[AX_C * AP + q] * rt, r1 = A.X[(AX_C + 1) * AP + q] * rt, r2 = A.X[(AX_C + 2) * AP + q] * rt;
  T fd[9], ux, uy, nrm[6], Rv[4];
  collide_shifted(f, Fx, Fy, r0, r1, r2, K, fd, ux, uy);
#pragma unroll
  for (int c = 0; c < 6; ++c) nrm[c] = A.X[(AX_N + c) * AP + q];
  recolour_R(r0, r1, r2, rt, nrm, K, Rv);
#pragma unroll
  for (int a = 0; a < 9; ++a) XP(A.X, AP, AX_P + a, q) = fd[a];
#pragma unroll
  for (int c = 0; c < 4; ++c) XP(A.X, AP, AX_P + 9 + c, q) = Rv[c];
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_zero(AdjArgs<S, T> A, int64_t n) {
  T *p = A.X + (int64_t)AL_P * A.aplane;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    p[k] = T(0);
}

// ---- transposes ----------------------------------------------------------------------------
// Adjoint of one read in the forward pull of the recoloured populations of direction dir of
// node q, weighted by coef: the read contributes coef * f'_dir to the destination's total
// (adjoint lf) and coef * (C_k (f'_dir + w) + w R_k.e_dir) to its partial density k (adjoint
// mu[k], already permuted for a fluid-exchanging boundary).
template <typename T>
__device__ __forceinline__ void scatter_parts(T *X, int64_t AP, int64_t q, int dir, T coef, const T mu[3], T lf) {
  const T f = X[(AX_P + dir) * AP + q];
  const T C0 = X[AX_C * AP + q], C1 = X[(AX_C + 1) * AP + q], C2 = X[(AX_C + 2) * AP + q];
  const T w = wgt<T>(dir);
  const int ex = lat_ex(dir), ey = lat_ey(dir);
  aadd(&X[(AL_P + dir) * AP + q], coef * (lf + mu[0] * C0 + mu[1] * C1 + mu[2] * C2));
  const T fw = coef * (f + w);
  aadd(&X[AL_C * AP + q], mu[0] * fw);
  aadd(&X[(AL_C + 1) * AP + q], mu[1] * fw);
  aadd(&X[(AL_C + 2) * AP + q], mu[2] * fw);
  const T a = coef * w * (mu[0] - mu[2]), b = coef * w * (mu[1] - mu[2]);
  if (ex) {
    aadd(&X[(AL_P + 9) * AP + q], a * T(ex));
    aadd(&X[(AL_P + 11) * AP + q], b * T(ex));
  }
  if (ey) {
    aadd(&X[(AL_P + 10) * AP + q], a * T(ey));
    aadd(&X[(AL_P + 12) * AP + q], b * T(ey));
  }
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_stream(AdjArgs<S, T> A, int64_t tplane) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || !fluid_node(A.flags, D, i, j)) return;
  const int64_t AP = A.aplane;
  const int64_t li = plane_index(i, j, D.pitch);
  const int64_t q = aidx(D, i, j);
  T lf[9], mu[3];
#pragma unroll
  for (int a = 0; a < 9; ++a) lf[a] = A.lin[9 * D.base + a * D.plane + li];
#pragma unroll
  for (int k = 0; k < 3; ++k) mu[k] = A.lin[9 * tplane + 3 * D.base + k * D.plane + li];
  if (D.bcx == BCX_ZOUHE && (i == 0 || i == D.nx - 1)) {
    // Zou-He: the unknown totals are affine in the known ones, which the columns next to the
    // boundary supply (no solid node lies within three columns of it and y is periodic).
    T ft[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const int si = i - lat_ex(a);
      int ii = si, jj = j - lat_ey(a);
      cmap(D, ii, jj);
      ft[a] = (si < 0 || si >= D.nx) ? T(0) : A.X[(AX_P + a) * AP + aidx(D, ii, jj)] + wgt<T>(a);
    }
    if (i == 0) {
      const T u = (T)D.u_in;
      const T ir = T(1) / (T(1) - u);
      const T r[9] = {ir, 0, ir, 2 * ir, ir, 0, 2 * ir, 2 * ir, 0};  // d rho_w / d ft_k
      const T l1 = lf[1] + mu[2], l5 = lf[5] + mu[2], l8 = lf[8] + mu[2];  // inflow is fluid 3
      const T lw = (T(2.0 / 3.0) * l1 + (l5 + l8) / T(6)) * u;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (k == 1 || k == 5 || k == 8) continue;
        T add = lw * r[k];
        if (k == 3) add += l1;
        if (k == 7) add += l5;
        if (k == 6) add += l8;
        if (k == 2) add += T(0.5) * (l8 - l5);
        if (k == 4) add += T(0.5) * (l5 - l8);
        lf[k] += add;
      }
    } else {
      const T ro = (T)D.rho_out;
      const T s[9] = {1, 2, 1, 0, 1, 2, 0, 0, 2};  // d (rho_out u_x) / d ft_k
      const T C0 = A.X[AX_C * AP + q], C1 = A.X[(AX_C + 1) * AP + q], C2 = A.X[(AX_C + 2) * AP + q];
      const T ux = -T(1) + (ft[0] + ft[2] + ft[4] + T(2) * (ft[1] + ft[5] + ft[8])) / ro;
      const T f3 = ft[1] - T(2.0 / 3.0) * ro * ux;
      const T f7 = ft[5] + T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
      const T f6 = ft[8] - T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
      const T su = f3 + f6 + f7;  // outflow carries the node's own composition
      aadd(&A.X[AL_C * AP + q], mu[0] * su);
      aadd(&A.X[(AL_C + 1) * AP + q], mu[1] * su);
      aadd(&A.X[(AL_C + 2) * AP + q], mu[2] * su);
      const T mc = mu[0] * C0 + mu[1] * C1 + mu[2] * C2;
      const T l3 = lf[3] + mc, l6 = lf[6] + mc, l7 = lf[7] + mc;
      const T lw = -(T(2.0 / 3.0) * l3 + (l7 + l6) / T(6));
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (k == 3 || k == 6 || k == 7) continue;
        T add = lw * s[k];
        if (k == 1) add += l3;
        if (k == 5) add += l7;
        if (k == 8) add += l6;
        if (k == 2) add += T(0.5) * (l7 - l6);
        if (k == 4) add += T(0.5) * (l6 - l7);
        lf[k] += add;
      }
    }
  }
  const uint8_t fl = A.flags[D.base + li];
  const IbbNode *ib = ((fl & FL_CURVED) && D.n_ibb > 0) ? find_ibb(A.ibb, D, li) : nullptr;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    const int sx = i - ex;
    if (D.bcx == BCX_ZOUHE && (sx < 0 || sx >= D.nx)) continue;  // unknown: handled above
    int si = sx, sj = j - ey;
    cmap(D, si, sj);
    if (!solid_at(A.flags, D, si, sj)) {
      const bool crossed = D.bcx == BCX_SWAP13 && (sx < 0 || sx >= D.nx);
      const T m[3] = {crossed ? mu[2] : mu[0], mu[1], crossed ? mu[0] : mu[2]};
      scatter_parts(A.X, AP, aidx(D, si, sj), a, T(1), m, lf[a]);
    } else {
      const int ab = lat_opp(a);
      const T qd = ib ? (T)ib->q[a - 1] : T(0.5);
      int ni = i + ex, nj = j + ey;
      cmap(D, ni, nj);
      if (qd < T(0.5) && !solid_at(A.flags, D, ni, nj)) {
        scatter_parts(A.X, AP, q, ab, T(2) * qd, mu, lf[a]);
        scatter_parts(A.X, AP, aidx(D, ni, nj), ab, T(1) - T(2) * qd, mu, lf[a]);
      } else if (qd < T(0.5)) {
        scatter_parts(A.X, AP, q, ab, T(1), mu, lf[a]);
      } else {
        const T c1 = rcp(T(2) * qd), c2 = T(1) - c1;
        scatter_parts(A.X, AP, q, ab, c1, mu, lf[a]);
        if (c2 != T(0)) scatter_parts(A.X, AP, q, a, c2, mu, lf[a]);
      }
    }
  }
}

// Adjoint of the per-node collision and recolouring: inputs f (9), F_s (2), C (3), rho (1),
// n (6) and g(X) of the three pairs (3); outputs f' (9) and R (4).
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_collide(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  double graw[3] = {0, 0, 0};
  if (tile_node(wk, i, j) && fluid_node(A.flags, D, i, j)) {
    const int64_t AP = A.aplane;
    const int64_t li = plane_index(i, j, D.pitch);
    const int64_t q = aidx(D, i, j);
    T in[24];
#pragma unroll
    for (int a = 0; a < 9; ++a) in[a] = load_s<S, T>(A.fin + 9 * D.base + a * D.plane + li);
    in[9] = A.X[AX_F * AP + q];
    in[10] = A.X[(AX_F + 1) * AP + q];
#pragma unroll
    for (int c = 0; c < 4; ++c) in[11 + c] = A.X[(AX_C + c) * AP + q];
#pragma unroll
    for (int c = 0; c < 6; ++c) in[15 + c] = A.X[(AX_N + c) * AP + q];
#pragma unroll
    for (int c = 0; c < 3; ++c) in[21 + c] = (T)D.gX[c];
    T lo[13];
#pragma unroll
    for (int c = 0; c < 13; ++c) lo[c] = A.X[(AL_P + c) * AP + q];
    T lc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) lc[c] = A.X[(AL_C + c) * AP + q];
#pragma unroll 1
    for (int s = 0; s < 24; ++s) {
      using DT = Dual<T>;
      DT f[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) f[a] = seeded(in[a], s, a);
      DT Fx = seeded(in[9], s, 9), Fy = seeded(in[10], s, 10);
      const DT C0 = seeded(in[11], s, 11), C1 = seeded(in[12], s, 12), C2 = seeded(in[13], s, 13);
      const DT rt = seeded(in[14], s, 14);
      DT nrm[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) nrm[c] = seeded(in[15 + c], s, 15 + c);
      KT<DT> K = make_kt<DT>(D);
#pragma unroll
      for (int c = 0; c < 3; ++c) K.gX[c] = seeded(in[21 + c], s, 21 + c);
      const DT r0 = C0 * rt, r1 = C1 * rt, r2 = C2 * rt;
      DT fd[9], ux, uy, Rv[4];
      collide_shifted(f, Fx, Fy, r0, r1, r2, K, fd, ux, uy);
      recolour_R(r0, r1, r2, rt, nrm, K, Rv);
      T g = T(0);
#pragma unroll
      for (int a = 0; a < 9; ++a) g += lo[a] * fd[a].d;
#pragma unroll
      for (int c = 0; c < 4; ++c) g += lo[9 + c] * Rv[c].d;
      if (s < 9) A.lout[9 * D.base + s * D.plane + li] = g;
      else if (s < 11) A.X[(AL_F + s - 9) * AP + q] = g;
      else if (s < 15) lc[s - 11] += g;
      else if (s < 21) A.X[(AL_N + s - 15) * AP + q] = g;
      else graw[s - 21] = (double)g;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) A.X[(AL_C + c) * AP + q] = lc[c];
  }
  block_add(graw, A.raw + 9 * wk.dom + 3);
}

// Adjoint of the stress divergence F(x) = 3 sum_a w_a T(x + e_a) . e_a (Eq. 12 on Eq. 10).
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_div(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || !fluid_node(A.flags, D, i, j)) return;
  const int64_t AP = A.aplane;
  const int64_t q = aidx(D, i, j);
  const T lx = A.X[AL_F * AP + q], ly = A.X[(AL_F + 1) * AP + q];
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    int ii = i + ex, jj = j + ey;
    tmap(D, ii, jj);
    const int64_t z = aidx(D, ii, jj);
    const T c = T(3) * wgt<T>(a);
    if (ex) aadd(&A.X[AL_T * AP + z], c * T(ex) * lx);
    aadd(&A.X[(AL_T + 1) * AP + z], c * (T(ey) * lx + T(ex) * ly));
    if (ey) aadd(&A.X[(AL_T + 2) * AP + z], c * T(ey) * ly);
  }
}

// Adjoint of the per-position stress and normals: inputs C (3), gradients (6), rho (1) and
// sigma (3).
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_stress(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  double sraw[3] = {0, 0, 0};
  if (tile_node(wk, i, j)) {
    const int64_t AP = A.aplane;
    const int64_t q = aidx(D, i, j);
    T lo[9];
    bool any = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = A.X[(AL_T + c) * AP + q];
      any |= lo[c] != T(0);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      lo[3 + c] = A.X[(AL_N + c) * AP + q];
      any |= lo[3 + c] != T(0);
    }
    if (any) {
      T in[13];
      int ci = i, cj = j;
      cmap(D, ci, cj);
      const int64_t qc = aidx(D, ci, cj);
#pragma unroll
      for (int c = 0; c < 3; ++c) in[c] = A.X[(AX_C + c) * AP + qc];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T c9[9];
        c9_at(A.X, AP, D, i, j, k, c9);
        grad9(c9, in[3 + 2 * k], in[4 + 2 * k]);
      }
      in[9] = A.X[(AX_C + 3) * AP + qc];
#pragma unroll
      for (int c = 0; c < 3; ++c) in[10 + c] = (T)D.sig[c];
#pragma unroll 1
      for (int s = 0; s < 13; ++s) {
        using DT = Dual<T>;
        const DT cc[3] = {seeded(in[0], s, 0), seeded(in[1], s, 1), seeded(in[2], s, 2)};
        DT g[3][2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          g[k][0] = seeded(in[3 + 2 * k], s, 3 + 2 * k);
          g[k][1] = seeded(in[4 + 2 * k], s, 4 + 2 * k);
        }
        const DT rho = seeded(in[9], s, 9);
        KT<DT> K = make_kt<DT>(D);
#pragma unroll
        for (int c = 0; c < 3; ++c) K.sig[c] = seeded(in[10 + c], s, 10 + c);
        DT txx, txy, tyy, nrm[6];
        pair_stress(cc, g, rho, K, DT((double)A.eps_g), txx, txy, tyy, nrm);
        T v = lo[0] * txx.d + lo[1] * txy.d + lo[2] * tyy.d;
#pragma unroll
        for (int c = 0; c < 6; ++c) v += lo[3 + c] * nrm[c].d;
        if (s < 3) aadd(&A.X[(AL_C + s) * AP + qc], v);
        else if (s < 9) A.X[(AL_G + s - 3) * AP + q] = v;
        else if (s == 9) aadd(&A.X[(AL_C + 3) * AP + qc], v);
        else sraw[s - 10] = (double)v;
      }
    }
  }
  block_add(sraw, A.raw + 9 * wk.dom);
}

// Adjoint of the colour-gradient stencil (Eq. 12).
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_grad(AdjArgs<S, T> A) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j)) return;
  const int64_t AP = A.aplane;
  const int64_t q = aidx(D, i, j);
  T lg[6];
  bool any = false;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    lg[c] = A.X[(AL_G + c) * AP + q];
    any |= lg[c] != T(0);
  }
  if (!any) return;
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    int ii = i + ex, jj = j + ey;
    cmap(D, ii, jj);
    const int64_t w = aidx(D, ii, jj);
    const T c = T(3) * wgt<T>(a);
#pragma unroll
    for (int k = 0; k < 3; ++k) aadd(&A.X[(AL_C + k) * AP + w], c * (T(ex) * lg[2 * k] + T(ey) * lg[2 * k + 1]));
  }
}

// Adjoint of C_k = rho_k / rho, rho = sum_k rho_k at fluid nodes.
template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_comp(AdjArgs<S, T> A, int64_t tplane) {
  const WorkItem wk = A.work[blockIdx.x];
  const DomainDev &D = A.doms[wk.dom];
  int i, j;
  if (!tile_node(wk, i, j) || !fluid_node(A.flags, D, i, j)) return;
  const int64_t AP = A.aplane;
  const int64_t q = aidx(D, i, j);
  const int64_t li = plane_index(i, j, D.pitch);
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

// Adjoint of the wetting fill of one node: its filled C_1, C_2 (C_3 = 1 - C_1 - C_2) as
// functions of the partial densities at the interpolation nodes of D0 and of the crossings of
// its four lines, and of theta13, theta23, theta12.
template <typename R>
__device__ __forceinline__ R cfr(const R *r3, int k) { return r3[k] / (r3[0] + r3[1] + r3[2]); }

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void adj_fill(AdjArgs<S, T> A, int64_t tplane) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= A.n_fill) return;
  const FillNode fn = A.fill[idx];
  const DomainDev &D = A.doms[fn.dom];
  const int64_t AP = A.aplane;
  const int64_t qa = aidx(D, fn.i, fn.j);
  const double lC0 = (double)A.X[AL_C * AP + qa], lC1 = (double)A.X[(AL_C + 1) * AP + qa];
  const double lC2 = (double)A.X[(AL_C + 2) * AP + qa];
  const double lam1 = lC0 - lC2, lam2 = lC1 - lC2;
  if (lam1 == 0.0 && lam2 == 0.0) return;
  const uint8_t *flags = A.flags + D.base;
  const T *r = A.rin + 3 * D.base;
  const int64_t P = D.plane;
  auto fluid_at = [&](int i, int j) -> bool {
    const int dx = i - fn.i, dy = j - fn.j;
    if (dx >= -3 && dx <= 3 && dy >= -3 && dy <= 3) return (fn.mask >> ((dy + 3) * 7 + dx + 3)) & 1;
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
  const double PI = 3.14159265358979323846;
  // forward values in FP64 as the fill kernel forms them: angles and the lines' crossings
  double rho_in[30];
  int64_t node_of[10];
  node_of[0] = fn.d0a;
  node_of[1] = fn.d0b;
  for (int c = 0; c < 3; ++c) {
    rho_in[c] = (double)r[c * P + fn.d0a];
    rho_in[3 + c] = (double)r[c * P + fn.d0b];
  }
  double Cb[3];
  for (int k = 0; k < 3; ++k) {
    const double ca = cfr(rho_in, k), cb = cfr(rho_in + 3, k);
    Cb[k] = ca + fn.d0w * (cb - ca);
  }
  double thv[2];
  {
    const double a = fmax(Cb[1], 0.0), b = fmax(Cb[2], 0.0), den = a + b;
    thv[0] = den > 1e-12 ? (b * D.th13 + a * D.th12) / den : 0.5 * (D.th13 + D.th12);
    const double a2 = fmax(Cb[0], 0.0), den2 = a2 + b;
    thv[1] = den2 > 1e-12 ? (b * D.th23 + a2 * (PI - D.th12)) / den2 : 0.5 * (D.th23 + PI - D.th12);
  }
  LineHit h[4];
  for (int l = 0; l < 4; ++l) {
    const int k = l >> 1;
    const double tk = fmin(fmax(thv[k], 5.0 * PI / 180.0), 175.0 * PI / 180.0);
    const double phi = fabs(0.5 * PI - tk);
    double sp, cp;
    sincos(phi, &sp, &cp);
    if (l & 1) sp = -sp;
    h[l] = march_line(fn.i, fn.j, cp * fn.nx + sp * (-fn.ny), cp * fn.ny + sp * fn.nx, fluid_at);
    const int64_t n0 = h[l].ok ? node_q(h[l].i0, h[l].j0) : fn.d0a;
    const int64_t n1 = h[l].ok ? node_q(h[l].i1, h[l].j1) : fn.d0a;
    node_of[2 + 2 * l] = n0;
    node_of[3 + 2 * l] = n1;
    for (int c = 0; c < 3; ++c) {
      rho_in[6 + 6 * l + c] = (double)r[c * P + n0];
      rho_in[9 + 6 * l + c] = (double)r[c * P + n1];
    }
  }
  double traw[3] = {0, 0, 0};
  // one dual evaluation per input: 30 densities, theta13, theta23, theta12
  for (int s = 0; s < 33; ++s) {
    if (s >= 6 && s < 30 && !h[(s - 6) / 6].ok) continue;  // a line that failed reads nothing
    using DD = Dual<double>;
    DD rin_d[30];
    for (int c = 0; c < 30; ++c) rin_d[c] = seeded(rho_in[c], s, c);
    const DD t13 = seeded(D.th13, s, 30), t23 = seeded(D.th23, s, 31), t12 = seeded(D.th12, s, 32);
    DD cb[3];
    for (int k = 0; k < 3; ++k) {
      const DD ca = cfr(rin_d, k), cbb = cfr(rin_d + 3, k);
      cb[k] = ca + DD(fn.d0w) * (cbb - ca);
    }
    DD th[2];
    {
      const DD a = fmax(cb[1], DD(0.0)), b = fmax(cb[2], DD(0.0)), den = a + b;
      th[0] = den.v > 1e-12 ? (b * t13 + a * t12) / den : DD(0.5) * (t13 + t12);
      const DD a2 = fmax(cb[0], DD(0.0)), den2 = a2 + b;
      const DD t21 = DD(PI) - t12;
      th[1] = den2.v > 1e-12 ? (b * t23 + a2 * t21) / den2 : DD(0.5) * (t23 + t21);
    }
    DD v[4], tkk[2];
    for (int l = 0; l < 4; ++l) {
      const int k = l >> 1;
      DD tk = th[k];
      if (tk.v < 5.0 * PI / 180.0) tk = DD(5.0 * PI / 180.0);
      if (tk.v > 175.0 * PI / 180.0) tk = DD(175.0 * PI / 180.0);
      tkk[k] = tk;
      if (!h[l].ok) continue;
      const DD phi = fabs(DD(0.5 * PI) - tk);
      DD sp, cp;
      sincos_dual(phi, sp, cp);
      if (l & 1) sp = -sp;
      const DD dx = cp * DD(fn.nx) + sp * DD(-fn.ny), dy = cp * DD(fn.ny) + sp * DD(fn.nx);
      DD w(0.0);
      if (h[l].i0 == h[l].i1 && h[l].j0 == h[l].j1) {
        w = DD(0.0);  // the line passes through a node
      } else if (h[l].j0 == h[l].j1) {  // row y = j0 crossed at x = pi + (j0 - pj) dx / dy
        w = DD((double)(fn.i - h[l].i0)) + DD((double)(h[l].j0 - fn.j)) * dx / dy;
      } else {  // column x = i0 crossed at y = pj + (i0 - pi) dy / dx
        w = DD((double)(fn.j - h[l].j0)) + DD((double)(h[l].i0 - fn.i)) * dy / dx;
      }
      const DD c0 = cfr(rin_d + 6 + 6 * l, k), c1 = cfr(rin_d + 9 + 6 * l, k);
      v[l] = c0 + w * (c1 - c0);
    }
    DD cpk[2];
    for (int k = 0; k < 2; ++k) {
      const bool ok1 = h[2 * k].ok, ok2 = h[2 * k + 1].ok;
      if (ok1 && ok2) cpk[k] = tkk[k].v <= 0.5 * PI ? fmax(v[2 * k], v[2 * k + 1]) : fmin(v[2 * k], v[2 * k + 1]);
      else if (ok1) cpk[k] = v[2 * k];
      else if (ok2) cpk[k] = v[2 * k + 1];
      else cpk[k] = cb[k];
    }
    const double g = lam1 * cpk[0].d + lam2 * cpk[1].d;
    if (g == 0.0) continue;
    if (s < 30) aadd(&A.lout[9 * tplane + 3 * D.base + (s % 3) * P + node_of[s / 3]], (T)g);
    else traw[s - 30] += g;
  }
  // a work-group of fill nodes may span domains: one atomic per node and parameter
  for (int c = 0; c < 3; ++c)
    if (traw[c] != 0.0) aadd(&A.raw[9 * fn.dom + 6 + c], traw[c]);
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

// ---- launchers -----------------------------------------------------------------------------
template <typename S, typename T>
hipError_t launch_adjoint(const AdjArgs<S, T> &a, int64_t tplane, hipStream_t s) {
  const dim3 g(a.n_work), b(kThreads);
  hipLaunchKernelGGL((adj_fwd_c<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_fwd_t<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_fwd_p<S, T>), g, b, 0, s, a);
  const int64_t nz = (int64_t)(A_PLANES - AL_P) * a.aplane;
  hipLaunchKernelGGL((adj_zero<S, T>), dim3(1024), b, 0, s, a, nz);
  hipLaunchKernelGGL((adj_stream<S, T>), g, b, 0, s, a, tplane);
  hipLaunchKernelGGL((adj_collide<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_div<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_stress<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_grad<S, T>), g, b, 0, s, a);
  hipLaunchKernelGGL((adj_comp<S, T>), g, b, 0, s, a, tplane);
  if (a.n_fill > 0)
    hipLaunchKernelGGL((adj_fill<S, T>), dim3((a.n_fill + kThreads - 1) / kThreads), b, 0, s, a, tplane);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_seed(const DomainDev *doms, const WorkItem *work, int n_work, const uint8_t *flags,
                               const double *g, T *lam, int64_t tplane, hipStream_t s) {
  if (n_work > 0)
    hipLaunchKernelGGL((adj_seed<T>), dim3(n_work), dim3(kThreads), 0, s, doms, work, flags, g, lam, tplane);
  return hipGetLastError();
}

template hipError_t launch_adjoint<double, double>(const AdjArgs<double, double> &, int64_t, hipStream_t);
template hipError_t launch_adjoint<float, float>(const AdjArgs<float, float> &, int64_t, hipStream_t);
template hipError_t launch_adjoint_seed<double>(const DomainDev *, const WorkItem *, int, const uint8_t *,
                                                const double *, double *, int64_t, hipStream_t);
template hipError_t launch_adjoint_seed<float>(const DomainDev *, const WorkItem *, int, const uint8_t *,
                                               const double *, float *, int64_t, hipStream_t);

}  // namespace lbm3
