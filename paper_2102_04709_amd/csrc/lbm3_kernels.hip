// lbm3_kernels.hip -- gfx950 kernels of the three-phase colour-gradient D2Q9 step
// (Li, Lu, Jiang & Liu, arXiv:2102.04709, Sec. II).
//
//   wet_fill     sparse kernel over the solid boundary list: Eq. (21)-(22) characteristic-line
//                fill of C at C_SB and the second solid layer, in FP64 for every precision.
//   step_fused   one pass per tile: C_k on tile+3 rings (Eq. 16 densities), Eq. (12) colour
//                gradients and the Eq. (10) stress on tile+2 rings, the stress divergence,
//                Eq. (11) velocity, Eq. (1)-(9) MRT collision and the Eq. (13)-(15) recolouring
//                on tile+1 ring (all in LDS), then the Eq. (16) pull-streaming of the total
//                distribution and of the three partial densities into the tile, with halfway or
//                interpolated bounce-back, the fluid-1/3 exchanging periodic boundary or the
//                Zou-He columns.  The state between steps is the total distribution (9 values)
//                and the partial densities (3 values) per node: the recoloured per-fluid
//                populations of Eq. (13) are f''_{a,k} = C_k f'_a + w_a R_k.e_a with
//                R_k = sum_{l!=k} beta_kl (rho_k rho_l / rho) n_kl, so both their sum over k and
//                their streamed sums over a follow from f', C_k and R_k of the source nodes.
//   mass_*       per-fluid FP64 mass with a fixed summation order.
// No MFMA: the step is a bandwidth-bound stencil with no dense contraction.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lbm3_internal.h"
#include "lbm3_kernels.h"

namespace lbm3 {

// D2Q9 velocities e_0..e_8 and opposite directions (compile-time after unrolling).
__host__ __device__ constexpr int lat_ex(int a) { return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0); }
__host__ __device__ constexpr int lat_ey(int a) { return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0); }
__host__ __device__ constexpr int lat_opp(int a) { return a == 0 ? 0 : (a <= 4 ? (a + 1) % 4 + 1 : (a + 1) % 4 + 5); }
static_assert(lat_opp(1) == 3 && lat_opp(2) == 4 && lat_opp(3) == 1 && lat_opp(4) == 2, "opposites");
static_assert(lat_opp(5) == 7 && lat_opp(6) == 8 && lat_opp(7) == 5 && lat_opp(8) == 6, "opposites");

template <typename T>
__device__ __forceinline__ T wgt(int a) {
  return a == 0 ? T(4.0 / 9.0) : (a < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

template <typename S>
__device__ __forceinline__ float to_f(S v);
template <>
__device__ __forceinline__ float to_f<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_f<__half>(__half v) { return __half2float(v); }

template <typename S, typename T>
__device__ __forceinline__ T load_s(const S *p) {
  return (T)to_f<S>(*p);
}
template <>
__device__ __forceinline__ double load_s<double, double>(const double *p) { return *p; }

template <typename S, typename T>
__device__ __forceinline__ void store_s(S *p, T v) {
  *p = (S)v;
}
template <>
__device__ __forceinline__ void store_s<__half, float>(__half *p, float v) { *p = __float2half_rn(v); }

__device__ __forceinline__ int wrapi(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Index of node (gx, gy) within the domain's plane: periodic axes wrap, the Zou-He x axis
// clamps to the boundary columns (zero-gradient ghost columns), a non-periodic y axis clamps to
// the two off-grid solid rows.
__device__ __forceinline__ int64_t node_index(int gx, int gy, const DomainDev &D) {
  gx = D.bcx == BCX_ZOUHE ? min(max(gx, 0), D.nx - 1) : wrapi(gx, D.nx);
  gy = D.yper ? wrapi(gy, D.ny) : min(max(gy, -2), D.ny + 1);
  return plane_index(gx, gy, D.pitch);
}

// ------------------------------------------------------------------------------------------
// Wetting fill, Eq. (19)-(22).
template <typename T>
__global__ __launch_bounds__(kThreads) void wet_fill(FillArgs<T> A) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= A.n_fill) return;
  const FillNode fn = A.fill[idx];
  const DomainDev &D = A.doms[fn.dom];
  const uint8_t *flags = A.flags + D.base;
  const T *r0 = A.rho + 3 * D.base, *r1 = r0 + D.plane, *r2 = r1 + D.plane;
  auto fluid_at = [&](int i, int j) -> bool {
    if (D.bcx == BCX_ZOUHE) {
      if (i < 0 || i >= D.nx) return false;
    } else {
      i = wrapi(i, D.nx);
    }
    if (D.yper) j = wrapi(j, D.ny);
    else if (j < 0 || j >= D.ny) return false;
    return (flags[plane_index(i, j, D.pitch)] & FL_SOLID) == 0;
  };
  auto cval = [&](int i, int j, double *c) {
    if (D.bcx != BCX_ZOUHE) i = wrapi(i, D.nx);
    if (D.yper) j = wrapi(j, D.ny);
    const int64_t q = plane_index(i, j, D.pitch);
    const double a = (double)r0[q], b = (double)r1[q], d = (double)r2[q];
    const double s = a + b + d;
    c[0] = a / s;
    c[1] = b / s;
    c[2] = d / s;
  };
  auto interp = [&](const LineHit &h, double *c) {
    double c0[3], c1[3];
    cval(h.i0, h.j0, c0);
    cval(h.i1, h.j1, c1);
    for (int k = 0; k < 3; ++k) c[k] = c0[k] + h.w * (c1[k] - c0[k]);
  };
  const double PI = 3.14159265358979323846;
  const double nx = fn.nx, ny = fn.ny, tx = -ny, ty = nx;
  // C used in the weighted contact angle (Eq. 21): the value where the normal line meets the
  // fluid (the set-up guarantees that it does).
  double Cb[3];
  interp(march_line(fn.i, fn.j, nx, ny, fluid_at), Cb);
  double th[2];
  {
    const double a = fmax(Cb[1], 0.0), b = fmax(Cb[2], 0.0), den = a + b;
    th[0] = den > 1e-12 ? (b * D.th13 + a * D.th12) / den : 0.5 * (D.th13 + D.th12);
    const double a2 = fmax(Cb[0], 0.0), den2 = a2 + b;
    const double th21 = PI - D.th12;
    th[1] = den2 > 1e-12 ? (b * D.th23 + a2 * th21) / den2 : 0.5 * (D.th23 + th21);
  }
  double CP[3];
  for (int k = 0; k < 2; ++k) {
    const double tk = fmin(fmax(th[k], 5.0 * PI / 180.0), 175.0 * PI / 180.0);
    const double phi = fabs(0.5 * PI - tk);
    const double c = cos(phi), s = sin(phi);
    const LineHit l1 = march_line(fn.i, fn.j, c * nx + s * tx, c * ny + s * ty, fluid_at);
    const LineHit l2 = march_line(fn.i, fn.j, c * nx - s * tx, c * ny - s * ty, fluid_at);
    double v;
    if (l1.ok && l2.ok) {
      double v1[3], v2[3];
      interp(l1, v1);
      interp(l2, v2);
      v = tk <= 0.5 * PI ? fmax(v1[k], v2[k]) : fmin(v1[k], v2[k]);  // Eq. (22)
    } else if (l1.ok || l2.ok) {
      double v1[3];
      interp(l1.ok ? l1 : l2, v1);
      v = v1[k];
    } else {
      v = Cb[k];
    }
    CP[k] = v;
  }
  CP[2] = 1.0 - CP[0] - CP[1];
  const int64_t q = fn.li;
  T *w0 = A.rho + 3 * D.base;
  w0[q] = (T)CP[0];
  w0[D.plane + q] = (T)CP[1];
  w0[2 * D.plane + q] = (T)CP[2];
}

// ------------------------------------------------------------------------------------------
// Fused step.
template <typename T>
struct Smem {
  T *C0, *C1, *C2, *RH;  // ring 3: mass fractions and total density
  T *Txx, *Txy, *Tyy;    // ring 2: stress of Eq. (10)
  T *N;                  // ring 1, 6 planes: n12, n13, n23 (x, y)
  T *PF;                 // ring 1, 9 planes: post-collision shifted distribution
  T *PR;                 // ring 1, 4 planes: R_1, R_2 of the recolouring
  uint8_t *FL;           // ring 3: flags
};

template <typename T>
__host__ __device__ inline size_t smem_bytes(int TX, int TY) {
  const size_t n3 = (size_t)(TX + 6) * (TY + 6), n2 = (size_t)(TX + 4) * (TY + 4),
               n1 = (size_t)(TX + 2) * (TY + 2);
  return (4 * n3 + 3 * n2 + 19 * n1) * sizeof(T) + ((n3 + 15) & ~(size_t)15);
}

template <typename S, typename T, bool FIELDS>
__global__ __launch_bounds__(kThreads) void step_fused(StepArgs<S, T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int TX = A.tile_x, TY = A.tile_y;
  const int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;
  const int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;
  const int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;
  Smem<T> L;
  {
    T *p = reinterpret_cast<T *>(smem_raw);
    L.C0 = p; p += N3; L.C1 = p; p += N3; L.C2 = p; p += N3; L.RH = p; p += N3;
    L.Txx = p; p += N2; L.Txy = p; p += N2; L.Tyy = p; p += N2;
    L.N = p; p += 6 * N1;
    L.PF = p; p += 9 * N1;
    L.PR = p; p += 4 * N1;
    L.FL = reinterpret_cast<uint8_t *>(p);
  }
  const int tid = threadIdx.x;
  const T eps_g = A.eps_g;

  for (int wi = A.work_begin + blockIdx.x; wi < A.work_end; wi += gridDim.x) {
    const WorkItem wk = A.work[wi];
    const DomainDev &D = A.doms[wk.dom];
    const int x0 = wk.x0, y0 = wk.y0;
    const uint8_t *flags = A.flags + D.base;
    const T *Rin = A.rin + 3 * D.base;
    const S *Fin = A.fin + 9 * D.base;
    const int64_t P = D.plane;

    // Phase A: C_k and rho on tile + 3 rings.
    for (int q = tid; q < N3; q += kThreads) {
      const int lx = q % W3, ly = q / W3;
      const int64_t li = node_index(x0 - 3 + lx, y0 - 3 + ly, D);
      const uint8_t fl = flags[li];
      const T a = Rin[li], b = Rin[P + li], c = Rin[2 * P + li];
      L.FL[q] = fl;
      if (fl & FL_SOLID) {  // the partial densities of solid nodes hold the filled C (rho = 1)
        L.C0[q] = a; L.C1[q] = b; L.C2[q] = c; L.RH[q] = T(1);
      } else {
        const T r = a + b + c;
        L.C0[q] = a / r; L.C1[q] = b / r; L.C2[q] = c / r; L.RH[q] = r;
      }
    }
    __syncthreads();

    // Phase B: Eq. (12) gradients and the Eq. (10) stress on tile + 2 rings.
    for (int q = tid; q < N2; q += kThreads) {
      const int lx = q % W2, ly = q / W2;
      const int p3 = (lx + 1) + (ly + 1) * W3;
      T g[3][2];
      const T *Cs[3] = {L.C0, L.C1, L.C2};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const T *c = Cs[k];
        // 3 * sum_a w_a C(x + e_a) e_a
        const T gx = T(1.0 / 3.0) * (c[p3 + 1] - c[p3 - 1]) +
                     T(1.0 / 12.0) * (c[p3 + 1 + W3] - c[p3 - 1 + W3] - c[p3 - 1 - W3] + c[p3 + 1 - W3]);
        const T gy = T(1.0 / 3.0) * (c[p3 + W3] - c[p3 - W3]) +
                     T(1.0 / 12.0) * (c[p3 + 1 + W3] + c[p3 - 1 + W3] - c[p3 - 1 - W3] - c[p3 + 1 - W3]);
        g[k][0] = gx;
        g[k][1] = gy;
      }
      const T cc[3] = {L.C0[p3], L.C1[p3], L.C2[p3]};
      const T rho = L.RH[p3];
      T txx = 0, txy = 0, tyy = 0;
      T nrm[6];
      const int pk[3] = {0, 0, 1}, pl[3] = {1, 2, 2};
#pragma unroll
      for (int pr = 0; pr < 3; ++pr) {
        const int k = pk[pr], l = pl[pr];
        const T Gx = cc[l] * g[k][0] - cc[k] * g[l][0];
        const T Gy = cc[l] * g[k][1] - cc[k] * g[l][1];
        const T mag = sqrt(Gx * Gx + Gy * Gy);
        const T rk = cc[k] * rho, rl = cc[l] * rho;
        const T Akl = fmin(fmax(T(1e6) * rk * rl, T(0)), T(1));
        if (mag > eps_g) {
          const T nx = Gx / mag, ny = Gy / mag;
          const T coef = (T)D.sig[pr] * Akl * mag;
          txx += coef * (T(1) - nx * nx);
          txy += coef * (-nx * ny);
          tyy += coef * (T(1) - ny * ny);
          nrm[2 * pr] = nx;
          nrm[2 * pr + 1] = ny;
        } else {
          nrm[2 * pr] = T(0);
          nrm[2 * pr + 1] = T(0);
        }
      }
      L.Txx[q] = txx; L.Txy[q] = txy; L.Tyy[q] = tyy;
      if (lx >= 1 && lx <= W2 - 2 && ly >= 1 && ly <= H2 - 2) {
        const int p1 = (lx - 1) + (ly - 1) * W1;
#pragma unroll
        for (int c = 0; c < 6; ++c) L.N[(c) * N1 + p1] = nrm[c];
      }
    }
    __syncthreads();

    // Phase C: force, velocity, MRT collision and recolouring parameters on tile + 1 ring.
    for (int q = tid; q < N1; q += kThreads) {
      const int lx = q % W1, ly = q / W1;
      const int p2 = (lx + 1) + (ly + 1) * W2;
      const int p3 = (lx + 2) + (ly + 2) * W3;
      if (L.FL[p3] & FL_SOLID) continue;
      const bool inside = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY;
      if (FIELDS && !inside) continue;
      const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
      // Zou-He ghost columns are never streaming sources; off-grid rows are flagged solid.
      if (D.bcx == BCX_ZOUHE && (gx < 0 || gx >= D.nx)) continue;
      if (FIELDS && (gx >= D.nx || gy >= D.ny)) continue;
      // F_s = div T, Eq. (12) on the stress components.
      T Fx, Fy;
      {
        const T *xx = L.Txx, *xy = L.Txy, *yy = L.Tyy;
        const int e = p2 + 1, w = p2 - 1, n = p2 + W2, s = p2 - W2;
        const int ne = n + 1, nw = n - 1, sw = s - 1, se = s + 1;
        Fx = T(1.0 / 3.0) * (xx[e] - xx[w]) + T(1.0 / 3.0) * (xy[n] - xy[s]) +
             T(1.0 / 12.0) * (xx[ne] - xx[nw] - xx[sw] + xx[se] + xy[ne] + xy[nw] - xy[sw] - xy[se]);
        Fy = T(1.0 / 3.0) * (xy[e] - xy[w]) + T(1.0 / 3.0) * (yy[n] - yy[s]) +
             T(1.0 / 12.0) * (xy[ne] - xy[nw] - xy[sw] + xy[se] + yy[ne] + yy[nw] - yy[sw] - yy[se]);
      }
      const int64_t li = node_index(gx, gy, D);
      T f[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) f[a] = load_s<S, T>(Fin + a * P + li);
      // moments of the shifted distribution (M of Eq. 4 applied to f - w)
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
      Fx += rho * (T)D.g[0];
      Fy += rho * (T)D.g[1];
      const T irho = T(1) / rho;
      const T ux = (jx + T(0.5) * Fx) * irho, uy = (jy + T(0.5) * Fy) * irho;  // Eq. (11)
      const T r0 = L.C0[p3] * L.RH[p3], r1 = L.C1[p3] * L.RH[p3], r2 = L.C2[p3] * L.RH[p3];
      if (FIELDS) {
        const int64_t o = (int64_t)gy * D.nx + gx;
        const int64_t n = (int64_t)D.nx * D.ny;
        if (A.out_u) {
          A.out_u[o] = ux;
          A.out_u[n + o] = uy;
        }
        if (A.out_force) {
          A.out_force[o] = Fx;
          A.out_force[n + o] = Fy;
        }
        continue;
      }
      // Eq. (7): tau = 1/2 + 3 / sum_k rho_k / mu_k; Eq. (6) rates.
      const T tau = T(0.5) + T(3) / (r0 / (T)D.nu[0] + r1 / (T)D.nu[1] + r2 / (T)D.nu[2]);
      const T s1 = T(1) / tau;
      const T s4 = T(8) * (T(2) - s1) / (T(8) - s1);
      const T uu = ux * ux + uy * uy;
      const T ruu = rho * uu;
      const T uF = ux * Fx + uy * Fy;
      const T h1 = T(1) - T(0.5) * s1, h4 = T(1) - T(0.5) * s4;
      // Delta_i = S_i (m_i - meq_i) - (1 - S_i/2) mF_i, scaled by diag(M M^T)^-1
      const T d1 = (s1 * (m1 - (-T(2) * drho + T(3) * ruu)) - h1 * T(6) * uF) * T(1.0 / 36.0);
      const T d2 = (s1 * (m2 - (drho - T(3) * ruu)) + h1 * T(6) * uF) * T(1.0 / 36.0);
      const T d3 = -Fx * T(1.0 / 6.0);
      const T d4 = (s4 * (m4 + rho * ux) + h4 * Fx) * T(1.0 / 12.0);
      const T d5 = -Fy * T(1.0 / 6.0);
      const T d6 = (s4 * (m6 + rho * uy) + h4 * Fy) * T(1.0 / 12.0);
      const T d7 = (s1 * (m7 - rho * (ux * ux - uy * uy)) - h1 * T(2) * (ux * Fx - uy * Fy)) * T(0.25);
      const T d8 = (s1 * (m8 - rho * ux * uy) - h1 * (ux * Fy + uy * Fx)) * T(0.25);
      // f' = f - M^T d
      T fd[9];
      fd[0] = f[0] - (-T(4) * d1 + T(4) * d2);
      fd[1] = f[1] - (-d1 - T(2) * d2 + d3 - T(2) * d4 + d7);
      fd[2] = f[2] - (-d1 - T(2) * d2 + d5 - T(2) * d6 - d7);
      fd[3] = f[3] - (-d1 - T(2) * d2 - d3 + T(2) * d4 + d7);
      fd[4] = f[4] - (-d1 - T(2) * d2 - d5 + T(2) * d6 - d7);
      fd[5] = f[5] - (T(2) * d1 + d2 + d3 + d4 + d5 + d6 + d8);
      fd[6] = f[6] - (T(2) * d1 + d2 - d3 - d4 + d5 + d6 - d8);
      fd[7] = f[7] - (T(2) * d1 + d2 - d3 - d4 - d5 - d6 + d8);
      fd[8] = f[8] - (T(2) * d1 + d2 + d3 + d4 - d5 - d6 - d8);
#pragma unroll
      for (int a = 0; a < 9; ++a) L.PF[(a) * N1 + q] = fd[a];
      // Recolouring, Eq. (13)-(15): R_1, R_2 (R_3 = -R_1 - R_2).
      const T rt = L.RH[p3];
      const T irt = T(1) / rt;
      T r3 = T(35) * r0 * r1 * r2 * irt * irt * irt;
      r3 = fmin(fmax(r3, T(0)), T(1));
      const T b0 = (T)D.beta0;
      const T b12 = b0 + b0 * r3 * (T)D.gX[0];
      const T b13 = b0 + b0 * r3 * (T)D.gX[1];
      const T b23 = b0 + b0 * r3 * (T)D.gX[2];
      const T a12 = b12 * r0 * r1 * irt, a13 = b13 * r0 * r2 * irt, a23 = b23 * r1 * r2 * irt;
      L.PR[(0) * N1 + q] = a12 * L.N[(0) * N1 + q] + a13 * L.N[(2) * N1 + q];
      L.PR[(1) * N1 + q] = a12 * L.N[(1) * N1 + q] + a13 * L.N[(3) * N1 + q];
      L.PR[(2) * N1 + q] = -a12 * L.N[(0) * N1 + q] + a23 * L.N[(4) * N1 + q];
      L.PR[(3) * N1 + q] = -a12 * L.N[(1) * N1 + q] + a23 * L.N[(5) * N1 + q];
    }
    if (FIELDS) {
      // partial densities (or filled C) of the tile
      for (int q = tid; q < TX * TY; q += kThreads) {
        const int lx = q % TX, ly = q / TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= D.nx || gy >= D.ny) continue;
        const int64_t li = plane_index(gx, gy, D.pitch);
        const int64_t o = (int64_t)gy * D.nx + gx, n = (int64_t)D.nx * D.ny;
        const bool solid = flags[li] & FL_SOLID;
        for (int k = 0; k < 3; ++k) A.out_rho[k * n + o] = Rin[k * P + li];
        if (solid) {
          if (A.out_u) { A.out_u[o] = 0; A.out_u[n + o] = 0; }
          if (A.out_force) { A.out_force[o] = 0; A.out_force[n + o] = 0; }
        }
      }
      __syncthreads();
      continue;
    }
    __syncthreads();

    // Phase D: pull-streaming into the tile, Eq. (16), with the boundary rules.
    T *Rout = A.rout + 3 * D.base;
    S *Fout = A.fout + 9 * D.base;
    for (int q = tid; q < TX * TY; q += kThreads) {
      const int lx = q % TX, ly = q / TX;
      const int gx = x0 + lx, gy = y0 + ly;
      if (gx >= D.nx || gy >= D.ny) continue;
      const int64_t li = plane_index(gx, gy, D.pitch);
      const int p1 = (lx + 1) + (ly + 1) * W1;
      const int p3 = (lx + 3) + (ly + 3) * W3;
      const uint8_t fl = L.FL[p3];
      if (fl & FL_SOLID) {
#pragma unroll
        for (int a = 0; a < 9; ++a) store_s<S, T>(Fout + a * P + li, T(0));
        Rout[li] = T(0); Rout[P + li] = T(0); Rout[2 * P + li] = T(0);
        continue;
      }
      T fo[9];
      T ra = 0, rb = 0, rc = 0;
      const T Cn[3] = {L.C0[p3], L.C1[p3], L.C2[p3]};
      const IbbNode *ib = nullptr;
      if ((fl & FL_CURVED) && D.n_ibb > 0) {
        int lo = D.ibb_off, hi = D.ibb_off + D.n_ibb - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (A.ibb[mid].li < li) lo = mid + 1;
          else hi = mid;
        }
        ib = &A.ibb[lo];
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const int ex = lat_ex(a), ey = lat_ey(a);
        const int sx = gx - ex;
        if (D.bcx == BCX_ZOUHE && (sx < 0 || sx >= D.nx)) {  // set by the Zou-He rule below
          fo[a] = 0;
          continue;
        }
        const T w = wgt<T>(a);
        const int s1 = p1 - ex - ey * W1, s3 = p3 - ex - ey * W3;
        if (!(L.FL[s3] & FL_SOLID)) {
          const T fs = L.PF[(a) * N1 + s1];
          fo[a] = fs;
          const T ft = fs + w;
          const T Cs0 = L.C0[s3], Cs1 = L.C1[s3], Cs2 = L.C2[s3];
          const T R1 = L.PR[(0) * N1 + s1] * ex + L.PR[(1) * N1 + s1] * ey;
          const T R2 = L.PR[(2) * N1 + s1] * ex + L.PR[(3) * N1 + s1] * ey;
          const T R3 = -(R1 + R2);
          const T c0 = Cs0 * ft + w * R1, c1 = Cs1 * ft + w * R2, c2 = Cs2 * ft + w * R3;
          const bool crossed = D.bcx == BCX_SWAP13 && (sx < 0 || sx >= D.nx);
          if (crossed) { ra += c2; rb += c1; rc += c0; }
          else { ra += c0; rb += c1; rc += c2; }
        } else {
          // the link x -> x - e_a ends in a solid node: bounce-back of the populations
          // leaving x along -e_a (direction ab)
          const int ab = lat_opp(a);
          const T qd = ib ? (T)ib->q[a - 1] : T(0.5);
          const int eax = -ex, eay = -ey;  // e_ab
          const T fab = L.PF[(ab) * N1 + p1];
          auto part = [&](int p1x, int p3x, int dir, int dx, int dy, T *out) {
            const T fv = L.PF[(dir) * N1 + p1x] + w;
            const T R1 = L.PR[(0) * N1 + p1x] * dx + L.PR[(1) * N1 + p1x] * dy;
            const T R2 = L.PR[(2) * N1 + p1x] * dx + L.PR[(3) * N1 + p1x] * dy;
            out[0] = L.C0[p3x] * fv + w * R1;
            out[1] = L.C1[p3x] * fv + w * R2;
            out[2] = L.C2[p3x] * fv + w * (-(R1 + R2));
          };
          T own_ab[3];
          part(p1, p3, ab, eax, eay, own_ab);
          const int n1 = p1 + ex + ey * W1, n3 = p3 + ex + ey * W3;
          if (qd < T(0.5) && !(L.FL[n3] & FL_SOLID)) {
            T nb_ab[3];
            part(n1, n3, ab, eax, eay, nb_ab);
            const T c1 = T(2) * qd, c2 = T(1) - T(2) * qd;
            fo[a] = c1 * fab + c2 * L.PF[(ab) * N1 + n1];
            ra += c1 * own_ab[0] + c2 * nb_ab[0];
            rb += c1 * own_ab[1] + c2 * nb_ab[1];
            rc += c1 * own_ab[2] + c2 * nb_ab[2];
          } else if (qd < T(0.5)) {
            fo[a] = fab;
            ra += own_ab[0]; rb += own_ab[1]; rc += own_ab[2];
          } else {
            T own_a[3];
            part(p1, p3, a, ex, ey, own_a);
            const T c1 = T(1) / (T(2) * qd), c2 = T(1) - c1;
            fo[a] = c1 * fab + c2 * L.PF[(a) * N1 + p1];
            ra += c1 * own_ab[0] + c2 * own_a[0];
            rb += c1 * own_ab[1] + c2 * own_a[1];
            rc += c1 * own_ab[2] + c2 * own_a[2];
          }
        }
      }
      if (D.bcx == BCX_ZOUHE && (gx == 0 || gx == D.nx - 1)) {
        // Zou-He non-equilibrium bounce-back on the total distribution (unshifted).
        T ft[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) ft[a] = fo[a] + wgt<T>(a);
        if (gx == 0) {
          const T u = (T)D.u_in;
          const T rw = (ft[0] + ft[2] + ft[4] + T(2) * (ft[3] + ft[6] + ft[7])) / (T(1) - u);
          ft[1] = ft[3] + T(2.0 / 3.0) * rw * u;
          ft[5] = ft[7] - T(0.5) * (ft[2] - ft[4]) + rw * u / T(6);
          ft[8] = ft[6] + T(0.5) * (ft[2] - ft[4]) + rw * u / T(6);
          // incoming populations carry pure fluid 3
          rc += ft[1] + ft[5] + ft[8];
          fo[1] = ft[1] - wgt<T>(1);
          fo[5] = ft[5] - wgt<T>(5);
          fo[8] = ft[8] - wgt<T>(8);
        } else {
          const T ro = (T)D.rho_out;
          const T ux = -T(1) + (ft[0] + ft[2] + ft[4] + T(2) * (ft[1] + ft[5] + ft[8])) / ro;
          ft[3] = ft[1] - T(2.0 / 3.0) * ro * ux;
          ft[7] = ft[5] + T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
          ft[6] = ft[8] - T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
          // unknown populations carry the node's own composition
          ra += Cn[0] * ft[3]; rb += Cn[1] * ft[3]; rc += Cn[2] * ft[3];
          ra += Cn[0] * ft[6]; rb += Cn[1] * ft[6]; rc += Cn[2] * ft[6];
          ra += Cn[0] * ft[7]; rb += Cn[1] * ft[7]; rc += Cn[2] * ft[7];
          fo[3] = ft[3] - wgt<T>(3);
          fo[6] = ft[6] - wgt<T>(6);
          fo[7] = ft[7] - wgt<T>(7);
        }
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) store_s<S, T>(Fout + a * P + li, fo[a]);
      Rout[li] = ra;
      Rout[P + li] = rb;
      Rout[2 * P + li] = rc;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Per-fluid mass: partial sums per (domain, 16-row chunk), then a fixed-order final sum.
template <typename T>
__global__ __launch_bounds__(kThreads) void mass_partial(MassArgs<T> A) {
  __shared__ double red[3][kThreads];
  const int c = blockIdx.x;
  const int dom = A.chunk_dom[c];
  const DomainDev &D = A.doms[dom];
  const int j0 = (c - A.chunk_first[dom]) * 16;
  const T *R = A.rho + 3 * D.base;
  const uint8_t *flags = A.flags + D.base;
  double s[3] = {0, 0, 0};
  int bad = 0;
  for (int j = j0; j < min(j0 + 16, D.ny); ++j)
    for (int i = threadIdx.x; i < D.nx; i += kThreads) {
      const int64_t li = plane_index(i, j, D.pitch);
      if (flags[li] & FL_SOLID) continue;
      for (int k = 0; k < 3; ++k) {
        const double v = (double)R[k * D.plane + li];
        if (!isfinite(v)) bad = 1;
        s[k] += v;
      }
    }
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
  if (bad) A.bad[0] = 1;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) A.partial[3 * c + k] = red[k][0];
}

__global__ void mass_final(const double *partial, const int *chunk_first, int n_dom, double *out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * n_dom) return;
  const int d = t / 3, k = t % 3;
  double s = 0;
  for (int c = chunk_first[d]; c < chunk_first[d + 1]; ++c) s += partial[3 * c + k];
  out[t] = s;
}

// ------------------------------------------------------------------------------------------
// Launchers.
template <typename T>
hipError_t launch_fill(const FillArgs<T> &a, hipStream_t s) {
  if (a.n_fill <= 0) return hipSuccess;
  const int blocks = (a.n_fill + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(wet_fill<T>, dim3(blocks), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <typename S, typename T>
hipError_t launch_step(const StepArgs<S, T> &a, int grid, bool fields, hipStream_t s) {
  const size_t sm = smem_bytes<T>(a.tile_x, a.tile_y);
  if (fields)
    hipLaunchKernelGGL((step_fused<S, T, true>), dim3(grid), dim3(kThreads), sm, s, a);
  else
    hipLaunchKernelGGL((step_fused<S, T, false>), dim3(grid), dim3(kThreads), sm, s, a);
  return hipGetLastError();
}

// Allows every fused-kernel instantiation the full 160 KiB of LDS of a gfx950 work-group.
hipError_t init_kernel_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess, r;
#define LBM3_ATTR(S, T, F)                                                                    \
  r = hipFuncSetAttribute((const void *)step_fused<S, T, F>,                                  \
                          hipFuncAttributeMaxDynamicSharedMemorySize, lim);                   \
  if (r != hipSuccess) e = r;
  LBM3_ATTR(double, double, false)
  LBM3_ATTR(double, double, true)
  LBM3_ATTR(float, float, false)
  LBM3_ATTR(float, float, true)
  LBM3_ATTR(__half, float, false)
  LBM3_ATTR(__half, float, true)
#undef LBM3_ATTR
  return e;
}

template <typename T>
hipError_t launch_mass(const MassArgs<T> &a, int n_chunks, int n_dom, double *out, hipStream_t s) {
  hipLaunchKernelGGL(mass_partial<T>, dim3(n_chunks), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(mass_final, dim3((3 * n_dom + 63) / 64), dim3(64), 0, s, a.partial, a.chunk_first, n_dom, out);
  return hipGetLastError();
}

size_t step_smem_bytes(int precision, int tx, int ty) {
  return precision == 0 ? smem_bytes<double>(tx, ty) : smem_bytes<float>(tx, ty);
}

template hipError_t launch_fill<double>(const FillArgs<double> &, hipStream_t);
template hipError_t launch_fill<float>(const FillArgs<float> &, hipStream_t);
template hipError_t launch_step<double, double>(const StepArgs<double, double> &, int, bool, hipStream_t);
template hipError_t launch_step<float, float>(const StepArgs<float, float> &, int, bool, hipStream_t);
template hipError_t launch_step<__half, float>(const StepArgs<__half, float> &, int, bool, hipStream_t);
template hipError_t launch_mass<double>(const MassArgs<double> &, int, int, double *, hipStream_t);
template hipError_t launch_mass<float>(const MassArgs<float> &, int, int, double *, hipStream_t);

}  // namespace lbm3
