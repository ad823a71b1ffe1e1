// lbm3_device.h -- per-node device code of liblbm3 shared by the forward kernels and the adjoint
// kernels (lattice constants, storage conversions, node indexing, the wetting fill of one node,
// the colour-gradient stress, the MRT collision with forcing, the recolouring vectors and the
// pull-streaming of one node).  Every function is a template on the arithmetic type (FP64 or
// FP32); the adjoint recomputes its forward intermediates with the same functions.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lbm3_internal.h"

namespace lbm3 {

// D2Q9 velocities e_0..e_8 and opposite directions (compile-time after unrolling).
__host__ __device__ constexpr int lat_ex(int a) { return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0); }
__host__ __device__ constexpr int lat_ey(int a) { return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0); }
__host__ __device__ constexpr int lat_opp(int a) { return a == 0 ? 0 : (a <= 4 ? (a + 1) % 4 + 1 : (a + 1) % 4 + 5); }
static_assert(lat_opp(1) == 3 && lat_opp(2) == 4 && lat_opp(3) == 1 && lat_opp(4) == 2, "opposites");
static_assert(lat_opp(5) == 7 && lat_opp(6) == 8 && lat_opp(7) == 5 && lat_opp(8) == 6, "opposites");

// e.(x, y) for lattice components in {-1, 0, 1} (compile-time after unrolling), written without
// products by zero: x * 0 does not fold away under IEEE rules, and the sum is exact either way.
template <typename T>
__device__ __forceinline__ T edot(int ex, int ey, T x, T y) {
  const T tx = ex > 0 ? x : -x, ty = ey > 0 ? y : -y;
  return ex == 0 ? (ey == 0 ? T(0) : ty) : (ey == 0 ? tx : tx + ty);
}

template <typename T>
__device__ __forceinline__ T wgt(int a) {
  return a == 0 ? T(4.0 / 9.0) : (a < 5 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

// Reciprocal: the hardware reciprocal (1 ulp) in FP32, an IEEE division in FP64.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }

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

// Element i of a plane whose base is the same for the whole wave, addressed as that base plus a
// 32-bit byte offset: gfx950's global loads and stores take this form directly (scalar base,
// 32-bit vector offset), so no 64-bit address is formed per lane.  The empty asm keeps the base
// in scalar registers and stops the compiler from folding the planes' distance into the per-lane
// address instead.  lbm3_create keeps every domain's plane of the arithmetic type below 4 GiB,
// and plane indices are never negative.
template <typename V>
__device__ __forceinline__ V *elem32(V *base, int64_t i) {
  using B = typename std::conditional<std::is_const<V>::value, const char, char>::type;
  using GB = __attribute__((address_space(1))) B;  // the global address space (not a flat access)
  uint64_t u = reinterpret_cast<uint64_t>(base);
  asm("" : "+s"(u));
  GB *g = reinterpret_cast<GB *>(u) + (uint32_t)i * (uint32_t)sizeof(V);
  return (V *)g;
}

template <typename S, typename T>
__device__ __forceinline__ void store_s(S *p, T v) {
  *p = (S)v;
}
template <>
__device__ __forceinline__ void store_s<__half, float>(__half *p, float v) { *p = __float2half_rn(v); }

// Streaming store of the next state: written once per step and read back only by the next
// launch, so it is marked non-temporal (the write does not displace cached neighbour rows).
template <typename S, typename T>
__device__ __forceinline__ void store_nt(S *p, T v) {
  __builtin_nontemporal_store((S)v, p);
}
template <>
__device__ __forceinline__ void store_nt<__half, float>(__half *p, float v) {
  const __half h = __float2half_rn(v);
  __builtin_nontemporal_store(*reinterpret_cast<const unsigned short *>(&h), reinterpret_cast<unsigned short *>(p));
}

// v mod n for any v (the characteristic lines of the wetting fill reach up to 24 nodes away).
__device__ __forceinline__ int wrap_small(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

// v mod n for v in [-n, 2n): the stencil and halo offsets (at most 3) on axes of at least 3 nodes,
// which lbm3_create requires.  One select instead of a loop (the adjoint's kernels; in the fused
// step kernel the loop form gives the better register allocation).
__device__ __forceinline__ int wrap_near(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Index of node (gx, gy) within the domain's plane: periodic axes wrap, the Zou-He x axis
// clamps to the boundary columns (zero-gradient ghost columns), a non-periodic y axis clamps to
// the two off-grid solid rows.
__device__ __forceinline__ int64_t node_index(int gx, int gy, const DomainDev &D) {
  gx = D.bcx == BCX_ZOUHE ? min(max(gx, 0), D.nx - 1) : wrap_small(gx, D.nx);
  gy = D.yper ? wrap_small(gy, D.ny) : min(max(gy, -2), D.ny + 1);
  return plane_index(gx, gy, D.pitch);
}

// ------------------------------------------------------------------------------------------
// Wetting fill, Eq. (19)-(22), of one solid boundary node (the wet_fill kernel runs it for every
// fill node once per step and writes the filled C to a compact array).  All geometry is FP64; C
// at fluid nodes is rho_k / rho of the stored densities.  The march tests fluid nodes with the
// node's 11 x 11 fluid mask and reads the flag plane only beyond it.
template <typename T>
__device__ __forceinline__ double cfrac_at(const T *r, int64_t P, int64_t q, int k) {
  const double a = (double)r[q], b = (double)r[P + q], d = (double)r[2 * P + q];
  const double v = k == 0 ? a : (k == 1 ? b : d);
  return v / (a + b + d);
}

// Lane `line` (0..3) of the four lanes that fill one node: fluid k = line / 2, side
// s = line % 2.  Every lane forms C at D0 and the angle of its fluid, marches its line and
// interpolates; the lanes of a fluid then combine their values with Eq. (22) and lane 0
// receives the second fluid's value.  Returns (C1, C2) in lane 0.  `stage` runs in every lane
// right before the march (it places the node's far mask at `far_rows`, a work-group barrier).
// cand (may be null): the line's crossings for the pure-composition angles of its fluid; when C at
// D0 leaves Eq. (21) one of them (the other two fluids' weights below 1e-15 of their sum, or both
// absent) the line takes that crossing instead of marching; a line whose angle lies in a
// candidate's range (FillCand) starts its march at the candidate's crossing.  The densities at the
// first candidate's nodes (the angle against fluid 3, the usual ambient) are loaded together with
// those of D0, and used wherever the line's crossing has those nodes.
template <typename T, class Stage>
__device__ __forceinline__ void fill_lanes(const FillNode &fn, const DomainDev &D, const uint8_t *flags,
                                           const T *r, const uint32_t *far_rows, const Stage &stage, int line,
                                           bool active, double &c1, double &c2, const FillCand *cand = nullptr) {
  const int64_t P = D.plane;
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
  const double PI = 3.14159265358979323846;
  const int k = line >> 1;
  // the line's first candidate crossing (the angle against fluid 3, the usual ambient) and its
  // densities, beside those of D0 (the other two candidates load where they are needed)
  const FillCand c0 = cand ? cand[0] : FillCand{-1, -1, 0.0, 1.0, 0.0, 1, 1};
  T rc0[2][3];
  {
    const int64_t qa = c0.a >= 0 ? c0.a : fn.d0a, qb = c0.a >= 0 ? c0.b : fn.d0a;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      rc0[0][q] = r[q * P + qa];
      rc0[1][q] = r[q * P + qb];
    }
  }
  // C at D0 for the weighted contact angle of Eq. (21).
  double Cb[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double ca = cfrac_at(r, P, fn.d0a, q), cb = cfrac_at(r, P, fn.d0b, q);
    Cb[q] = ca + fn.d0w * (cb - ca);
  }
  double th;
  int pick = -1;  // the candidate crossing that applies (-1: march)
  if (k == 0) {
    const double a = fmax(Cb[1], 0.0), b = fmax(Cb[2], 0.0), den = a + b;
    th = den > 1e-12 ? (b * D.th13 + a * D.th12) / den : 0.5 * (D.th13 + D.th12);
    pick = !(den > 1e-12) ? 2 : (a <= 1e-15 * den ? 0 : (b <= 1e-15 * den ? 1 : -1));
  } else {
    const double a2 = fmax(Cb[0], 0.0), b = fmax(Cb[2], 0.0), den2 = a2 + b;
    const double th21 = PI - D.th12;
    th = den2 > 1e-12 ? (b * D.th23 + a2 * th21) / den2 : 0.5 * (D.th23 + th21);
    pick = !(den2 > 1e-12) ? 2 : (a2 <= 1e-15 * den2 ? 0 : (b <= 1e-15 * den2 ? 1 : -1));
  }
  if (!cand) pick = -1;
  const double tk = fmin(fmax(th, 5.0 * PI / 180.0), 175.0 * PI / 180.0);
  double v = 0.0;
  int ok = 0;
  stage();
  // the crossing's interpolation nodes and weight (qa < 0: none)
  int64_t qa = -1, qb = -1;
  double w_hit = 0.0;
  if (active && pick >= 0) {  // a precomputed crossing
    const FillCand h = pick == 0 ? c0 : cand[pick];
    if (h.a >= 0) { qa = h.a; qb = h.b; w_hit = h.w; }
  } else if (active) {
    const double phi = fabs(0.5 * PI - tk);
    double sp, cp;
    sincos_quadrant(phi, sp, cp);
    if (line & 1) sp = -sp;
    const double nx = fn.nx, ny = fn.ny, tx = -ny, ty = nx;
    // within a candidate's angle range the march meets its hit at the candidate's crossing: it
    // starts there (the usual case of a composition with traces of a third fluid)
    int kx = 1, ky = 1;
    if (phi >= c0.phi_lo && phi <= c0.phi_hi) {
      kx = c0.kx; ky = c0.ky;
    } else if (cand) {
#pragma unroll
      for (int c = 1; c < kFillCands; ++c) {
        const FillCand h = cand[c];
        if (phi >= h.phi_lo && phi <= h.phi_hi) { kx = h.kx; ky = h.ky; }
      }
    }
    const LineHit h = march_line_masked(fn.i, fn.j, cp * nx + sp * tx, cp * ny + sp * ty, fn.mask, far_rows,
                                        fluid_at, kx, ky);
    if (h.ok) { qa = node_q(h.i0, h.j0); qb = node_q(h.i1, h.j1); w_hit = h.w; }
  }
  if (qa >= 0 && c0.a == qa && c0.b == qb) {  // the first candidate's nodes: densities in
    const double ca = (double)rc0[0][k] / ((double)rc0[0][0] + (double)rc0[0][1] + (double)rc0[0][2]);
    const double cb = (double)rc0[1][k] / ((double)rc0[1][0] + (double)rc0[1][1] + (double)rc0[1][2]);
    v = ca + w_hit * (cb - ca);
    ok = 1;
  } else if (qa >= 0) {
    const double ca = cfrac_at(r, P, qa, k), cb = cfrac_at(r, P, qb, k);
    v = ca + w_hit * (cb - ca);
    ok = 1;
  }
  const double vo = __shfl_xor(v, 1);
  const int oko = __shfl_xor(ok, 1);
  double c;
  if (ok && oko) c = tk <= 0.5 * PI ? fmax(v, vo) : fmin(v, vo);  // Eq. (22)
  else if (ok) c = v;
  else if (oko) c = vo;
  else c = Cb[k];
  c1 = c;
  c2 = __shfl_xor(c, 2);
}

// Index of the fill node whose data a solid fill node's first density slot holds.
__device__ __forceinline__ int fill_index(float v) { return __float_as_int(v); }
__device__ __forceinline__ int fill_index(double v) { return (int)__double_as_longlong(v); }

// C and rho of a loaded node for the colour-gradient stencil: fluid nodes give rho_k / rho;
// fill nodes the filled C of this step (rho := 1); other solid nodes zero (rho := 1).
template <typename T>
__device__ __forceinline__ void node_composition(uint8_t fl, T a, T b, T c, const T *fillC, T out[4]) {
  if (fl & FL_SOLID) {
    if (fl & FL_FILL) {
      const T *v = fillC + 3 * fill_index(a);
      out[0] = v[0]; out[1] = v[1]; out[2] = v[2];
    } else {
      out[0] = out[1] = out[2] = T(0);
    }
    out[3] = T(1);
  } else {
    const T r = a + b + c;
    const T ir = rcp(r);
    out[0] = a * ir; out[1] = b * ir; out[2] = c * ir; out[3] = r;
  }
}

// ------------------------------------------------------------------------------------------
// Per-node pieces of the fused step, shared by the tile and the strip kernels.  Neighbour
// values are passed in D2Q9 order c[a] = psi(x + e_a).

// Per-domain constants in the compute type, read once per work item.
template <typename T>
struct KT {
  T inu[3];  // 1 / nu_k
  T sig[3];  // sigma12, sigma13, sigma23
  T gX[3];   // g(X_kl) for the pairs 12, 13, 23
  T b0, g0, g1, u_in, rho_out;
};

template <typename T>
__device__ __forceinline__ KT<T> make_kt(const DomainDev &D) {
  KT<T> K;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    K.inu[k] = (T)D.inu[k];
    K.sig[k] = (T)D.sig[k];
    K.gX[k] = (T)D.gX[k];
  }
  K.b0 = (T)D.beta0;
  K.g0 = (T)D.g[0];
  K.g1 = (T)D.g[1];
  K.u_in = (T)D.u_in;
  K.rho_out = (T)D.rho_out;
  return K;
}

// Eq. (12): (1/c_s^2) sum_a w_a psi(x + e_a) e_a.
template <typename T>
__device__ __forceinline__ void grad9(const T *c, T &gx, T &gy) {
  gx = T(1.0 / 3.0) * (c[1] - c[3]) + T(1.0 / 12.0) * (c[5] - c[6] - c[7] + c[8]);
  gy = T(1.0 / 3.0) * (c[2] - c[4]) + T(1.0 / 12.0) * (c[5] + c[6] - c[7] - c[8]);
}

// |G| and 1/|G| of a colour-gradient difference, when |G| > eps (else false): the hardware
// reciprocal square root (1 ulp) in FP32, an IEEE square root and division in FP64.
__device__ __forceinline__ bool pair_norm(float gx, float gy, float eps, float &mag, float &im) {
  const float s2 = gx * gx + gy * gy;
  if (!(s2 > eps * eps)) return false;
  im = __builtin_amdgcn_rsqf(s2);
  mag = s2 * im;
  return true;
}
__device__ __forceinline__ bool pair_norm(double gx, double gy, double eps, double &mag, double &im) {
  mag = sqrt(gx * gx + gy * gy);
  if (!(mag > eps)) return false;
  im = 1.0 / mag;
  return true;
}

// Eq. (10) stress sum over the fluid pairs 12, 13, 23 (the double sum over ordered pairs with
// the factor 1/2 equals the sum over unordered pairs, since G_lk = -G_kl), and the pair normals
// n_kl = G_kl / |G_kl| (zero when |G_kl| <= eps).  Returns whether any pair had |G_kl| > eps
// (otherwise the stress is +0 in all three components and the normals are zero).
template <typename T>
__device__ __forceinline__ bool pair_stress(const T cc[3], const T g[3][2], T rho, const KT<T> &K,
                                            T eps, T &txx, T &txy, T &tyy, T nrm[6]) {
  txx = txy = tyy = T(0);
  bool any = false;
  const int pk[3] = {0, 0, 1}, pl[3] = {1, 2, 2};
#pragma unroll
  for (int pr = 0; pr < 3; ++pr) {
    const int k = pk[pr], l = pl[pr];
    const T Gx = cc[l] * g[k][0] - cc[k] * g[l][0];
    const T Gy = cc[l] * g[k][1] - cc[k] * g[l][1];
    const T rk = cc[k] * rho, rl = cc[l] * rho;
    const T Akl = fmin(fmax(T(1e6) * rk * rl, T(0)), T(1));
    T mag, im;
    if (pair_norm(Gx, Gy, eps, mag, im)) {
      any = true;
      const T nx = Gx * im, ny = Gy * im;
      const T coef = K.sig[pr] * Akl * mag;
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
  return any;
}

// F_s = div T with Eq. (12) on the stress components.
template <typename T>
__device__ __forceinline__ void div_stress(const T *xx, const T *xy, const T *yy, T &Fx, T &Fy) {
  Fx = T(1.0 / 3.0) * (xx[1] - xx[3]) + T(1.0 / 3.0) * (xy[2] - xy[4]) +
       T(1.0 / 12.0) * (xx[5] - xx[6] - xx[7] + xx[8] + xy[5] + xy[6] - xy[7] - xy[8]);
  Fy = T(1.0 / 3.0) * (xy[1] - xy[3]) + T(1.0 / 3.0) * (yy[2] - yy[4]) +
       T(1.0 / 12.0) * (xy[5] - xy[6] - xy[7] + xy[8] + yy[5] + yy[6] - yy[7] - yy[8]);
}

// Eq. (1)-(9), (11) on the shifted distribution f - w: MRT collision with the forcing term at
// the mixture relaxation time of Eq. (7).  Fx, Fy enter as the interfacial force and leave as
// the total force (the body acceleration times rho added).
template <typename T>
__device__ __forceinline__ void collide_shifted(const T f[9], T &Fx, T &Fy, T r0, T r1, T r2,
                                                const KT<T> &K, T fd[9], T &ux, T &uy) {
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
  Fx += rho * K.g0;
  Fy += rho * K.g1;
  const T irho = rcp(rho);
  ux = (jx + T(0.5) * Fx) * irho;
  uy = (jy + T(0.5) * Fy) * irho;
  // s1 = 1 / tau with tau = 1/2 + 3 / sum_k rho_k / mu_k
  const T sum = r0 * K.inu[0] + r1 * K.inu[1] + r2 * K.inu[2];
  const T s1 = sum * rcp(T(0.5) * sum + T(3));
  const T s4 = T(8) * (T(2) - s1) * rcp(T(8) - s1);
  const T ruu = rho * (ux * ux + uy * uy);
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
  fd[0] = f[0] - (-T(4) * d1 + T(4) * d2);
  fd[1] = f[1] - (-d1 - T(2) * d2 + d3 - T(2) * d4 + d7);
  fd[2] = f[2] - (-d1 - T(2) * d2 + d5 - T(2) * d6 - d7);
  fd[3] = f[3] - (-d1 - T(2) * d2 - d3 + T(2) * d4 + d7);
  fd[4] = f[4] - (-d1 - T(2) * d2 - d5 + T(2) * d6 - d7);
  fd[5] = f[5] - (T(2) * d1 + d2 + d3 + d4 + d5 + d6 + d8);
  fd[6] = f[6] - (T(2) * d1 + d2 - d3 - d4 + d5 + d6 - d8);
  fd[7] = f[7] - (T(2) * d1 + d2 - d3 - d4 - d5 - d6 + d8);
  fd[8] = f[8] - (T(2) * d1 + d2 + d3 + d4 - d5 - d6 - d8);
}

// Eq. (13)-(15): R_k = sum_{l != k} beta_kl (rho_k rho_l / rho) n_kl for k = 1, 2
// (R_3 = -R_1 - R_2); out = (R_1x, R_1y, R_2x, R_2y).
template <typename T>
__device__ __forceinline__ void recolour_R(T r0, T r1, T r2, T rt, const T nrm[6], const KT<T> &K, T out[4]) {
  const T irt = rcp(rt);
  T r3 = T(35) * r0 * r1 * r2 * irt * irt * irt;
  r3 = fmin(fmax(r3, T(0)), T(1));
  const T b0 = K.b0;
  const T b12 = b0 + b0 * r3 * K.gX[0];
  const T b13 = b0 + b0 * r3 * K.gX[1];
  const T b23 = b0 + b0 * r3 * K.gX[2];
  const T a12 = b12 * r0 * r1 * irt, a13 = b13 * r0 * r2 * irt, a23 = b23 * r1 * r2 * irt;
  out[0] = a12 * nrm[0] + a13 * nrm[2];
  out[1] = a12 * nrm[1] + a13 * nrm[3];
  out[2] = -a12 * nrm[0] + a23 * nrm[4];
  out[3] = -a12 * nrm[1] + a23 * nrm[5];
}

__device__ __forceinline__ const IbbNode *find_ibb(const IbbNode *ibb, const DomainDev &D, int64_t li) {
  int lo = D.ibb_off, hi = D.ibb_off + D.n_ibb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (ibb[mid].li < li) lo = mid + 1;
    else hi = mid;
  }
  return &ibb[lo];
}

// Recoloured populations f''_{dir,k} of Eq. (13) at a node (through the accessor): C_k (f'+w)
// + w R_k.e_dir.
template <typename T, class Acc>
__device__ __forceinline__ void fluid_parts_of(const Acc &acc, int dx, int dy, int dir, T fv, T out[3]) {
  const T w = wgt<T>(dir);
  const int ex = lat_ex(dir), ey = lat_ey(dir);
  if (dir == 0) {  // e = 0: no recolouring term
    out[0] = acc.C(0, dx, dy) * fv;
    out[1] = acc.C(1, dx, dy) * fv;
    out[2] = acc.C(2, dx, dy) * fv;
    return;
  }
  const T R1 = edot<T>(ex, ey, acc.R(0, dx, dy), acc.R(1, dx, dy));
  const T R2 = edot<T>(ex, ey, acc.R(2, dx, dy), acc.R(3, dx, dy));
  out[0] = acc.C(0, dx, dy) * fv + w * R1;
  out[1] = acc.C(1, dx, dy) * fv + w * R2;
  out[2] = acc.C(2, dx, dy) * fv + w * (-(R1 + R2));
}

// The same for the node's own post-collision population (shifted) in direction dir.
template <typename T, class Acc>
__device__ __forceinline__ void fluid_parts(const Acc &acc, int dx, int dy, int dir, T out[3]) {
  fluid_parts_of<T>(acc, dx, dy, dir, acc.f(dir, dx, dy) + wgt<T>(dir), out);
}

// Eq. (16) pull-streaming into a fluid node whose eight neighbours are fluid and whose links cross
// no x boundary with a rule of its own: the same sums as stream_node without its branches.  The
// partial densities end with + 0, which turns a sum of zeros of either sign into +0 (a fluid absent
// from the whole neighbourhood), so that stream_plain_bulk below gives the same bits.
template <typename T, class Acc>
__device__ __forceinline__ void stream_plain(const Acc &acc, T fo[9], T &ra, T &rb, T &rc) {
  ra = rb = rc = T(0);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    T c[3];
    fluid_parts<T>(acc, -ex, -ey, a, c);
    fo[a] = acc.f(a, -ex, -ey);
    ra += c[0]; rb += c[1]; rc += c[2];
  }
  ra = ra + T(0); rb = rb + T(0); rc = rc + T(0);
}

// stream_plain where every recolouring vector the node reads is zero (no pair normal in reach): each
// term C_k (f' + w) + w e.R_k is then C_k (f' + w) rounded the same way, so the sums match
// stream_plain bit for bit without reading R.
template <typename T, class Acc>
__device__ __forceinline__ void stream_plain_bulk(const Acc &acc, T fo[9], T &ra, T &rb, T &rc) {
  ra = rb = rc = T(0);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    fo[a] = acc.f(a, -ex, -ey);
    const T fv = fo[a] + wgt<T>(a);
    const T c0 = acc.C(0, -ex, -ey) * fv, c1 = acc.C(1, -ex, -ey) * fv, c2 = acc.C(2, -ex, -ey) * fv;
    ra += c0; rb += c1; rc += c2;
  }
  ra = ra + T(0); rb = rb + T(0); rc = rc + T(0);
}

// Eq. (16) pull-streaming into one fluid node (gx, gy) from the post-collision data around it,
// with halfway / interpolated bounce-back, the fluid-1/3 exchanging periodic x boundary and the
// Zou-He columns.  Produces the shifted total distribution and the three partial densities.  ib:
// the node's interpolated-bounce-back record (null without curved links).
template <typename T, class Acc>
__device__ __forceinline__ void stream_node(const Acc &acc, int gx, const DomainDev &D, const KT<T> &K,
                                            const IbbNode *ib, T fo[9], T &ra, T &rb, T &rc) {
  ra = rb = rc = T(0);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const int ex = lat_ex(a), ey = lat_ey(a);
    const int sx = gx - ex;
    if (D.bcx == BCX_ZOUHE && (sx < 0 || sx >= D.nx)) {  // set by the Zou-He rule below
      fo[a] = T(0);
      continue;
    }
    if (!acc.solid(-ex, -ey)) {
      T c[3];
      fluid_parts<T>(acc, -ex, -ey, a, c);
      fo[a] = acc.f(a, -ex, -ey);
      const bool crossed = D.bcx == BCX_SWAP13 && (sx < 0 || sx >= D.nx);
      if (crossed) { ra += c[2]; rb += c[1]; rc += c[0]; }
      else { ra += c[0]; rb += c[1]; rc += c[2]; }
    } else {
      // the link x -> x - e_a ends in a solid node: bounce-back of the populations leaving x
      // along -e_a (direction ab).  The interpolated bounce-back acts on the total; each fluid
      // takes its halfway-reflected recoloured population plus its share C_k(x) of the
      // interpolation's change of the total (Eq. 13 at x applied to the interpolated total).
      const int ab = lat_opp(a);
      const T qd = ib ? (T)ib->q[a - 1] : T(0.5);
      const T fab = acc.f(ab, 0, 0);
      T v;
      if (qd < T(0.5) && !acc.solid(ex, ey)) {
        const T c1 = T(2) * qd, c2 = T(1) - T(2) * qd;
        v = c1 * fab + c2 * acc.f(ab, ex, ey);
      } else if (qd < T(0.5)) {
        v = fab;
      } else {
        const T c1 = rcp(T(2) * qd), c2 = T(1) - c1;
        v = c1 * fab + c2 * acc.f(a, 0, 0);
      }
      fo[a] = v;
      // Eq. (13) at x with the reflected total v in place of f'_ab (at q = 1/2, v = f'_ab)
      T own_ab[3];
      fluid_parts_of<T>(acc, 0, 0, ab, v + wgt<T>(ab), own_ab);
      ra += own_ab[0];
      rb += own_ab[1];
      rc += own_ab[2];
    }
  }
  if (D.bcx == BCX_ZOUHE && (gx == 0 || gx == D.nx - 1)) {
    // Zou-He non-equilibrium bounce-back on the total distribution (unshifted).
    T ft[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) ft[a] = fo[a] + wgt<T>(a);
    if (gx == 0) {
      const T u = K.u_in;
      const T rw = (ft[0] + ft[2] + ft[4] + T(2) * (ft[3] + ft[6] + ft[7])) / (T(1) - u);
      ft[1] = ft[3] + T(2.0 / 3.0) * rw * u;
      ft[5] = ft[7] - T(0.5) * (ft[2] - ft[4]) + rw * u / T(6);
      ft[8] = ft[6] + T(0.5) * (ft[2] - ft[4]) + rw * u / T(6);
      rc += ft[1] + ft[5] + ft[8];  // incoming populations carry pure fluid 3
      fo[1] = ft[1] - wgt<T>(1);
      fo[5] = ft[5] - wgt<T>(5);
      fo[8] = ft[8] - wgt<T>(8);
    } else {
      const T ro = K.rho_out;
      const T ux = -T(1) + (ft[0] + ft[2] + ft[4] + T(2) * (ft[1] + ft[5] + ft[8])) / ro;
      ft[3] = ft[1] - T(2.0 / 3.0) * ro * ux;
      ft[7] = ft[5] + T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
      ft[6] = ft[8] - T(0.5) * (ft[2] - ft[4]) - ro * ux / T(6);
      // unknown populations carry the node's own composition
      const T C0 = acc.C(0, 0, 0), C1 = acc.C(1, 0, 0), C2 = acc.C(2, 0, 0);
      ra += C0 * ft[3]; rb += C1 * ft[3]; rc += C2 * ft[3];
      ra += C0 * ft[6]; rb += C1 * ft[6]; rc += C2 * ft[6];
      ra += C0 * ft[7]; rb += C1 * ft[7]; rc += C2 * ft[7];
      fo[3] = ft[3] - wgt<T>(3);
      fo[6] = ft[6] - wgt<T>(6);
      fo[7] = ft[7] - wgt<T>(7);
    }
  }
  ra = ra + T(0); rb = rb + T(0); rc = rc + T(0);  // +0 for a sum of zeros, as in stream_plain
}

}  // namespace lbm3
