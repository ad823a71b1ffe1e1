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

#include "lbm3_device.h"
#include "lbm3_internal.h"
#include "lbm3_adjoint.h"
#include "lbm3_kernels.h"

#include <mutex>

namespace lbm3 {

// Wetting-fill kernel: four lanes per fill node, kFillNodes nodes of one domain per work-group
// (so the domain's constants load with the node records instead of after them).  The three
// filled C's go to the compact array fillC[3 * node] that the fused kernels read (so the solid
// slots of the state stay constant).
// blocks .. doms: the fields of A that the first two rounds of loads need, as scalar arguments,
// which the compiler preloads into registers at wave launch (A's copies are not read).
template <typename T>
__global__ __launch_bounds__(4 * kFillNodes) void wet_fill(const FillBlock *__restrict__ blocks,
                                                           const FillNode *__restrict__ fill,
                                                           const FillCand *__restrict__ cand,
                                                           const DomainDev *__restrict__ doms, FillArgs<T> A) {
  __shared__ uint32_t far[kFillNodes][kFarW];  // the nodes' far fluid masks (for lines leaving the near one)
  const FillBlock B = blocks[blockIdx.x];
  const DomainDev &D = doms[B.dom];
  const int e = threadIdx.x >> 2, line = threadIdx.x & 3;
  const bool active = e < B.count;
  const int idx = B.first + (active ? e : 0);
  const FillNode fn = fill[idx];
  // The far mask is loaded with the node and stored to LDS once the densities at D0 are in.
  constexpr int kFarPerLane = (kFarW + 3) / 4;
  uint32_t fr[kFarPerLane];
#pragma unroll
  for (int c = 0; c < kFarPerLane; ++c) {
    const int k = line + 4 * c;
    fr[c] = k < kFarW ? A.far[(size_t)idx * kFarW + k] : 0u;
  }
  auto stage = [&]() {
#pragma unroll
    for (int c = 0; c < kFarPerLane; ++c)
      if (line + 4 * c < kFarW) far[e][line + 4 * c] = fr[c];
    __syncthreads();
  };
  double c1, c2;
  fill_lanes<T>(fn, D, A.flags + D.base, A.rho + 3 * D.base, far[e], stage, line, active, c1, c2,
                cand + ((size_t)idx * 4 + line) * kFillCands);
  if (active && line == 0) {
    A.fillC[3 * idx] = (T)c1;
    A.fillC[3 * idx + 1] = (T)c2;
    A.fillC[3 * idx + 2] = (T)(1.0 - c1 - c2);
  }
}

// Work item of this work-group.  With remap, consecutive items go to the same XCD (gfx950
// dispatches work-group b to XCD b % 8), so neighbouring tiles share an L2 and their halo
// rows are fetched from HBM once; the grid is then a multiple of 8 with one item per group.
__device__ __forceinline__ int first_item(int remap) {
  if (!remap) return blockIdx.x;
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// The same with the groups per XCD (grid / 8) given by the launch, which the tile kernel takes as
// a scalar argument: preloaded into registers with the other leading arguments, so the first work
// item's address needs no load.
__device__ __forceinline__ int first_item(int remap, int per) {
  return remap ? (blockIdx.x & 7) * per + (blockIdx.x >> 3) : blockIdx.x;
}

// ------------------------------------------------------------------------------------------
// Tile kernel: one work-group per (domain, TX x TY tile); C on tile+3 rings, stress on tile+2
// (with the recolouring vectors of tile+1), collision on tile+1, all in LDS.  Also provides the field export (FIELDS = true).
// The stress (ring 2) is dead once the force is formed, so the post-collision populations reuse
// its LDS; the total density is kept on ring 2, where it is read.
template <typename T>
struct Smem {
  T *C0, *C1, *C2;       // ring 3: mass fractions
  T *RH;                 // ring 2: total density
  T *Txx, *Txy, *Tyy;    // ring 2: stress of Eq. (10) (phases B, C)
  T *PF;                 // ring 1, 9 planes: post-collision shifted distribution (phases C, D;
                         // same LDS as the stress)
  T *PR;                 // ring 1, 4 planes: R_1, R_2 of the recolouring
  uint8_t *FL;           // ring 3: flags
  int *any_stress;       // set in phase B when some pair normal of the tile + 2 rings is nonzero
  int *present_w;        // phase A, one per wave: bit k set when some C_k the wave formed is nonzero
};

template <typename T>
__host__ __device__ inline size_t smem_bytes(int TX, int TY) {
  const size_t n3 = (size_t)(TX + 6) * (TY + 6), n2 = (size_t)(TX + 4) * (TY + 4),
               n1 = (size_t)(TX + 2) * (TY + 2);
  const size_t shared = 3 * n2 > 9 * n1 ? 3 * n2 : 9 * n1;
  return (3 * n3 + n2 + shared + 4 * n1) * sizeof(T) + ((n3 + 15) & ~(size_t)15) + 48;
}

template <typename T, int W1, int W3, int N1>
struct TileAcc {
  const Smem<T> &L;
  int p1, p3;
  __device__ bool solid(int dx, int dy) const { return L.FL[p3 + dx + dy * W3] & FL_SOLID; }
  __device__ T f(int dir, int dx, int dy) const { return L.PF[dir * N1 + p1 + dx + dy * W1]; }
  // f for a rarely taken branch: the index is formed where it is used (an opaque copy of p1 keeps
  // the compiler from computing such indices for every link up front and holding them live)
  __device__ T f_rare(int dir, int dx, int dy) const {
    int p = p1;
    asm volatile("" : "+v"(p));
    return L.PF[dir * N1 + p + dx + dy * W1];
  }
  __device__ T R(int c, int dx, int dy) const { return L.PR[c * N1 + p1 + dx + dy * W1]; }
  __device__ T C(int k, int dx, int dy) const {
    const int q = p3 + dx + dy * W3;
    return k == 0 ? L.C0[q] : (k == 1 ? L.C1[q] : L.C2[q]);
  }
};

// Register budget (second launch bound: waves per SIMD): the FP32 kernels are held to 6 (80
// VGPRs: six 256-thread or three 512-thread work-groups per CU, which their LDS also allows), the
// FP16-storage ones to 5 except the 512-thread 64-wide tiles, which fit 80 VGPRs without spilling
// (0.552 -> 0.418 ms per 4000 x 4000 launch at 6 waves); the FP64 ones are limited by their LDS.
template <typename S, typename T, int OUT, int TX, int TY, int NT>
__global__ __launch_bounds__(NT, sizeof(T) == 8 ? 1 : (sizeof(S) == 2 ? ((TX == 64 && NT == 512) ? 6 : 5) : 6))
void step_fused(const WorkItem *__restrict__ work, const DomainDev *__restrict__ doms, int work_begin, int work_end,
                int remap, int per, StepArgs<S, T> A) {
  // (work .. per: the leading fields of A that locate the first work item, as scalar arguments,
  // which the compiler preloads into registers at wave launch; A's copies are not read)
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int W3 = TX + 6, H3 = TY + 6, N3 = W3 * H3;
  constexpr int W2 = TX + 4, H2 = TY + 4, N2 = W2 * H2;
  constexpr int W1 = TX + 2, H1 = TY + 2, N1 = W1 * H1;
  Smem<T> L;
  {
    T *p = reinterpret_cast<T *>(smem_raw);
    L.C0 = p; p += N3; L.C1 = p; p += N3; L.C2 = p; p += N3; L.RH = p; p += N2;
    L.Txx = p; L.Txy = p + N2; L.Tyy = p + 2 * N2;
    L.PF = p; p += (3 * N2 > 9 * N1 ? 3 * N2 : 9 * N1);
    L.PR = p; p += 4 * N1;
    L.FL = reinterpret_cast<uint8_t *>(p);
    L.any_stress = reinterpret_cast<int *>(L.FL + ((N3 + 15) & ~15));
    L.present_w = L.any_stress + 4;
  }
  constexpr bool FIELDS = OUT == OUT_FIELDS, ADJ = OUT == OUT_ADJ;
  // single-fluid tiles skip phase B in the streaming step; not in the 16-wide tiles, where the
  // test's registers cost a spill in the collision (and tiles of small, latency-bound domains
  // gain little from it)
  constexpr bool SKIP1 = !FIELDS && !ADJ && TX >= 32;
  const int tid = threadIdx.x;
  const T eps_g = A.eps_g;

  for (int wi = work_begin + first_item(remap, per); wi < work_end; wi += remap ? work_end : gridDim.x) {
    const WorkItem wk = work[wi];
    const DomainDev &D = doms[wk.dom];
    const int x0 = wk.x0, y0 = wk.y0;
    // (the state's offset, plane and pitch from the work item: the first loads need not wait for
    // the domain record)
    const int pitch = wk.pitch;
    const uint8_t *flags = A.flags + wk.base;
    const T *Rin = A.rin + 3 * wk.base;
    const S *Fin = A.fin + 9 * wk.base;
    const int64_t P = wk.plane;
    const KT<T> K = make_kt<T>(D);
    const bool inner = wk.kind & WK_INNER, plain = wk.kind & WK_PLAIN;

    // Phase A: C_k and rho on tile + 3 rings (with the wetting fill at the fill nodes).
    if (tid == 0) *L.any_stress = 0;
    int fluids = 0;  // bit k: some C_k this thread formed is nonzero
    for (int q = tid; q < N3; q += NT) {
      const int lx = q % W3, ly = q / W3;
      const int64_t li = inner ? plane_index(x0 - 3 + lx, y0 - 3 + ly, pitch)
                               : node_index(x0 - 3 + lx, y0 - 3 + ly, D);
      const uint8_t fl = *elem32(flags, li);
      T v[4];
      node_composition<T>(fl, *elem32(Rin, li), *elem32(Rin + P, li), *elem32(Rin + 2 * P, li), A.fillC, v);
      L.FL[q] = fl;
      L.C0[q] = v[0]; L.C1[q] = v[1]; L.C2[q] = v[2];
      if (SKIP1) fluids |= (v[0] != T(0) ? 1 : 0) | (v[1] != T(0) ? 2 : 0) | (v[2] != T(0) ? 4 : 0);
      if (lx >= 1 && lx <= W3 - 2 && ly >= 1 && ly <= H3 - 2) L.RH[(lx - 1) + (ly - 1) * W2] = v[3];
      if (ADJ) {  // C_k and rho at the tile's in-grid positions
        const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        if (lx >= 3 && ly >= 3 && gx < wk.x1 && gy < wk.y1 && gx >= 0 && gx < D.nx) {
          const int64_t a = adj_index(D, gx, gy);
#pragma unroll
          for (int c = 0; c < 4; ++c) A.adj_X[(AX_C + c) * A.adj_plane + a] = v[c];
        }
      }
    }
    if (SKIP1) {  // the fluids present in the wave's positions: one LDS word per wave (each wave
                  // writes its own every work item, so nothing needs clearing)
      const int wf = (__ballot(fluids & 1) ? 1 : 0) | (__ballot(fluids & 2) ? 2 : 0) | (__ballot(fluids & 4) ? 4 : 0);
      if ((tid & 63) == 0) L.present_w[tid >> 6] = wf;
    }
    __syncthreads();

    // Phase B: Eq. (12) gradients and the Eq. (10) stress on tile + 2 rings; recolouring vectors.
    // A plain tile whose tile + 3 rings hold a single fluid (every other C_k exactly zero) has
    // G_kl = C_l grad C_k - C_k grad C_l = 0 for every pair, so no pair passes |G| > eps: phase B
    // would leave the stress +0 and the normals zero, which the force loop and the plain streaming
    // of such a tile do not read (they are skipped below), so it is skipped as well.
    int fluids_here = 0;  // the fluids present in the tile + 3 rings (uniform: a scalar)
    if (SKIP1) {
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) fluids_here |= L.present_w[w];
      fluids_here = __builtin_amdgcn_readfirstlane(fluids_here);
    }
    const bool single_fluid = SKIP1 && plain && (fluids_here & (fluids_here - 1)) == 0;
    bool any_g = false;
    for (int q = single_fluid ? N2 : tid; q < N2; q += NT) {
      const int lx = q % W2, ly = q / W2;
      const int p3 = (lx + 1) + (ly + 1) * W3;
      const int off[9] = {0, 1, W3, -1, -W3, 1 + W3, -1 + W3, -1 - W3, 1 - W3};
      T g[3][2];
      const T *Cs[3] = {L.C0, L.C1, L.C2};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T c9[9];
#pragma unroll
        for (int a = 0; a < 9; ++a) c9[a] = Cs[k][p3 + off[a]];
        grad9(c9, g[k][0], g[k][1]);
      }
      const T cc[3] = {L.C0[p3], L.C1[p3], L.C2[p3]};
      T txx, txy, tyy, nrm[6];
      const bool node_g = pair_stress(cc, g, L.RH[q], K, eps_g, txx, txy, tyy, nrm);
      any_g |= node_g;
      L.Txx[q] = txx; L.Txy[q] = txy; L.Tyy[q] = tyy;
      // Eq. (13)-(15): the recolouring vectors of the fluid nodes of tile + 1 ring, from the
      // normals just formed (phase C needs only them, not the normals)
      if (!FIELDS && lx >= 1 && lx <= W2 - 2 && ly >= 1 && ly <= H2 - 2 && !(L.FL[p3] & FL_SOLID)) {
        if (!ADJ) {  // (the adjoint's tiles do not stream)
          const int p1 = (lx - 1) + (ly - 1) * W1;
          const T rt = L.RH[q];
          // with all normals zero the vectors are zeros (of either sign), which the streaming
          // sums treat exactly as +0: they are written as +0 without being formed
          T Rv[4] = {T(0), T(0), T(0), T(0)};
          if (node_g) recolour_R(cc[0] * rt, cc[1] * rt, cc[2] * rt, rt, nrm, K, Rv);
#pragma unroll
          for (int c = 0; c < 4; ++c) L.PR[c * N1 + p1] = Rv[c];
        }
        if (ADJ) {  // pair normals of the tile's fluid nodes
          const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
          if (lx >= 2 && ly >= 2 && gx < wk.x1 && gy < wk.y1 && gx >= 0 && gx < D.nx && gy >= 0 && gy < D.ny) {
            const int64_t a = adj_index(D, gx, gy);
#pragma unroll
            for (int c = 0; c < 6; ++c) A.adj_X[(AX_N + c) * A.adj_plane + a] = nrm[c];
          }
        }
      }
    }
    if (any_g) *L.any_stress = 1;
    __syncthreads();

    // Phase C: force (all ring-1 nodes first: the populations then overwrite the stress),
    // velocity and MRT collision on tile + 1 ring.
    constexpr int IC = (N1 + NT - 1) / NT;
    auto active_c = [&](int q) -> bool {
      if (q >= N1) return false;
      const int lx = q % W1, ly = q / W1;
      if (L.FL[(lx + 2) + (ly + 2) * W3] & FL_SOLID) return false;
      const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
      if ((FIELDS || ADJ) && !(lx >= 1 && lx <= TX && ly >= 1 && ly <= TY)) return false;
      // Zou-He ghost columns are never streaming sources; off-grid rows are flagged solid.
      if (D.bcx == BCX_ZOUHE && (gx < 0 || gx >= D.nx)) return false;
      if (FIELDS && (gx >= D.nx || gy >= D.ny)) return false;
      return true;
    };
    // Where no pair normal of the tile + 2 rings passed |G| > eps (the bulk of each fluid), every
    // stress there is +0 and so is its divergence: the force loop is skipped, with the same result.
    const bool any_stress = __builtin_amdgcn_readfirstlane(*L.any_stress) != 0;
    T Fxs[IC], Fys[IC];
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      const int q = tid + it * NT;
      Fxs[it] = Fys[it] = T(0);
      if (!any_stress || !active_c(q)) continue;
      const int lx = q % W1, ly = q / W1;
      const int p2 = (lx + 1) + (ly + 1) * W2;
      const int off2[9] = {0, 1, W2, -1, -W2, 1 + W2, -1 + W2, -1 - W2, 1 - W2};
      T xx[9], xy[9], yy[9];
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        xx[a] = L.Txx[p2 + off2[a]];
        xy[a] = L.Txy[p2 + off2[a]];
        yy[a] = L.Tyy[p2 + off2[a]];
      }
      div_stress(xx, xy, yy, Fxs[it], Fys[it]);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IC; ++it) {
      const int q = tid + it * NT;
      if (!active_c(q)) continue;
      const int lx = q % W1, ly = q / W1;
      const int p2 = (lx + 1) + (ly + 1) * W2;
      const int p3 = (lx + 2) + (ly + 2) * W3;
      const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
      T Fx = Fxs[it], Fy = Fys[it];
      const bool zh_out = D.bcx == BCX_ZOUHE && gx >= D.nx - 2;
      if (ADJ) {  // interfacial force of the tile's fluid nodes
        if (!(gx < wk.x1 && gy < wk.y1 && gy >= 0 && gy < D.ny)) continue;
        const int64_t a = adj_index(D, gx, gy);
        A.adj_X[AX_F * A.adj_plane + a] = Fx;
        A.adj_X[(AX_F + 1) * A.adj_plane + a] = Fy;
        // the collision below only where a Zou-He outlet node or a neighbour's interpolated
        // bounce-back reads its result
        if (!zh_out && !(L.FL[p3] & FL_IBBSRC)) continue;
      }
      T f[9];
      {
        const int64_t li = inner ? plane_index(gx, gy, pitch) : node_index(gx, gy, D);
#pragma unroll
        for (int a = 0; a < 9; ++a) f[a] = load_s<S, T>(elem32(Fin + a * P, li));
      }
      const T rt = L.RH[p2];
      const T r0 = L.C0[p3] * rt, r1 = L.C1[p3] * rt, r2 = L.C2[p3] * rt;
      T fd[9], ux, uy;
      collide_shifted(f, Fx, Fy, r0, r1, r2, K, fd, ux, uy);
      if (FIELDS) {
        const int64_t o = (int64_t)gy * D.nx + gx;
        const int64_t n = (int64_t)D.nx * D.ny;
        if (A.out_u) { A.out_u[o] = ux; A.out_u[n + o] = uy; }
        if (A.out_force) { A.out_force[o] = Fx; A.out_force[n + o] = Fy; }
        continue;
      }
      if (ADJ) {  // the post-collision populations that a Zou-He outlet node or an interpolated
                  // bounce-back reads (the adjoint's node kernel recomputes its own elsewhere)
        const int64_t a = adj_index(D, gx, gy);
#pragma unroll
        for (int c = 0; c < 9; ++c) A.adj_X[(AX_P + c) * A.adj_plane + a] = fd[c];
        continue;
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) L.PF[a * N1 + q] = fd[a];
    }
    if (ADJ) {
      __syncthreads();
      continue;
    }
    if (FIELDS) {
      // partial densities (or filled C) of the tile
      for (int q = tid; q < TX * TY; q += NT) {
        const int lx = q % TX, ly = q / TX;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= D.nx || gy >= D.ny) continue;
        const int64_t li = plane_index(gx, gy, pitch);
        const int64_t o = (int64_t)gy * D.nx + gx, n = (int64_t)D.nx * D.ny;
        const bool solid = flags[li] & FL_SOLID;
        const int p3 = (lx + 3) + (ly + 3) * W3;
        if (solid) {  // the filled C (zero at solid nodes that are not filled)
          A.out_rho[o] = L.C0[p3]; A.out_rho[n + o] = L.C1[p3]; A.out_rho[2 * n + o] = L.C2[p3];
        } else {
          for (int k = 0; k < 3; ++k) A.out_rho[k * n + o] = Rin[k * P + li];
        }
        if (solid) {
          if (A.out_u) { A.out_u[o] = 0; A.out_u[n + o] = 0; }
          if (A.out_force) { A.out_force[o] = 0; A.out_force[n + o] = 0; }
        }
      }
      __syncthreads();
      continue;
    }
    __syncthreads();

    // The interpolated-bounce-back records of the tile's curved nodes, mapped from their tile
    // positions in the LDS of the total density (dead after phase C).
    int *ibm = reinterpret_cast<int *>(L.RH);
    if (wk.ibb_count > 0) {
      for (int e = tid; e < wk.ibb_count; e += NT) {
        const TileIbb t = A.tibb[wk.ibb_begin + e];
        ibm[t.q] = t.idx;
      }
      __syncthreads();
    }

    // Phase D: pull-streaming into the tile, Eq. (16), with the boundary rules.
    T *Rout = A.rout + 3 * wk.base;
    S *Fout = A.fout + 9 * wk.base;
    for (int q = tid; q < TX * TY; q += NT) {
      const int lx = q % TX, ly = q / TX;
      const int gx = x0 + lx, gy = y0 + ly;
      if (gx >= D.nx || gy >= D.ny) continue;
      const int64_t li = plane_index(gx, gy, pitch);
      const int p1 = (lx + 1) + (ly + 1) * W1;
      const int p3 = (lx + 3) + (ly + 3) * W3;
      const uint8_t fl = L.FL[p3];
      if (fl & FL_SOLID) continue;  // solid slots keep their constant contents
      TileAcc<T, W1, W3, N1> acc{L, p1, p3};
      T fo[9], ra, rb, rc;
      if (plain) {
        // no pair normal in the tile + 2 rings: every recolouring vector streaming reads is zero
        if (any_stress) stream_plain<T>(acc, fo, ra, rb, rc);
        else stream_plain_bulk<T>(acc, fo, ra, rb, rc);
      } else {
        stream_node<T>(acc, gx, D, K, (fl & FL_CURVED) ? A.ibb + ibm[q] : nullptr, fo, ra, rb, rc);
      }
      // Non-temporal stores where a tile row covers whole 128-byte lines of a plane; narrower rows
      // share lines with the neighbouring tile, which the L2 then merges before writing back.
      if constexpr (TX * sizeof(S) >= 128) {
#pragma unroll
        for (int a = 0; a < 9; ++a) store_nt<S, T>(elem32(Fout + a * P, li), fo[a]);
      } else {
#pragma unroll
        for (int a = 0; a < 9; ++a) store_s<S, T>(elem32(Fout + a * P, li), fo[a]);
      }
      if constexpr (TX * sizeof(T) >= 128) {
        store_nt<T, T>(elem32(Rout, li), ra);
        store_nt<T, T>(elem32(Rout + P, li), rb);
        store_nt<T, T>(elem32(Rout + 2 * P, li), rc);
      } else {
        *elem32(Rout, li) = ra;
        *elem32(Rout + P, li) = rb;
        *elem32(Rout + 2 * P, li) = rc;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------
// Strip kernel: one work-group of NT threads owns a strip of NT-6 columns and marches up a
// segment of rows.  Thread c holds column x0-3+c.  Per row r it loads C_k of row r (ring of 6
// rows), forms the stress of row r-1 (ring of 3), collides row r-2 (ring of 3 rows of
// post-collision data) and streams row r-3 into HBM, so every row is read once and halos in y
// are reused from LDS; only the 6 halo columns of the strip are recomputed.
template <typename T>
__host__ __device__ inline size_t strip_smem_bytes(int nt) {
  return (size_t)nt * ((6 * 4 + 3 * 3 + 3 * 13) * sizeof(T) + 6);
}

template <typename T, int NT>
struct StripAcc {
  const T *Cr, *Pr;       // C ring [6][4][NT], post-collision ring [3][13][NT]
  const uint8_t *Fr;      // flag ring [6][NT]
  int c;                  // column
  int cs[3], ps[3];       // C / post-collision ring slots of rows y-1, y, y+1
  __device__ bool solid(int dx, int dy) const { return Fr[cs[dy + 1] * NT + c + dx] & FL_SOLID; }
  __device__ T f(int dir, int dx, int dy) const { return Pr[(ps[dy + 1] * 13 + dir) * NT + c + dx]; }
  __device__ T f_rare(int dir, int dx, int dy) const { return f(dir, dx, dy); }
  __device__ T R(int k, int dx, int dy) const { return Pr[(ps[dy + 1] * 13 + 9 + k) * NT + c + dx]; }
  __device__ T C(int k, int dx, int dy) const { return Cr[(cs[dy + 1] * 4 + k) * NT + c + dx]; }
};

__device__ __forceinline__ int mod_pos(int v, int m) {
  const int r = v % m;
  return r < 0 ? r + m : r;
}

template <typename S, typename T, int NT>
__global__ __launch_bounds__(NT) void step_strip(StepArgs<S, T> A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *Cr = reinterpret_cast<T *>(smem_raw);  // [6][4][NT]: C0, C1, C2, rho
  T *Tr = Cr + 6 * 4 * NT;                  // [3][3][NT]: Txx, Txy, Tyy
  T *Pr = Tr + 3 * 3 * NT;                  // [3][13][NT]: f'(9), R(4)
  uint8_t *Fr = reinterpret_cast<uint8_t *>(Pr + 3 * 13 * NT);  // [6][NT]
  const int c = threadIdx.x;
  const T eps_g = A.eps_g;

  for (int wi = A.work_begin + first_item(A.remap); wi < A.work_end; wi += A.remap ? A.work_end : gridDim.x) {
    const WorkItem wk = A.work[wi];
    const DomainDev &D = A.doms[wk.dom];
    const int x0 = wk.x0, x1 = wk.x1, y0 = wk.y0, y1 = wk.y1;
    const uint8_t *flags = A.flags + D.base;
    const T *Rin = A.rin + 3 * D.base;
    const S *Fin = A.fin + 9 * D.base;
    T *Rout = A.rout + 3 * D.base;
    S *Fout = A.fout + 9 * D.base;
    const int64_t P = D.plane;
    const KT<T> K = make_kt<T>(D);
    const int gx = x0 - 3 + c;
    const int gxm = D.bcx == BCX_ZOUHE ? min(max(gx, 0), D.nx - 1) : wrap_small(gx, D.nx);
    const int yend = min(y1, D.ny);

    for (int r = y0 - 3; r <= y1 + 2; ++r) {
      // Stage A: C_k and rho of row r.
      {
        const int gy = D.yper ? wrap_small(r, D.ny) : min(max(r, -2), D.ny + 1);
        const int64_t li = plane_index(gxm, gy, D.pitch);
        const uint8_t fl = flags[li];
        T v[4];
        node_composition<T>(fl, Rin[li], Rin[P + li], Rin[2 * P + li], A.fillC, v);
        const int sl = mod_pos(r, 6);
        T *cr = Cr + sl * 4 * NT;
        Fr[sl * NT + c] = fl;
        cr[c] = v[0]; cr[NT + c] = v[1]; cr[2 * NT + c] = v[2]; cr[3 * NT + c] = v[3];
      }
      __syncthreads();
      // Stage B: stress of row r-1.
      if (r - 1 >= y0 - 2 && c >= 1 && c < NT - 1) {
        const int sm = mod_pos(r - 2, 6), s0 = mod_pos(r - 1, 6), sp = mod_pos(r, 6);
        T g[3][2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const T *lo = Cr + (sm * 4 + k) * NT + c, *mi = Cr + (s0 * 4 + k) * NT + c, *hi = Cr + (sp * 4 + k) * NT + c;
          const T c9[9] = {mi[0], mi[1], hi[0], mi[-1], lo[0], hi[1], hi[-1], lo[-1], lo[1]};
          grad9(c9, g[k][0], g[k][1]);
        }
        const T *mi = Cr + s0 * 4 * NT + c;
        const T cc[3] = {mi[0], mi[NT], mi[2 * NT]};
        T txx, txy, tyy, nrm[6];
        pair_stress(cc, g, mi[3 * NT], K, eps_g, txx, txy, tyy, nrm);
        T *tr = Tr + mod_pos(r - 1, 3) * 3 * NT;
        tr[c] = txx; tr[NT + c] = txy; tr[2 * NT + c] = tyy;
      }
      __syncthreads();
      // Stage C: collision and recolouring vectors of row r-2.
      const int yc = r - 2;
      if (yc >= y0 - 1 && yc <= y1 && c >= 2 && c < NT - 2) {
        const int s0 = mod_pos(yc, 6);
        const uint8_t fl = Fr[s0 * NT + c];
        const bool ghost = D.bcx == BCX_ZOUHE && (gx < 0 || gx >= D.nx);
        if (!(fl & FL_SOLID) && !ghost) {
          const int tm = mod_pos(yc - 1, 3), t0 = mod_pos(yc, 3), tp = mod_pos(yc + 1, 3);
          T xx[9], xy[9], yy[9];
          const T *trs[3] = {Tr + tm * 3 * NT + c, Tr + t0 * 3 * NT + c, Tr + tp * 3 * NT + c};
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const T *lo = trs[0] + q * NT, *mi = trs[1] + q * NT, *hi = trs[2] + q * NT;
            const T v9[9] = {mi[0], mi[1], hi[0], mi[-1], lo[0], hi[1], hi[-1], lo[-1], lo[1]};
#pragma unroll
            for (int a = 0; a < 9; ++a) (q == 0 ? xx : (q == 1 ? xy : yy))[a] = v9[a];
          }
          T Fx, Fy;
          div_stress(xx, xy, yy, Fx, Fy);
          // normals of row yc (gradients again, from the C ring)
          const int cm = mod_pos(yc - 1, 6), cp = mod_pos(yc + 1, 6);
          T g[3][2];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const T *lo = Cr + (cm * 4 + k) * NT + c, *mi = Cr + (s0 * 4 + k) * NT + c, *hi = Cr + (cp * 4 + k) * NT + c;
            const T c9[9] = {mi[0], mi[1], hi[0], mi[-1], lo[0], hi[1], hi[-1], lo[-1], lo[1]};
            grad9(c9, g[k][0], g[k][1]);
          }
          const T *mi = Cr + s0 * 4 * NT + c;
          const T cc[3] = {mi[0], mi[NT], mi[2 * NT]};
          const T rt = mi[3 * NT];
          T txx, txy, tyy, nrm[6];
          pair_stress(cc, g, rt, K, eps_g, txx, txy, tyy, nrm);
          const int gy = D.yper ? wrap_small(yc, D.ny) : yc;
          const int64_t li = plane_index(gxm, gy, D.pitch);
          T f[9];
#pragma unroll
          for (int a = 0; a < 9; ++a) f[a] = load_s<S, T>(Fin + a * P + li);
          const T r0 = cc[0] * rt, r1 = cc[1] * rt, r2 = cc[2] * rt;
          T fd[9], ux, uy, Rv[4];
          collide_shifted(f, Fx, Fy, r0, r1, r2, K, fd, ux, uy);
          recolour_R(r0, r1, r2, rt, nrm, K, Rv);
          T *pr = Pr + mod_pos(yc, 3) * 13 * NT + c;
#pragma unroll
          for (int a = 0; a < 9; ++a) pr[a * NT] = fd[a];
#pragma unroll
          for (int q = 0; q < 4; ++q) pr[(9 + q) * NT] = Rv[q];
        }
      }
      __syncthreads();
      // Stage D: stream row r-3 into HBM.
      const int yd = r - 3;
      const int x = x0 + c - 3;
      if (yd >= y0 && yd < yend && c >= 3 && c < NT - 3 && x < x1) {
        const int64_t li = plane_index(x, yd, D.pitch);
        const int s0 = mod_pos(yd, 6);
        const uint8_t fl = Fr[s0 * NT + c];
        if (!(fl & FL_SOLID)) {
          StripAcc<T, NT> acc;
          acc.Cr = Cr; acc.Pr = Pr; acc.Fr = Fr; acc.c = c;
          acc.cs[0] = mod_pos(yd - 1, 6); acc.cs[1] = s0; acc.cs[2] = mod_pos(yd + 1, 6);
          acc.ps[0] = mod_pos(yd - 1, 3); acc.ps[1] = mod_pos(yd, 3); acc.ps[2] = mod_pos(yd + 1, 3);
          T fo[9], ra, rb, rc;
          const IbbNode *ib = ((fl & FL_CURVED) && D.n_ibb > 0) ? find_ibb(A.ibb, D, li) : nullptr;
          stream_node<T>(acc, x, D, K, ib, fo, ra, rb, rc);
#pragma unroll
          for (int a = 0; a < 9; ++a) store_nt<S, T>(Fout + a * P + li, fo[a]);
          store_nt<T, T>(Rout + li, ra);
          store_nt<T, T>(Rout + P + li, rb);
          store_nt<T, T>(Rout + 2 * P + li, rc);
        }
      }
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
  if (bad && A.bad) A.bad[0] = 1;
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
  if (a.n_fill <= 0 || a.n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(wet_fill<T>, dim3(a.n_blocks), dim3(4 * kFillNodes), 0, s, a.blocks, a.fill, a.cand, a.doms, a);
  return hipGetLastError();
}

// Tile shapes compiled into the tile kernel (LDS neighbour offsets become immediates): 256-thread
// work-groups (MODE_TILE) and 512-thread work-groups (MODE_TILE512, fewer halo nodes per tile
// node and half the loop trips per phase).
#define LBM3_TILE_SHAPES(X) X(32, 8, 256) X(16, 16, 256) X(64, 4, 256) X(64, 8, 256) \
  X(16, 16, 512) X(32, 16, 512) X(64, 8, 512)

bool tile_supported(int mode, int tx, int ty) {
  const int nt = mode == MODE_TILE512 ? 512 : 256;
#define LBM3_TS(a, b, c) if (tx == a && ty == b && nt == c) return true;
  LBM3_TILE_SHAPES(LBM3_TS)
#undef LBM3_TS
  return false;
}

template <typename S, typename T>
hipError_t launch_step(const StepArgs<S, T> &a, int grid, int mode, int out, hipStream_t s) {
  if (out == OUT_ADJ) {  // the adjoint's tiles: 32 x 8, 256 threads
    if (a.tile_x != 32 || a.tile_y != 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL((step_fused<S, T, OUT_ADJ, 32, 8, 256>), dim3(grid), dim3(256), smem_bytes<T>(32, 8), s, a.work,
                       a.doms, a.work_begin, a.work_end, a.remap, grid >> 3, a);
    return hipGetLastError();
  }
  const bool fields = out == OUT_FIELDS;
  if (fields || mode == MODE_TILE || mode == MODE_TILE512) {
    const size_t sm = smem_bytes<T>(a.tile_x, a.tile_y);
    const int nt = (!fields && mode == MODE_TILE512) ? 512 : 256;
#define LBM3_TL(X, Y, N)                                                                           \
    if (a.tile_x == X && a.tile_y == Y && nt == N) {                                               \
      if (fields) hipLaunchKernelGGL((step_fused<S, T, OUT_FIELDS, X, Y, N>), dim3(grid), dim3(N), sm, s, a.work, a.doms,     \
                                     a.work_begin, a.work_end, a.remap, grid >> 3, a);                              \
      else hipLaunchKernelGGL((step_fused<S, T, OUT_STEP, X, Y, N>), dim3(grid), dim3(N), sm, s, a.work, a.doms, a.work_begin, \
                              a.work_end, a.remap, grid >> 3, a);                                                   \
      return hipGetLastError();                                                                    \
    }
    LBM3_TILE_SHAPES(LBM3_TL)
#undef LBM3_TL
    return hipErrorInvalidValue;
  } else if (mode == MODE_STRIP128) {
    hipLaunchKernelGGL((step_strip<S, T, 128>), dim3(grid), dim3(128), strip_smem_bytes<T>(128), s, a);
  } else {
    hipLaunchKernelGGL((step_strip<S, T, 256>), dim3(grid), dim3(256), strip_smem_bytes<T>(256), s, a);
  }
  return hipGetLastError();
}

// Allows every fused-kernel instantiation the full 160 KiB of LDS of a gfx950 work-group.
hipError_t init_kernel_attributes() {
  const int lim = 160 * 1024;
  hipError_t e = hipSuccess, r;
#define LBM3_ATTR1(S, T, F, X, Y, N)                                                        \
  r = hipFuncSetAttribute((const void *)step_fused<S, T, F, X, Y, N>,                         \
                          hipFuncAttributeMaxDynamicSharedMemorySize, lim);                   \
  if (r != hipSuccess) e = r;
#define LBM3_ATTRT(X, Y, N)                                                                   \
  LBM3_ATTR1(double, double, OUT_STEP, X, Y, N) LBM3_ATTR1(double, double, OUT_FIELDS, X, Y, N) \
  LBM3_ATTR1(float, float, OUT_STEP, X, Y, N) LBM3_ATTR1(float, float, OUT_FIELDS, X, Y, N)     \
  LBM3_ATTR1(__half, float, OUT_STEP, X, Y, N) LBM3_ATTR1(__half, float, OUT_FIELDS, X, Y, N)
  LBM3_TILE_SHAPES(LBM3_ATTRT)
#undef LBM3_ATTRT
  LBM3_ATTR1(double, double, OUT_ADJ, 32, 8, 256)
  LBM3_ATTR1(float, float, OUT_ADJ, 32, 8, 256)
#undef LBM3_ATTR1
#define LBM3_ATTR2(S, T, N)                                                                   \
  r = hipFuncSetAttribute((const void *)step_strip<S, T, N>,                                  \
                          hipFuncAttributeMaxDynamicSharedMemorySize, lim);                   \
  if (r != hipSuccess) e = r;
  LBM3_ATTR2(double, double, 128)
  LBM3_ATTR2(double, double, 256)
  LBM3_ATTR2(float, float, 128)
  LBM3_ATTR2(float, float, 256)
  LBM3_ATTR2(__half, float, 128)
  LBM3_ATTR2(__half, float, 256)
#undef LBM3_ATTR2
  return e;
}

template <typename T>
hipError_t launch_mass(const MassArgs<T> &a, int n_chunks, int n_dom, double *out, hipStream_t s) {
  hipLaunchKernelGGL(mass_partial<T>, dim3(n_chunks), dim3(kThreads), 0, s, a);
  hipLaunchKernelGGL(mass_final, dim3((3 * n_dom + 63) / 64), dim3(64), 0, s, a.partial, a.chunk_first, n_dom, out);
  return hipGetLastError();
}

// Partial sums of the mass reduction for lbm3_mass_device, the entry point that allocates
// nothing: a fixed array of the library, one copy per GPU (at its own address there), shared by
// every call on that GPU and kept until the process ends.  Host code reaches it only through the
// device address hipGetSymbolAddress gives with that GPU current.
static __device__ __align__(256) double scratch[3 * kMassScratchChunks];

hipError_t mass_scratch_init(int device, double **out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double *ptr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[device] = static_cast<double *>(p);
  }
  *out = ptr[device];
  return hipSuccess;
}

size_t step_smem_bytes(int precision, int mode, int tx, int ty) {
  if (mode == MODE_TILE || mode == MODE_TILE512)
    return precision == 0 ? smem_bytes<double>(tx, ty) : smem_bytes<float>(tx, ty);
  const int nt = mode == MODE_STRIP128 ? 128 : 256;
  return precision == 0 ? strip_smem_bytes<double>(nt) : strip_smem_bytes<float>(nt);
}

template hipError_t launch_step<double, double>(const StepArgs<double, double> &, int, int, int, hipStream_t);
template hipError_t launch_step<float, float>(const StepArgs<float, float> &, int, int, int, hipStream_t);
template hipError_t launch_step<__half, float>(const StepArgs<__half, float> &, int, int, int, hipStream_t);
template hipError_t launch_fill<double>(const FillArgs<double> &, hipStream_t);
template hipError_t launch_fill<float>(const FillArgs<float> &, hipStream_t);
template hipError_t launch_mass<double>(const MassArgs<double> &, int, int, double *, hipStream_t);
template hipError_t launch_mass<float>(const MassArgs<float> &, int, int, double *, hipStream_t);

}  // namespace lbm3
