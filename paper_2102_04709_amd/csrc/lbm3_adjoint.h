// lbm3_adjoint.h -- argument block and launcher of the adjoint step (internal to liblbm3).
//
// The adjoint works on an extended grid per domain: columns -1..nx (the two outer columns are
// the zero-gradient ghost columns of a Zou-He x boundary) and rows -2..ny+1 (the off-grid solid
// rows of a non-periodic y boundary); element (i, j) of a domain's extended plane is
// abase + (i + 1) + (nx + 2) (j + 2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm3_internal.h"

namespace lbm3 {

// Planes of the adjoint scratch (each of total_aplane elements of type T).  The forward
// intermediates (AX_*) are written by the tile kernel in its OUT_ADJ mode.
enum {
  AX_C = 0,      // 4: C_k, rho of the forward state (every in-grid position)
  AX_N = 4,      // 6: pair normals (fluid nodes)
  AX_F = 10,     // 2: interfacial force (fluid nodes)
  AX_P = 12,     // 9: post-collision shifted f (fluid nodes of the two columns next to a Zou-He
                 //    outlet, whose node reads its neighbours', and nodes flagged FL_IBBSRC, whose
                 //    neighbour's interpolated bounce-back reads them; elsewhere recomputed)
  AL_F = 21,     // 2: adjoint of F (fluid nodes)
  AL_N = 23,     // 6: adjoint of n (fluid nodes)
  AL_C = 29,     // 4: adjoint of C_k and rho
  A_PLANES = 33
};

template <typename S, typename T>
struct AdjArgs {
  const DomainDev *doms;
  const WorkItem *work;  // tiles of 32 x 8 over each domain's extended range
  int n_work;
  const uint8_t *flags;
  const IbbNode *ibb;
  const uint32_t *far;    // [kFarW * n_fill] far fluid masks of the fill nodes
  const int32_t *ibb_of;  // per node of the state planes (D.base + plane index): its IbbNode index
  // per fluid node of the state planes: bit d = the node read at x + e_d is solid, bit 9 + d = it
  // has curved links, bit 18 + d = the node read at x + 2 e_d is solid, bit 27 = x has curved links
  const uint32_t *links;
  const FillNode *fill;
  int n_fill;
  const T *fillC;
  const S *fin;     // forward state at t: distributions
  const T *rin;     //                      densities
  T *X;             // adjoint scratch, A_PLANES planes
  int64_t aplane;   // elements per scratch plane (sum over domains)
  const T *lin;     // adjoint of the state at t+1 (copy), 12 planes in the state layout
  T *lout;          // adjoint of the state at t, 12 planes in the state layout
  double *raw;      // [9 n_dom] raw parameter partials
  T eps_g;
  T eps_n;          // |G| below which the adjoint treats a pair normal as constant
};

// The transposes of one step, in order (the forward intermediates must be in the scratch).
// tplane = elements of one state plane summed over the domains (the offset of the density
// planes in the state layout, over 9).
template <typename S, typename T>
hipError_t launch_adjoint(const AdjArgs<S, T> &a, int64_t tplane, hipStream_t s);

// Writes dL/drho_k from g (flat [3][ny][nx] per domain) into the density planes of lam at fluid
// nodes; work = 32 x 8 tiles over the real nodes.
template <typename T>
hipError_t launch_adjoint_seed(const DomainDev *doms, const WorkItem *work, int n_work, const uint8_t *flags,
                               const double *g, T *lam, int64_t tplane, hipStream_t s);

// Phase-field mismatch loss of the state (rho: its density planes) against target (flat
// [3][ny][nx] FP64 per domain): writes dL/drho_k into the density planes of lam at fluid nodes,
// one loss partial per tile into part[n_work], and the per-domain losses into loss[n_dom]
// (tiles first[d] .. first[d+1]-1 belong to domain d); work = 32 x 8 tiles over the real nodes.
template <typename T>
hipError_t launch_loss_seed(const DomainDev *doms, const WorkItem *work, int n_work, const int *first, int n_dom,
                            const uint8_t *flags, const T *rho, int64_t tplane, const double *target, T *lam,
                            double *part, double *loss, hipStream_t s);

}  // namespace lbm3
