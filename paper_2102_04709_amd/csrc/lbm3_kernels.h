// lbm3_kernels.h -- argument blocks and launchers of the gfx950 kernels (internal to liblbm3).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lbm3_internal.h"

namespace lbm3 {

template <typename T>
struct FillArgs {
  const FillNode *fill;
  int n_fill;
  const FillBlock *blocks;  // the work-groups' fill ranges
  int n_blocks;
  const uint32_t *far;      // [kFarW * n_fill] far fluid masks of the fill nodes
  const FillCand *cand;     // [n_fill][4 lines][kFillCands] crossings of the pure-composition angles
  const DomainDev *doms;
  const uint8_t *flags;
  const T *rho;  // density planes of the current state
  T *fillC;      // [3 * n_fill] filled C of this step
};

template <typename S, typename T>
struct StepArgs {
  const DomainDev *doms;
  const WorkItem *work;
  int work_begin, work_end;
  const uint8_t *flags;
  const IbbNode *ibb;
  const T *fillC;  // [3 * n_fill] filled C of this step, indexed from the fill nodes' first slot
  // tile step only: the interpolated-bounce-back nodes of each tile (work[w].ibb_begin .. + ibb_count)
  const TileIbb *tibb;
  int remap;  // 1: XCD-aware mapping, one work item per work-group
  const S *fin;
  const T *rin;
  S *fout;
  T *rout;
  int tile_x, tile_y;
  T eps_g;
  // fields mode only: [comp][ny][nx] outputs of one domain
  T *out_rho, *out_u, *out_force;
  // adjoint-intermediates mode only: the scratch planes of the adjoint (extended grid) and their
  // size in elements
  T *adj_X;
  int64_t adj_plane;
};

// What the tile kernel produces: the next state, the fields of the current state, or the
// forward intermediates of the current state that the adjoint step reads.
enum { OUT_STEP = 0, OUT_FIELDS = 1, OUT_ADJ = 2 };

template <typename T>
struct MassArgs {
  const DomainDev *doms;
  const uint8_t *flags;
  const T *rho;
  const int *chunk_dom;    // [n_chunks]
  const int *chunk_first;  // [n_dom + 1]
  double *partial;         // [3 * n_chunks]
  int *bad;                // set to 1 on a non-finite density (may be null)
};

// Chunks (16 rows of one domain each) the fixed scratch of lbm3_mass_device holds: 3 doubles
// each, 1.5 MiB per GPU.
constexpr int kMassScratchChunks = 65536;
// Device address of that scratch on `device`, which must be the current device on the first call
// for it (the address is looked up once per device and kept).
hipError_t mass_scratch_init(int device, double **out);

enum { MODE_TILE = 0, MODE_STRIP128 = 1, MODE_STRIP256 = 2, MODE_TILE512 = 3 };
inline bool is_tile_mode(int mode) { return mode == MODE_TILE || mode == MODE_TILE512; }

template <typename T>
hipError_t launch_fill(const FillArgs<T> &a, hipStream_t s);
template <typename S, typename T>
hipError_t launch_step(const StepArgs<S, T> &a, int grid, int mode, int out, hipStream_t s);
template <typename T>
hipError_t launch_mass(const MassArgs<T> &a, int n_chunks, int n_dom, double *out, hipStream_t s);
size_t step_smem_bytes(int precision, int mode, int tx, int ty);
bool tile_supported(int mode, int tx, int ty);
hipError_t init_kernel_attributes();

}  // namespace lbm3
