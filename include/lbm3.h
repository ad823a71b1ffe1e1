/* lbm3.h -- C ABI of the MI355X (gfx950) library for the three-phase colour-gradient D2Q9
 * lattice update of Li, Lu, Jiang & Liu, "Lattice Boltzmann simulation of three-phase flows
 * with moving contact lines on curved surfaces" (arXiv:2102.04709).
 *
 * One time step (Sec. II of the paper) is: partial densities and mass fractions C_k (Eq. 16,
 * C_k = rho_k / rho), the characteristic-line wetting fill of C at solid boundary nodes
 * (Sec. II B, Eq. 19-22), colour gradients (Eq. 12), the interfacial force (Eq. 10), velocity
 * (Eq. 11), MRT collision with forcing (Eq. 1-9) at the mixture relaxation time (Eq. 7),
 * recolouring (Eq. 13-15) and streaming (Eq. 16) with halfway bounce-back, interpolated
 * bounce-back on exact circles, the fluid-1/fluid-3 exchanging periodic boundary (Sec. III C)
 * or a Zou-He velocity inlet and pressure outlet (Sec. III D).
 *
 * Conventions for every call:
 *  - Every call returns an lbm3_status; nothing aborts and no exception crosses the ABI.
 *    lbm3_last_error() gives the message of the last failure on a context.
 *  - Parameters are validated on the host before any device work.
 *  - Host inputs are copied during the call.  Device memory passed in (workspace, state and
 *    field buffers) belongs to the caller and must outlive the context.
 *  - All device work is enqueued on the stream given at creation; only lbm3_mass,
 *    lbm3_kernel_times and lbm3_autotune synchronise that stream.
 *  - A context is not thread-safe; separate contexts on separate streams are independent.
 *  - Lattice node (i, j) sits at (x, y) = (i, j); host arrays are [ny][nx] with x fastest.
 *  - Fluids 1, 2, 3 are the paper's red, green and blue.
 */
#ifndef LBM3_H
#define LBM3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3_ctx lbm3_ctx; /* opaque; created by lbm3_create, freed by lbm3_destroy */

typedef enum {
  LBM3_OK = 0,
  LBM3_EINVAL = 1,      /* invalid argument or inconsistent physical parameters */
  LBM3_ENOMEM = 2,      /* workspace too small or host allocation failed */
  LBM3_EHIP = 3,        /* a HIP runtime call failed */
  LBM3_ESTATE = 4,      /* call not valid in the context's current state */
  LBM3_ENUMERIC = 5,    /* a NaN or Inf was found in the densities */
  LBM3_EUNSUPPORTED = 6 /* combination of options not supported */
} lbm3_status;

/* Arithmetic and storage of the distributions (the densities rho_k are stored in the compute
 * type).  The distributions are stored as the shift f_a - w_a (rho^0 = 1). */
typedef enum {
  LBM3_F64 = 0,          /* FP64 compute and storage */
  LBM3_F32 = 1,          /* FP32 compute and storage */
  LBM3_F32_STORE_F16 = 2 /* FP32 compute, FP16 storage of the shifted distributions */
} lbm3_precision;

/* Boundary in x. */
typedef enum {
  LBM3_X_PERIODIC = 0,        /* periodic */
  LBM3_X_PERIODIC_SWAP13 = 1, /* periodic; populations crossing x exchange fluids 1 and 3
                                 (Sec. III C modified periodic condition) */
  LBM3_X_ZOUHE = 2            /* Zou-He velocity inlet (u_in, 0) at x = 0 carrying pure
                                 fluid 3, pressure outlet rho_out at x = nx-1 carrying the
                                 node's own composition (Sec. III D); needs y_periodic = 1 and
                                 no solid within 3 columns of either end */
} lbm3_bc_x;

/* One domain.  Equal densities rho_k^0 = 1 (Sec. II A), so the dynamic viscosity of each pure
 * fluid equals its kinematic viscosity nu_k. */
typedef struct {
  int32_t nx, ny;        /* lattice nodes, >= 3 each; (nx rounded up to 64) x (ny + 4) below
                            2^30 (LBM3_F32, LBM3_F32_STORE_F16) or 2^29 (LBM3_F64) */
  int32_t y_periodic;    /* 1: periodic in y; 0: every node outside 0 <= y < ny is solid
                            (flat walls are solid rows inside the mask) */
  int32_t bc_x;          /* lbm3_bc_x */
  double u_in, rho_out;  /* Zou-He inlet velocity and outlet density (bc_x = LBM3_X_ZOUHE) */
  double nu[3];          /* viscosities; tau = 1/2 + 3 nu must lie in (0.5, 10] (Eq. 7) */
  double sigma[3];       /* sigma12, sigma13, sigma23, each > 0 (Eq. 10, Eq. 15) */
  double theta_deg[2];   /* theta13, theta23 in (0, 180) degrees, measured inside fluids 1
                            and 2; theta12 follows from Eq. (18) and must satisfy
                            |cos theta12| <= 1 */
  double body_force[2];  /* uniform acceleration added as rho*g to the interfacial force
                            (test hook; 0 for the paper's cases) */
  int32_t n_circles;     /* number of exact solid circles (for interpolated bounce-back) */
  int32_t reserved;      /* must be 0 */
  const double *circles; /* host [3*n_circles] (cx, cy, R); NULL if n_circles = 0.  A solid
                            link whose solid node lies in a circle uses Bouzidi interpolated
                            bounce-back with the exact wall distance; other solid links use
                            halfway bounce-back.  Not allowed with LBM3_X_PERIODIC_SWAP13. */
  const uint8_t *solid;  /* host [ny*nx], 1 = solid; copied */
  const double *rho_init;/* host [3][ny*nx] initial partial densities (velocity 0); copied */
} lbm3_domain;

typedef struct {
  int32_t precision;         /* lbm3_precision */
  int32_t graph_block_steps; /* > 0: lbm3_step replays a captured hipGraph of this many steps
                                (rounded up to even); 0: plain launches */
  double beta0;              /* reference segregation parameter of Eq. (14); <= 0 selects the
                                paper's 0.7 */
  int32_t kernel;            /* fused-step kernel: 0 = tiles (tile_x x tile_y nodes per
                                256-thread work-group), 1 = row strips of 122 columns (128
                                threads), 2 = row strips of 250 columns (256 threads), 3 = tiles
                                with 512-thread work-groups; -1 = let lbm3_autotune choose
                                (tiles until it runs) */
  int32_t tile_x, tile_y;    /* tiles: the tile shape (0 = default, the first listed; 256
                                threads: 32x8, 16x16, 64x4, 64x8; 512 threads: 64x8, 16x16,
                                32x16); strips: tile_y = rows per segment (0 = default), tile_x
                                unused */
  int32_t persistent_blocks; /* > 0: the fused kernel runs this many work-groups that loop over
                                the (domain, tile) work list; 0: one work-group per work item */
  int32_t adjoint;           /* 1: also lay out the scratch of the adjoint step (lbm3_adjoint_*,
                                lbm3_loss_seed); LBM3_F64 and LBM3_F32 only; 0: forward only */
  const char *tune_cache;    /* path of the autotuner's JSON cache (NULL = none): lbm3_autotune
                                takes a configuration stored there for the same device
                                architecture, precision and domain shapes without timing, and
                                stores what it times; copied at creation */
} lbm3_options;

/* Bytes of device workspace lbm3_create needs for n domains (d[0..n-1]) and these options: the
 * state of Sec. II A in its compact form (total distributions and partial densities, Eq. 13 and
 * 16), twice, and the boundary tables of Sec. II B.  Host only; LBM3_EINVAL with
 * lbm3_plan_error() on an invalid description (the checks of lbm3_create). */
lbm3_status lbm3_workspace_bytes(const lbm3_domain *d, int32_t n, const lbm3_options *o,
                                 size_t *bytes);

/* Validates the domains (Eq. 18, tensions, viscosities, masks -- every fill node must have a
 * solid normal and its normal line must reach a fluid node), builds the boundary tables
 * (Eq. 19-20 normals, link fractions), lays out and initialises the state in the caller's
 * device workspace (256-byte aligned, at least lbm3_workspace_bytes long), and returns a
 * context.  hip_stream is a hipStream_t (NULL = the null stream).  Synchronises the stream
 * once at the end.  n = 1 is a single domain; n > 1 advances all domains together. */
lbm3_status lbm3_create(const lbm3_domain *d, int32_t n, const lbm3_options *o,
                        void *dev_workspace, size_t bytes, void *hip_stream, lbm3_ctx **out);

/* Advances every domain by nsteps time steps of Sec. II: the wetting fill (Eq. 19-22), colour
 * gradients and interfacial force (Eq. 10-12), MRT collision with forcing (Eq. 1-9, 11),
 * recolouring (Eq. 13-15) and streaming with the boundary rules (Eq. 16, Sec. III).
 * Asynchronous on the context's stream; with graph_block_steps > 0, whole blocks of steps are
 * replayed from a captured hipGraph.  LBM3_EINVAL for nsteps < 0; LBM3_EHIP if a launch fails. */
lbm3_status lbm3_step(lbm3_ctx *c, int32_t nsteps);

/* Writes fields of the current state of domain `domain` into caller device buffers of element
 * type dtype (LBM3_F64 -> double for FP64 contexts, LBM3_F32 -> float otherwise), layout
 * [comp][ny][nx]:
 *   dev_rho [3]: partial densities at fluid nodes; at the solid boundary nodes the mass
 *                fractions C_k of the wetting fill (Eq. 21-22) of this state, 0 at other solid
 *                nodes;
 *   dev_u   [2]: velocity of Eq. (11) including the interfacial force (0 at solid nodes); may
 *                be NULL;
 *   dev_force [2]: interfacial force of Eq. (10) plus the body force; may be NULL.
 * Asynchronous. */
lbm3_status lbm3_fields(lbm3_ctx *c, int32_t domain, void *dev_rho, void *dev_u,
                        void *dev_force, int32_t dtype);

/* Per-fluid mass sum_x rho_k over fluid nodes (rho_k = sum_a f_{a,k}, Eq. 16; conserved by
 * recolouring, Eq. 13, and by the closed boundaries), in FP64 and a fixed summation order, for
 * every domain: host_out[3*n].  Synchronises.  Returns LBM3_ENUMERIC if a NaN/Inf was found. */
lbm3_status lbm3_mass(lbm3_ctx *c, double *host_out);

/* For callers that cannot allocate device memory or synchronise (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the masses of lbm3_mass, bit for bit, written
 * asynchronously into the caller's device buffer dev_out[3*n] (FP64), allocating nothing.  The
 * reduction's partial sums live in a fixed device array of the library, 3 * 65536 doubles
 * (1.5 MiB) per GPU, held until the process ends; a context with more than 65536 chunks of 16
 * rows (the sum over its domains of ceil(ny / 16)) gets LBM3_EINVAL.  Every call on one GPU, from
 * any context or stream, shares that array: calls that overlap in time on one GPU race, so
 * serialise them (e.g. one stream).  A NaN/Inf density shows as a non-finite sum (there is no
 * LBM3_ENUMERIC here).  No memset is enqueued, so the call can be captured into a hipGraph. */
lbm3_status lbm3_mass_device(lbm3_ctx *c, double *dev_out);

/* Checkpointing of the whole state (all domains; the compact state of Eq. 13 and 16): a
 * device-to-device copy of the raw state planes, lbm3_state_bytes long, into / from a caller
 * buffer.  set_state(get_state(s)) continues bit-identically.  Asynchronous. */
lbm3_status lbm3_state_bytes(const lbm3_ctx *c, size_t *bytes);
lbm3_status lbm3_get_state(lbm3_ctx *c, void *dev_dst);
lbm3_status lbm3_set_state(lbm3_ctx *c, const void *dev_src);

/* Changes the wetting (Sec. II B) and tension (Eq. 10) parameters of domain `domain` (theta_deg[2] = theta13,
 * theta23 in degrees; sigma[3] = sigma12, sigma13, sigma23) with the checks of lbm3_create:
 * Eq. (18) fixes theta12 and Eq. (15) the factors g(X_kl).  The state is kept.  Synchronises. */
lbm3_status lbm3_set_params(lbm3_ctx *c, int32_t domain, const double *theta_deg, const double *sigma);

/* ---- Adjoint (reverse-mode derivative) of the time step --------------------------------------
 * For a loss L of the partial densities after T steps, the adjoint state lambda_t = dL/ds_t
 * (s_t = the state at step t: shifted distributions and partial densities at fluid nodes) obeys
 * lambda_t = (ds_{t+1}/ds_t)^T lambda_{t+1}; the parameter gradient sums
 * (ds_{t+1}/dp)^T lambda_{t+1} over the steps.  The derivative is that of the discrete update
 * as implemented (Eq. 1-22; at the non-smooth points -- the max/min of Eq. 22, clamps, the
 * |G| threshold of the normals -- the branch the forward took).  Needs a context created with
 * options.adjoint = 1.  lambda buffers are device buffers of lbm3_state_bytes in the state
 * layout and compute type; entries at solid nodes are zero, and lbm3_adjoint_step leaves the
 * layout's padding (plane columns beyond nx, off-grid rows of a periodic y axis) unwritten.
 *
 * lbm3_adjoint_seed starts a backward pass: clears the parameter-gradient accumulators and
 * writes lambda_T = dL/drho_k into dev_lambda (distribution part zero).  dev_grad_rho: device,
 * FP64, the domains' [3][ny][nx] arrays concatenated in domain order; values at solid nodes are
 * ignored.  Asynchronous. */
lbm3_status lbm3_adjoint_seed(lbm3_ctx *c, const double *dev_grad_rho, void *dev_lambda);

/* Starts a backward pass for the phase-field mismatch loss of the inverse problem (the loss of
 * the differentiation form; the mass fractions C_k = rho_k / rho of Eq. 16):
 *   L_d = sum over the fluid nodes of domain d of sum_k (C_k - C*_k)^2
 * of the context's current state.  Clears the parameter-gradient accumulators, writes
 * lambda_T = dL/ds_T into dev_adj (a device buffer of lbm3_state_bytes in the state layout:
 * dL/drho_k = (2/rho) [(C_k - C*_k) - sum_l C_l (C_l - C*_l)] at fluid nodes, zero elsewhere and in
 * the distribution part) and the losses into dev_loss[n] (device, FP64, summed in a fixed order).
 * dev_target_C: device, FP64, the domains' [3][ny][nx] target fractions concatenated in domain
 * order (values at solid nodes ignored).  Needs options.adjoint = 1.  Asynchronous. */
lbm3_status lbm3_loss_seed(lbm3_ctx *c, const double *dev_target_C, void *dev_adj, double *dev_loss);

/* One step back: from the forward state s_t (dev_state, as written by lbm3_get_state) and
 * lambda_{t+1} (dev_lambda_in) writes lambda_t (dev_lambda_out, a different buffer) and adds
 * step t's parameter partials to the accumulators.  Leaves the context's own state alone.
 * Asynchronous. */
lbm3_status lbm3_adjoint_step(lbm3_ctx *c, const void *dev_state, const void *dev_lambda_in,
                              void *dev_lambda_out);

/* The accumulated gradient dL/dp per domain: host_grad[5*n] = (theta13 [per degree], theta23
 * [per degree], sigma12, sigma13, sigma23), the chain rule through theta12 (Eq. 18) and g(X_kl)
 * (Eq. 15) included.  Synchronises. */
lbm3_status lbm3_adjoint_grad(lbm3_ctx *c, double *host_grad);

/* Average device time (ms) of one launch of the wetting-fill kernel (Eq. 19-22) and of the fused
 * step kernel (Eq. 1-16):
 * HIP events on the context's stream around nsteps back-to-back fills of the current state and
 * then nsteps back-to-back fused launches that all compute the same next step into the spare
 * buffer.  The state does not advance.  Synchronises. */
lbm3_status lbm3_kernel_times(lbm3_ctx *c, int32_t nsteps, double *ms_fill, double *ms_step);

/* Times the candidate configurations of the fused kernel (tile shapes, strip widths and
 * segment lengths) on the live state and keeps the fastest; returns (kernel, tile_x, tile_y)
 * in choice[3].  Every candidate computes the same result bit for bit (the step of Sec. II);
 * each candidate's two warm-up steps advance the state.  With options.tune_cache, a stored
 * choice for this device, precision and set of domain shapes is taken without timing (the state
 * does not advance), and a timed choice is stored (LBM3_EINVAL if the file cannot be written).
 * Synchronises. */
lbm3_status lbm3_autotune(lbm3_ctx *c, int32_t steps_per_candidate, int32_t *choice);

/* Information about the step of Sec. II: key 0 = algorithmic bytes per lattice update of the
 * fused kernel (state read
 * once and written once), 1 = total nodes, 2 = fill nodes, 3 = interpolated-bounce-back nodes,
 * 4 = tile_x, 5 = tile_y, 6 = work items, 7 = steps taken, 8 = kernel (0/3 tiles of 256/512
 * threads, 1/2 strips), 9 = hipGraph replays so far, 10 = steps per replayed graph (0: none). */
lbm3_status lbm3_query(const lbm3_ctx *c, int32_t key, double *value);

/* Status text: the message of the last failure on a context (never NULL; the string lives until
 * the next call on that context). */
const char *lbm3_last_error(const lbm3_ctx *c);
/* Message of the last failed lbm3_workspace_bytes or lbm3_create on the calling thread (those
 * calls have no context to attach it to). */
const char *lbm3_plan_error(void);
/* Short text of an lbm3_status code (static storage). */
const char *lbm3_status_string(int32_t code);

/* Frees host bookkeeping, graphs and events; never frees the caller's workspace. */
void lbm3_destroy(lbm3_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* LBM3_H */
