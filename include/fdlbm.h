/*
 * fdlbm.h -- C ABI of the MI355X (gfx950) library for the FD-LBM D2Q9 time step and the
 * MRT D2Q9 stream-collide step of Dubois, Lallemand, Obrecht and Tekitek, "Lattice
 * Boltzmann model approximated with finite difference expressions" (Computers & Fluids
 * 155, 2017; arXiv 1803.00437).
 *
 * Conventions shared by every entry point
 *   - Grid nx * ny, node (x=i, y=j) at linear index j*nx + i (x fastest).  x is always
 *     periodic.  y is periodic (FDLBM_BC_PERIODIC) or closed by two walls parallel to Ox
 *     at y = -1/2 and y = ny - 1/2 (FDLBM_BC_WALLS_Y; the channel of section 3-c with the
 *     wall half-way between the last fluid node and the first node outside), or the grid
 *     holds a disk closed by a curved no-slip wall (FDLBM_BC_DISK, the Stokes-mode test of
 *     section 3-b; see fdlbm_params.disk_r).
 *   - The state is stored as deviations from the rest state rho = 1, J = 0, in the storage
 *     dtype with no padding, row-interleaved: with F fields, row y of field f starts at
 *     element (F*y + f)*nx, so node (x, y) of field f is element (F*y + f)*nx + x (the rows
 *     a step reads and writes together are adjacent in memory).  FD-LBM and LW-ACM: F = 3,
 *     fields drho = rho - 1, jx, jy.  MRT: F = 9, fields f_k - w_k in velocity order.  The
 *     host arrays of set_state, get_state, set_populations and get_populations are plain
 *     planes of nx*ny values (x fastest) in every case.
 *   - Velocity order of the populations (section 1): e_0 = (0,0), e_1..e_4 = (1,0), (0,1),
 *     (-1,0), (0,-1), e_5..e_8 = (1,1), (-1,1), (-1,-1), (1,-1).
 *   - Device buffers are owned by the caller (allocated e.g. by PyTorch) and must stay
 *     valid until fdlbm_destroy.  The library never allocates or frees device memory.
 *   - All work is issued on the HIP stream given at creation (NULL = the default stream).
 *     Steps return without synchronising; fdlbm_get_state, fdlbm_get_populations,
 *     fdlbm_diagnostics and fdlbm_mode_projection synchronise that stream.
 *   - A context is used by one host thread at a time.
 *   - Every function returns FDLBM_OK (0) or a negative code; no C++ exception crosses the
 *     ABI.  After FDLBM_EDEVICE, fdlbm_last_error() returns the HIP error text.
 */
#ifndef FDLBM_H
#define FDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDLBM_OK 0
#define FDLBM_EINVAL (-1)    /* invalid parameter, NULL pointer, or call on the wrong scheme */
#define FDLBM_ENOMEM (-2)    /* a caller buffer is smaller than fdlbm_workspace_bytes requires */
#define FDLBM_EDEVICE (-3)   /* a HIP runtime call failed */
#define FDLBM_EUNSTABLE (-4) /* the periodic check found a non-finite value in the state */

/* FD: the FD-LBM step of section 2.  MRT: the D2Q9 MRT step of section 1.  LWACM: the
 * link-wise artificial-compressibility step of section 1-b that FD-LBM starts from
 * (periodic grids, or the disk of FDLBM_BC_DISK; no body force; same stored state as
 * FD-LBM). */
enum { FDLBM_SCHEME_FD = 0, FDLBM_SCHEME_MRT = 1, FDLBM_SCHEME_LWACM = 2 };
enum { FDLBM_BC_PERIODIC = 0, FDLBM_BC_WALLS_Y = 1, FDLBM_BC_DISK = 2 };
/* Storage dtype of the state.  F64: FP64 storage and arithmetic.  F32: FP32 storage and
 * arithmetic.  F16DEV: FP16 storage of the deviations (drho, jx, jy), FP32 arithmetic
 * (FD-LBM and LW-ACM only), new values rounded to nearest.  F16DEV_SR: the same storage,
 * with each step's new values rounded stochastically (up or down to the neighbouring FP16
 * values with probabilities given by the distances, so increments smaller than half an FP16
 * unit are kept on average); the random bits come from a counter-based hash of the node and
 * the step count, so a run is reproducible and the sweep and reference kernels agree bit for
 * bit; single grids only.  Diagnostics are always reduced in FP64. */
enum { FDLBM_F64 = 0, FDLBM_F32 = 1, FDLBM_F16DEV = 2, FDLBM_F16DEV_SR = 3 };
/* Kernel selection.  AUTO picks the vectorised sweep kernels (FD-LBM: one fused pass per
 * step; MRT: lane groups with DPP column shifts).  REFERENCE: the plain kernels (FD-LBM:
 * post-collision planes then gather; MRT: one thread per node).  SWEEP: FD-LBM sweep
 * kernel, rejected if the grid width does not allow it. */
enum { FDLBM_KERNEL_AUTO = 0, FDLBM_KERNEL_REFERENCE = 1, FDLBM_KERNEL_SWEEP = 2 };

typedef struct fdlbm_params {
    int32_t nx, ny;     /* grid; FD-LBM: nx >= 8; walls: ny >= 4; periodic y: ny >= 8      */
    int32_t scheme;     /* FDLBM_SCHEME_FD, FDLBM_SCHEME_MRT or FDLBM_SCHEME_LWACM          */
    int32_t stencil;    /* FD-LBM finite differences of section 2: 3 or 5 points           */
    int32_t bc;         /* FDLBM_BC_PERIODIC, FDLBM_BC_WALLS_Y or FDLBM_BC_DISK             */
    int32_t dtype;      /* FDLBM_F64, FDLBM_F32, FDLBM_F16DEV, FDLBM_F16DEV_SR               */
    /* Relaxation rates, each in (0, 2).  Section 1-a: nu = (1/s_xx - 1/2)/3,
     * zeta = (1/s_e - 1/2)/3.  FD-LBM uses s_xx and s_e (its q and eps moments sit at
     * equilibrium, section 2); MRT uses all four.                                            */
    double s_xx, s_e, s_q, s_eps;
    int32_t quartic;    /* MRT: nonzero replaces s_q by the value that satisfies
                         * (1/s_xx - 1/2)(1/s_q - 1/2) = 1/6 (section 3-b)                   */
    double force_x, force_y; /* uniform body force per node and step, Strang-split (section 1) */
    int32_t kernel;     /* FDLBM_KERNEL_*                                                     */
    int32_t tile_rows;  /* sweep kernel: rows per wavefront, 2..1024 (0 or 1 = choose); tuning */
    int32_t check_every;/* > 0: fdlbm_step / mrt_step scan the state for non-finite values
                         * every check_every steps and return FDLBM_EUNSTABLE if one is found
                         * (this synchronises the stream at each check)                       */
    int32_t lane_cols;  /* sweep kernel: grid columns per lane, 0 (choose), 1 (3-point only),
                         * 2, or 4 (FP32 / FP16); any nx: where nx is not a multiple, a lane's
                         * columns are one element-aligned access (FP32, FP64) or one access
                         * each (FP16), with the same results; tuning knob                    */
    double wall_xi;     /* walls: their distance beyond the first and last fluid rows, in
                         * (0, 1]; 0 selects 1/2 (sections 3-b, 3-c: the channel
                         * [1 - xi, N + xi] of Fig. 6).  FD-LBM: ghost rows by linear
                         * extrapolation with zero velocity on the wall, the expression chosen
                         * by where the wall cuts the link.  MRT: interpolated bounce-back of
                         * Bouzidi et al. (halfway bounce-back at 1/2), in either MRT
                         * kernel.  Ignored without walls.                                   */
    /* FDLBM_BC_DISK: a disk of radius disk_r centred at
     * (disk_cx, disk_cy), in node units, inside the grid; section 3-b.  Fluid nodes lie at
     * distance r < disk_r from the centre.  Ghost nodes are the other nodes within Chebyshev
     * distance 3 of a fluid node; at r = disk_r + d on the ray of unit vector n, a ghost
     * takes the state at its mirror point centre + (disk_r - d) n, momentum negated and
     * density kept, by bilinear interpolation when the four nodes around that point are
     * fluid; otherwise the momentum of the sample at depth 3/2, scaled by -d / (3/2) (zero
     * velocity on the wall, linear across it), and that sample's density.  Every other node
     * is set to rest.  Each step first fills the ghost and rest nodes from the fluid, then
     * takes one periodic step of the whole grid (any kernel, dtype and stencil; force
     * allowed for FD-LBM).  The disk must lie in [2, nx - 3] x [2, ny - 3] (every fluid
     * node is then 3 nodes from the edges, so no periodic image enters a fluid update),
     * disk_r must exceed 3/2 (the sample at depth 3/2 then always has four fluid nodes) and
     * nx * ny must stay below 2^31.
     * MRT D2Q9 (FP64 or FP32, either kernel, force allowed): every non-fluid node is solid
     * and held at rest; after each periodic step of the whole grid, every population that
     * re-enters a fluid node x across a boundary link (x + e_k solid, the wall cutting the
     * link at x + q e_k) is the linear interpolated bounce-back of Bouzidi et al.:
     * 2q f*_k(x) + (1 - 2q) f*_k(x - e_k) for q < 1/2 (halfway bounce-back f*_k(x) if
     * x - e_k is solid), f*_k(x)/(2q) + (2q - 1)/(2q) f*_-k(x) for q >= 1/2.
     * Diagnostics sum over every node, ghost nodes included; give fdlbm_set_mode a J0 that
     * is zero outside the fluid to project on the fluid only.  Ignored for other bc.      */
    double disk_cx, disk_cy, disk_r;
} fdlbm_params;

typedef struct fdlbm_diag {
    double mass;       /* sum of drho over all nodes (total mass minus nx*ny)              */
    double mom_x;      /* sum of jx                                                         */
    double mom_y;      /* sum of jy                                                         */
    double kin_energy; /* 1/2 sum |J|^2 / rho                                               */
    double max_abs_j;  /* max |J|                                                           */
    double proj_num;   /* sum J . J0 (0 when no mode was set)                               */
    double proj_den;   /* sum J0 . J0                                                       */
    int64_t nonfinite; /* number of nodes with a NaN or Inf in drho, jx or jy              */
} fdlbm_diag;

typedef struct fdlbm_ctx fdlbm_ctx;

/* Sizes of the caller-owned device buffers for these parameters: each of the two state
 * buffers (ping-pong) needs *state_bytes, the scratch buffer *scratch_bytes.  Returns
 * FDLBM_EINVAL for parameters fdlbm_create would reject. */
int fdlbm_workspace_bytes(const fdlbm_params *p, size_t *state_bytes, size_t *scratch_bytes);

/* Validate p, bind the caller's device buffers (state_a, state_b: state_bytes each;
 * scratch: scratch_bytes; all 256-byte aligned) and the HIP stream (hipStream_t, may be
 * NULL), and return a context in *out.  The state is zero (rest) until set. */
int fdlbm_create(const fdlbm_params *p, void *state_a, void *state_b, void *scratch, size_t scratch_bytes,
                 void *hip_stream, fdlbm_ctx **out);

/* Upload a state from host FP64 arrays of nx*ny values each (drho = rho - 1, jx, jy),
 * converting to the storage dtype on the device.  MRT: the populations become
 * f^eq(rho, J) of section 1-a (the initial state of an MRT run).  Resets the step count. */
int fdlbm_set_state(fdlbm_ctx *c, const double *drho, const double *jx, const double *jy);

/* Download the current (drho, jx, jy) into host FP64 arrays.  MRT: the conserved moments
 * of the populations.  With a body force the physical momentum is J + F/2 (Strang). */
int fdlbm_get_state(fdlbm_ctx *c, double *drho, double *jx, double *jy);

/* MRT only: upload / download the nine population planes (f_k - w_k), host FP64,
 * 9*nx*ny values, plane k at offset k*nx*ny.  get/set round-trips exactly in FP64. */
int fdlbm_set_populations(fdlbm_ctx *c, const double *df);
int fdlbm_get_populations(fdlbm_ctx *c, double *df);

/* Advance the FD-LBM state by nsteps time steps (section 2): finite differences of the
 * stored (rho, J), theta terms, post-collision moments, f* = M^{-1} m*, propagation
 * (eq. 2), new (rho, J).  Asynchronous.  FDLBM_EINVAL if the context is MRT. */
int fdlbm_step(fdlbm_ctx *c, int64_t nsteps);

/* Advance the MRT populations by nsteps stream-collide steps (section 1, eqs. 1-2) with
 * halfway bounce-back on walls.  Asynchronous.  FDLBM_EINVAL if the context is FD-LBM. */
int mrt_step(fdlbm_ctx *c, int64_t nsteps);

/* Advance the LW-ACM state (drho, Jx, Jy) by nsteps steps of section 1-b:
 * f*_k(x) = f^eq_k(x) + Theta (f^eo_k(x + e_k) - f^eo_k(x)), Theta = 1 - 6 nu with
 * nu = (1/s_xx - 1/2)/3, f^eo the part of f^eq odd in the velocity, then propagation
 * (eq. 2).  Same kernels, layout, dtypes and tuning knobs as fdlbm_step (stencil, s_e and
 * the MRT rates are ignored).  Asynchronous.  FDLBM_EINVAL if the context is not LW-ACM. */
int lwacm_step(fdlbm_ctx *c, int64_t nsteps);

/* FP64 reduction over the current state (section 3-a diagnostics): totals, kinetic
 * energy, max |J|, non-finite count and, if a mode was set, sum J.J0.  Synchronises. */
int fdlbm_diagnostics(fdlbm_ctx *c, fdlbm_diag *out);

/* Allocation-free diagnostics, for callers that cannot allocate device memory or hand the
 * library a scratch buffer: work recorded under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It computes what fdlbm_diagnostics computes, with the
 * same kernels in the same order (the results are identical bit for bit), but
 *   - takes the state directly: `state` is a device buffer in the layout fdlbm_create's
 *     state buffers use for `p` (scheme, dtype, nx, ny; FD-LBM and LW-ACM: the
 *     row-interleaved drho, Jx, Jy fields; MRT: the nine row-interleaved populations), e.g. the
 *     buffer a context's current state is in (state_a after an even number of steps
 *     since fdlbm_create, else state_b);
 *   - j0x, j0y: optional device FP64 planes (nx*ny each, both or neither) for the sums
 *     <J, J0> and <J0, J0>; NULL leaves those two slots 0;
 *   - out: caller-owned device memory for 8 doubles, written in the order mass, mom_x,
 *     mom_y, kin_energy, max_abs_j, proj_num, proj_den, nonfinite (as a double);
 *   - is asynchronous on hip_stream (NULL = default stream): nothing is copied to the host
 *     and nothing synchronises, so the call can be recorded into a graph.
 * It calls no allocation routine.  The reduction's block partials live in a static device
 * array of 64 KiB (1024 blocks x 8 doubles) that each device holds from the first call until
 * the process ends; every block overwrites its own partial, so nothing needs clearing.  The
 * array's size does not depend on the grid: every p that fdlbm_workspace_bytes accepts fits,
 * and any other returns FDLBM_EINVAL (also for a NULL state or out, or one J0 plane alone).
 * All calls on one device share the array: calls that overlap on one device (concurrent
 * streams or host threads) race.  FDLBM_EDEVICE if a launch fails. */
int fdlbm_diagnostics_static(const fdlbm_params *p, const void *state, const double *j0x, const double *j0y,
                             void *hip_stream, double *out);

/* Store a reference velocity field J0 (host FP64, nx*ny each) in the scratch buffer for
 * the correlation A(t) = <J(t), J0> / <J0, J0> of section 3-a. */
int fdlbm_set_mode(fdlbm_ctx *c, const double *j0x, const double *j0y);

/* A(t) for the current state (FDLBM_EINVAL if no mode was set).  Synchronises. */
int fdlbm_mode_projection(fdlbm_ctx *c, double *out);

/* Number of steps taken since the last set_state / set_populations (or since the count was
 * set with fdlbm_set_step_count).  -1 for a NULL context. */
int64_t fdlbm_step_count(const fdlbm_ctx *c);

/* Set the step count (steps >= 0).  The count seeds the random bits of stochastic rounding
 * (FDLBM_F16DEV_SR): step n draws bits from a hash of n.  To continue a saved run bit for bit,
 * restore its state with fdlbm_set_state and then its count with this call; set_state
 * alone starts the count at 0 and so replays the bits of the run's first steps.  Other
 * dtypes ignore the count.  FDLBM_EINVAL for a NULL context or a negative count. */
int fdlbm_set_step_count(fdlbm_ctx *c, int64_t steps);

/* Tile-shape tuning (not part of the method; the results do not depend on the shape, only
 * the speed does).  Times `reps` launches (1..10000) of this context's step kernel for
 * each candidate shape on its own grid and keeps the fastest in the context: FD-LBM sweep
 * kernel: grid columns per lane (1, 2, 4 where supported) x rows per wavefront (4, 6, 8,
 * 12, 16, 24); MRT sweep kernel: rows per tile (1, 2, 4, 8, 16).  The reference kernels have
 * no shape and are only timed.  The state does not advance: each timed launch reads the
 * current state and writes the spare buffer, which the next step overwrites.  Synchronises
 * the stream.  The chosen shape goes to *out_lane_cols and *out_tile_rows (0 where the
 * kernel has no such parameter) and its time per step in ms to *out_ms; each may be NULL.
 * FDLBM_EINVAL for a NULL context or reps out of range, FDLBM_EDEVICE on a HIP error. */
int fdlbm_autotune(fdlbm_ctx *c, int32_t reps, int32_t *out_lane_cols, int32_t *out_tile_rows, double *out_ms);

/* Release the context.  Frees nothing the caller owns. */
void fdlbm_destroy(fdlbm_ctx *c);

/* Measurement utility: a plain streaming copy of `bytes` (a multiple of 16; both device
 * pointers 16-byte aligned) from src to dst, 16-byte accesses, issued asynchronously on
 * the HIP stream (NULL = default).  It gives the achievable HBM bandwidth that the step
 * kernels' algorithmic bandwidth is compared with, and a kernel of known traffic for
 * calibrating hardware byte counters.  Not part of the method. */
int fdlbm_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Static text for a return code, and the last HIP error text of this thread. */
const char *fdlbm_strerror(int code);
const char *fdlbm_last_error(void);

/* ---------------------------------------------------------------------------------- */
/* Batches: many independent periodic FD-LBM grids (3-point differences, no force) of   */
/* different sizes and rates, advanced together.  Each instance evolves exactly as the   */
/* same grid would in its own fdlbm_ctx (same bits).  Its correlation with its initial   */
/* state, A(t) = <J(t), J0> / <J0, J0> (section 3-a), is reduced on the device in FP64    */
/* every `sample_every` steps into a count x max_samples table.                           */
/* ---------------------------------------------------------------------------------- */
typedef struct fdlbm_instance {
    int32_t nx, ny;    /* >= 8 each                                                    */
    double s_xx, s_e;  /* rates in (0, 2)                                              */
} fdlbm_instance;

typedef struct fdlbm_batch fdlbm_batch;

/* Sizes of the two caller-owned state buffers (each) and of the scratch buffer. */
int fdlbm_batch_workspace_bytes(const fdlbm_instance *instances, int32_t count, int32_t dtype, int32_t max_samples,
                                size_t *state_bytes, size_t *scratch_bytes);

/* Lay out `count` instances (dtype FDLBM_F64 / F32 / F16DEV; not F16DEV_SR) in the caller's buffers
 * (256-byte aligned), upload the tile tables and bind the HIP stream.  All states are
 * zero until set.  A stream other than the default one is needed for graph replay. */
int fdlbm_batch_create(const fdlbm_instance *instances, int32_t count, int32_t dtype, int32_t max_samples,
                       void *state_a, void *state_b, void *scratch, size_t scratch_bytes, void *hip_stream,
                       fdlbm_batch **out);

/* Set / read instance i from host FP64 arrays (nx*ny each).  Setting a state also makes
 * its momentum the reference J0 of instance i and clears the sample table. */
int fdlbm_batch_set_state(fdlbm_batch *b, int32_t i, const double *drho, const double *jx, const double *jy);
int fdlbm_batch_get_state(fdlbm_batch *b, int32_t i, double *drho, double *jx, double *jy);

/* Advance every instance by nsteps (one launch per step for all instances).  With
 * sample_every > 0 (nsteps must be a multiple), A(t) of every instance is recorded after
 * each sample_every steps; with use_graph != 0 each chunk of sample_every steps plus its
 * sample is captured once in a HIP graph and replayed.  Asynchronous. */
int fdlbm_batch_step(fdlbm_batch *b, int64_t nsteps, int32_t sample_every, int32_t use_graph);

/* The same steps with one launch per instance per step (the comparison path). */
int fdlbm_batch_step_per_instance(fdlbm_batch *b, int64_t nsteps);

/* Tile-height tuning of the batched launch: times `reps` (1..10000) one-launch steps of
 * all instances for 4, 6, 8, 12 and 16 rows per wavefront, keeps the fastest (it is 8
 * until tuned) and drops the cached graph replays, which are captured again on the next
 * fdlbm_batch_step.  No step is taken (timed launches write the spare buffer).
 * Synchronises the stream.  *out_rows, *out_ms (may be NULL): the choice and its time
 * per step in ms.  FDLBM_EINVAL for a NULL batch or reps out of range. */
int fdlbm_batch_autotune(fdlbm_batch *b, int32_t reps, int32_t *out_rows, double *out_ms);

/* Number of recorded samples in *nsamples and, if out != NULL, the count x max_samples
 * table (row i: instance i; entries beyond *nsamples are undefined).  Synchronises. */
int fdlbm_batch_amplitudes(fdlbm_batch *b, double *out, int32_t *nsamples);

int64_t fdlbm_batch_step_count(const fdlbm_batch *b);
void fdlbm_batch_destroy(fdlbm_batch *b);
const char *fdlbm_batch_last_error(void);

/* The transport-coefficient map of section 1-a: s = 1 / (1/2 + 3 nu). */
double fdlbm_rate_from_viscosity(double nu);
/* The quartic rate of section 3-b: s_q with (1/s_xx - 1/2)(1/s_q - 1/2) = 1/6. */
double fdlbm_quartic_s_q(double s_xx);

#ifdef __cplusplus
}
#endif
#endif /* FDLBM_H */
