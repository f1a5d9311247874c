/*
 * fdlbm3d.h -- C ABI of the FD-LBM step on the three-dimensional D3Q19 lattice, part of the
 * MI355X (gfx950) library libfdlbm.so (the two-dimensional steps are in fdlbm.h).
 *
 * The Conclusion of Dubois, Lallemand, Obrecht and Tekitek (arXiv 1803.00437) reports that
 * the analysis of section 2 was also carried out for D3Q19, without printing it.  This step
 * applies section 2's construction to D3Q19: the stored state is (rho, J); the six
 * second-order moments of the polynomial D3Q19 basis (energy e, 3p_xx, p_ww, p_xy, p_yz,
 * p_xz) take their equilibrium plus (1 - 1/s) times the defect of conservation theta
 * (eq. theta, at rho close to 1, from 3-point differences of the stored fields), every other
 * moment its equilibrium; f* = M^{-1} m* propagates (eq. 2) and the new (rho, J) is kept.
 * Transport coefficients: shear viscosity nu = (1/s_nu - 1/2)/3, bulk viscosity
 * (2/9)(1/s_e - 1/2), sound speed 1/sqrt(3); in a mean flow V the shear and bulk viscosities
 * carry the factor (1 - 3V^2) that section 2 states for D2Q9.
 *
 * Conventions
 *   - Periodic grid nx * ny * nz, node (x=i, y=j, z=k) at linear index (k*ny + j)*nx + i.
 *   - The state is four planes of nx*ny*nz values in the storage dtype, in the order
 *     drho = rho - 1, Jx, Jy, Jz, with no padding.
 *   - Error codes, the caller-owned device buffers, the stream and the threading rules are
 *     those of fdlbm.h.  After FDLBM_EDEVICE, fdlbm3d_last_error() returns the HIP error
 *     text.
 */
#ifndef FDLBM3D_H
#define FDLBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "fdlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdlbm3d_params {
    int32_t nx, ny, nz;  /* periodic grid, each 3 .. 2^20, nx*ny*nz < 2^40, one x-y plane below
                            2^31 bytes (nx*ny < 2^29 in FP32, 2^28 in FP64)                       */
    int32_t dtype;       /* FDLBM_F64 or FDLBM_F32: storage and arithmetic                        */
    double s_nu, s_e;    /* relaxation rates in (0, 2): shear (five traceless moments), energy    */
    int32_t kernel;      /* FDLBM_KERNEL_AUTO or _SWEEP: the fused sweep kernel; _REFERENCE: the
                            post-collision planes then a gather (needs the larger scratch)        */
    int32_t tile_rows;   /* sweep: wavefronts per block along y, 8, 12 or 16 (0 = 12), two of which
                            hold halo rows                                                        */
    int32_t tile_planes; /* sweep: planes per block along z, 1 .. 4096 (0 = 64 in FP32, 32 in FP64) */
} fdlbm3d_params;

typedef struct fdlbm3d_diag {
    double mass;       /* sum of drho                                                     */
    double mom_x, mom_y, mom_z;
    double kin_energy; /* 1/2 sum |J|^2 / rho                                             */
    double max_abs_j;
    int64_t nonfinite; /* nodes with a NaN or Inf in any field                            */
} fdlbm3d_diag;

typedef struct fdlbm3d_ctx fdlbm3d_ctx;

/* Sizes of the caller-owned device buffers: each of the two state buffers needs
 * *state_bytes, the scratch buffer *scratch_bytes (FP64 staging of the host arrays, the
 * diagnostics and, for the reference kernels, 18 post-collision planes).  FDLBM_EINVAL for
 * parameters fdlbm3d_create would reject. */
int fdlbm3d_workspace_bytes(const fdlbm3d_params *p, size_t *state_bytes, size_t *scratch_bytes);

/* Validate p, bind the device buffers (256-byte aligned; ownership stays with the caller,
 * who keeps them valid until fdlbm3d_destroy) and the HIP stream (NULL = default stream). */
int fdlbm3d_create(const fdlbm3d_params *p, void *state_a, void *state_b, void *scratch, size_t scratch_bytes,
                   void *hip_stream, fdlbm3d_ctx **out);

/* Upload / download the state as four host FP64 arrays of nx*ny*nz values (drho, Jx, Jy,
 * Jz); conversion to the storage dtype happens on the device.  set_state resets the step
 * count; both synchronise the stream. */
int fdlbm3d_set_state(fdlbm3d_ctx *c, const double *drho, const double *jx, const double *jy, const double *jz);
int fdlbm3d_get_state(fdlbm3d_ctx *c, double *drho, double *jx, double *jy, double *jz);

/* Advance the state by nsteps steps (asynchronous): 3-point differences of the stored
 * fields, defects theta, post-collision moments, f* = M^{-1} m*, propagation (eq. 2),
 * new (rho, J). */
int fdlbm3d_step(fdlbm3d_ctx *c, int64_t nsteps);

/* FP64 reduction over the current state.  Synchronises the stream. */
int fdlbm3d_diagnostics(fdlbm3d_ctx *c, fdlbm3d_diag *out);

/* Time every sweep tile shape (rows per block 8, 12, 16 x planes per block 16, 32, 64, 128)
 * on this grid, reps steps each after one warm-up, and keep the fastest for later steps.  The
 * timed steps read the current state and write the spare buffer, so the state does not
 * advance; all shapes give the same bits.  The reference kernels have no shape (their time is
 * reported).  Chosen rows, planes and ms per step go to the out pointers (each may be NULL).
 * Synchronises the stream.  FDLBM_EINVAL for a NULL context or reps outside 1..10000. */
int fdlbm3d_autotune(fdlbm3d_ctx *c, int32_t reps, int32_t *out_rows, int32_t *out_planes, double *out_ms);

int64_t fdlbm3d_step_count(const fdlbm3d_ctx *c);
void fdlbm3d_destroy(fdlbm3d_ctx *c);
const char *fdlbm3d_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDLBM3D_H */
