// Host-side declarations shared between the C ABI (abi.cpp) and the kernel translation
// units.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/fdlbm.h"

namespace fdlbm {

// Bytes of one stored value for a dtype.
inline size_t dtype_bytes(int dtype) { return dtype == FDLBM_F64 ? 8 : dtype == FDLBM_F32 ? 4 : 2; }
// Bytes of one arithmetic value (FP16 storage computes in FP32).
inline size_t compute_bytes(int dtype) { return dtype == FDLBM_F64 ? 8 : 4; }
// FP16 deviations, rounded to nearest or stochastically (the same layout)
inline bool is_f16(int dtype) { return dtype == FDLBM_F16DEV || dtype == FDLBM_F16DEV_SR; }

// Geometry and coefficients of one FD-LBM step, as the kernels need them.
// FD-LBM step arguments; the LW-ACM step (section 1-b) runs on the same kernels with
// stencil = LWACM_STENCIL (no differences, periodic, no force).
constexpr int LWACM_STENCIL = 1;
struct FdArgs {
    int nx, ny, stencil, walls, dtype;
    double s_xx, s_e, fx, fy;
    double xi;  // walls: their distance beyond the first and last rows (0 < xi <= 1)
    uint32_t seed = 0;  // FDLBM_F16DEV_SR: pcg_hash of the step count (random bits of the rounding)
};

struct MrtArgs {
    int nx, ny, walls, dtype;
    double s_e, s_xx, s_q, s_eps, fx, fy;
    int kernel, tile_rows;  // FDLBM_KERNEL_REFERENCE: one thread per node; else the vector sweep
    double xi;              // walls: distance beyond the first and last rows (interpolated bounce-back)
};

// FD-LBM, reference path: pass 1 writes the nine f* planes (compute dtype) for every
// node that sends a population into the fluid (ny + 2 rows with walls), pass 2 gathers.
hipError_t launch_fd_reference(const FdArgs &a, const void *src, void *dst, void *fstar, hipStream_t s);
size_t fd_reference_scratch_bytes(const FdArgs &a);

// FD-LBM, fused sweep path: one kernel per step, no scratch.  tile_rows: rows per
// wavefront (0 or 1 = default for the dtype and stencil); lane_cols: columns per lane
// (0 = default; 1 for 3-point differences only, 2, or 4 for FP32/FP16 only).
hipError_t launch_fd_sweep(const FdArgs &a, int tile_rows, int lane_cols, const void *src, void *dst, hipStream_t s);
bool fd_sweep_supported(const FdArgs &a, int lane_cols);

// Batch of independent periodic FD-LBM grids (3-point differences) -------------------
constexpr int BATCH_CHUNK = 65536;  // nodes per block of the A(t) reduction
struct BatchInstance {
    size_t offset;       // element offset of the instance's state (row-interleaved) in the state buffers
    size_t mode_offset;  // element offset of its J0 planes (jx, jy) in the mode buffer
    int nx, ny, strips_x, nbands;
    int cls;             // lane class of its tiles (BATCH_CLASSES)
    int first_chunk, nchunks;
    double ke, kxx;      // (1 - 1/s_e) / 2 and (1 - 1/s_xx) / 2 (3-point scale folded in)
};
struct BatchBlock {
    int instance, tile;
};
struct BatchChunk {
    int instance, chunk;
};
// Lane classes of the batched step, one launch each; W = 4 columns per lane (FP32, FP16)
// or 2 (FP64):
//   0: W columns as one vector access (nx a multiple of W)
//   1: 2 columns as one vector access (FP16, nx even)
//   2: W columns, any nx: element-aligned vector accesses (FP32, FP64) or one access per
//      column (FP16)
// The block table holds the tiles of class 0, 1, 2 in that order; class c starts at
// class_begin[c] and has class_blocks[c] entries.
constexpr int BATCH_CLASSES = 3;
inline int batch_class_cpl(int cls, int dtype) { return cls == 1 ? 2 : dtype == FDLBM_F64 ? 2 : 4; }
struct BatchLaunch {
    int dtype, count, rows, nblocks, nchunks, max_samples;
    int class_begin[BATCH_CLASSES], class_blocks[BATCH_CLASSES];
    const BatchInstance *inst;
    const BatchBlock *blocks;
    const BatchChunk *chunks;
    const void *mode;
    double *partials;
    int *counter;
    double *amps;
};
int batch_strip_stride(int cpl);  // columns stored per strip at `cpl` columns per lane
int batch_rows_per_block(int rows);
hipError_t launch_batch_step(const BatchLaunch &L, const void *src, void *dst, hipStream_t s);
hipError_t launch_batch_single(const BatchLaunch &L, int i, int cls, int nblocks, const void *src, void *dst,
                               hipStream_t s);
hipError_t launch_batch_sample(const BatchLaunch &L, const void *state, hipStream_t s);

// Curved no-slip wall around a disk (section 3-b) ----------------------------------------
// Ghost nodes, filled from the fluid before each periodic step: per ghost its linear index,
// the linear index of the lower-left node of its interpolation cell, and (wx, wy, sj): the
// bilinear weights of the right and upper neighbours and the factor on the momentum.  Per
// row j, the nodes [span[2j], span[2j+1]] are fluid or ghost; the others are set to rest.
// ring: the rest nodes within the step's reach (3) of a fluid or ghost node, periodic images
// included: without a body force the only rest nodes a step can move.
struct DiskTable {
    std::vector<int32_t> dst, src, span, ring;
    std::vector<double> w;  // 3 per ghost
    size_t nfluid = 0;
    // MRT D2Q9 (interpolated bounce-back on the circle): per boundary link its fluid node,
    // k | back << 4 (k: direction 1..8 toward the solid node; back: the node behind, x -
    // e_k, is fluid) and the wall cut q in (0, 1]; the solid nodes the links reach (their
    // streamed values are cleared after each step); per row j the fluid columns
    // [fspan[2j], fspan[2j+1]] (empty when the first exceeds the second).
    std::vector<int32_t> link_node, link_kb, solid_ring, fspan;
    std::vector<double> link_q;
};
// Builds the table; false if the disk does not fit the grid (the fluid must stay 3 nodes
// from every edge), holds no fluid node, or a ghost finds no fluid interpolation cell.
bool build_disk_table(int nx, int ny, double cx, double cy, double r, DiskTable *out);
struct DiskFill {
    int nx, ny, nghost, nring;
    const int32_t *dst, *src, *span, *ring;
    const double *w;
};
// full: set every rest node to rest (first step after the state was set, or a body force
// acts); otherwise the ring only
hipError_t launch_disk_fill(const DiskFill &f, int dtype, void *state, bool full, hipStream_t s);
// MRT in the disk: after the periodic step of the whole grid (populations `pop`, in place),
// the interpolated bounce-back of every boundary link, then the solid nodes set to rest
// (full: every non-fluid node; otherwise the solid ring the links reach).  Two launches.
struct MrtDisk {
    int nx, ny, nlinks, nring;
    const int32_t *node, *kb, *ring, *fspan;
    const double *q;
};
hipError_t launch_mrt_disk(const MrtDisk &d, int dtype, void *pop, bool full, hipStream_t s);

// MRT D2Q9 stream-collide (push) step.
hipError_t launch_mrt(const MrtArgs &a, const void *src, void *dst, hipStream_t s);

// Conversions between host-staged FP64 planes and device storage: element by element (the
// D3Q19 state, the batch modes), and row by row between nf FP64 planes and the
// row-interleaved storage of the two-dimensional states (row_elem).
hipError_t launch_pack(int dtype, const double *in, void *out, size_t count, hipStream_t s);
hipError_t launch_unpack(int dtype, const void *in, double *out, size_t count, hipStream_t s);
// nf (3 or 9) host-order FP64 planes of nx*ny values to and from the row-interleaved storage
hipError_t launch_pack_rows(int dtype, int nf, const double *in, void *out, int nx, int ny, hipStream_t s);
hipError_t launch_unpack_rows(int dtype, int nf, const void *in, double *out, int nx, int ny, hipStream_t s);
// MRT: populations f^eq(rho, J) from FP64 (drho, jx, jy) planes, and the conserved moments back.
hipError_t launch_mrt_init(int dtype, const double *dr, const double *jx, const double *jy, void *pop, int nx, int ny,
                           hipStream_t s);
hipError_t launch_mrt_moments(int dtype, const void *pop, double *dr, double *jx, double *jy, int nx, int ny,
                              hipStream_t s);

// Streaming device-to-device copy (bytes a multiple of 16, 16-byte aligned pointers).
hipError_t launch_device_copy(void *dst, const void *src, size_t bytes, hipStream_t s);

// FP64 diagnostics: totals, kinetic energy, max |J|, non-finite count and sum J.J0.
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_SLOTS = 8;  // doubles per block partial
hipError_t launch_diag(int scheme, int dtype, const void *state, int nx, int ny, const double *j0x, const double *j0y,
                       double *partials, double *out, hipStream_t s);
// The same reduction with its partials in a file-scope device array (no scratch argument);
// out: DIAG_SLOTS doubles of device memory.  Calls that overlap on one device race.
hipError_t launch_diag_static(int scheme, int dtype, const void *state, int nx, int ny, const double *j0x,
                              const double *j0y, double *out, hipStream_t s);

// ---- FD-LBM on the D3Q19 lattice (fd3d.hip) -------------------------------------------
struct Dim3Grid {
    int x, y, z;
};
// reference path: 18 post-collision planes in fstar (18 * nx*ny*nz elements), then gather
hipError_t launch_d3_reference(int dtype, const void *in, void *out, void *fstar, int nx, int ny, int nz, double s_nu,
                               double s_e, hipStream_t s);
// sweep path: wy wavefronts (8, 12 or 16) per block along y, tz planes per block along z
Dim3Grid d3_sweep_grid(int nx, int ny, int nz, int wy, int tz);
hipError_t launch_d3_sweep(int dtype, const void *in, void *out, int nx, int ny, int nz, double s_nu, double s_e,
                           int wy, int tz, hipStream_t s);
// FP64 reduction: out[0..6] = mass, momentum x, y, z, kinetic energy, max |J|, non-finite
// count; partials: 8 doubles per block of d3_diag_blocks(n)
int d3_diag_blocks(size_t n);
hipError_t launch_d3_diagnostics(int dtype, const void *state, size_t n, double *partials, double *out, hipStream_t s);

}  // namespace fdlbm
