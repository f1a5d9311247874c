// FD-LBM step, fused sweep path: one kernel per time step, state read once and written
// once (3 values per node each way), no scratch memory.
//
// Mapping (designed for CDNA4's 64-wide wavefronts):
//   * a block is WV wavefronts stacked in y over one strip of W = 64*CPL consecutive
//     columns (CPL columns per lane, loaded and stored as one aligned vector per field
//     where the grid width allows, else as element-aligned vectors or column by column);
//     each wavefront sweeps its own R rows of the strip;
//   * x-neighbours of a lane's outer columns come from the adjacent lanes through DPP
//     whole-wave shifts (wave_shl:1 / wave_shr:1), so no LDS and no barrier is needed
//     along x.  A node update needs h+1 columns on each side (h = 1 for 3-point, 2 for
//     5-point differences); neighbouring strips overlap by whole halo lanes so that every
//     access stays aligned;
//   * y-neighbours live in a rolling window of 2h+1 input rows held in registers, with the
//     next one or two rows in flight; the row loop is unrolled by the window length so
//     that the window rotates by renaming, not by register moves;
//   * the post-collision populations of a row are exchanged along x with the same DPP
//     shifts and split into the parts landing on the row itself, the row above and the
//     row below; the output row below the current one is then complete and is stored
//     with a non-temporal hint (it is read again only at the next step);
//   * the first and last output rows of a wavefront also need the populations sent by the
//     rows just outside it.  Inside a block those rows belong to the neighbouring
//     wavefronts, which publish their partial sums in LDS; after one barrier every
//     wavefront finishes its two boundary rows.  Only the block's outermost wavefronts
//     compute the populations of one extra row each;
//   * blocks are dealt out row band after row band, so the resident blocks cover a compact
//     block of rows: the halo rows a block shares with the bands above and below are then
//     re-read from cache, and HBM sees a few long sequential streams;
//   * all row bookkeeping is wave-uniform (scalar registers).
// Per node the arithmetic is fd_node_fstar() and the update is formed with the helpers and
// in the order of fdlbm_device.hpp, so the result equals the reference path bit for bit.
// A run without body force uses kernels built without the force additions.
//
// Walls (rows -1 .. -(h+1) and ny .. ny+h are ghosts): each ghost row is formed as it is
// loaded, by the rule of ghost_rules() for the wall distance xi (sections 3-b, 3-c: linear
// extrapolation with zero velocity on the wall; at xi = 1/2 the mirror, drho even, J odd).
#include "fd_sweep_body.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {
using namespace sweep;

template <typename T> struct SweepArgs {
    TileArgs<T> t;
    int strips_x;
};

template <typename T, int CPL, int ST, bool WALLS, bool FORCE, int AM>
__global__ void __launch_bounds__(64 * WV) fd_sweep_kernel(SweepArgs<T> a)
{
    // blocks dealt out row band after row band
    const int band = blockIdx.x / a.strips_x;
    const int sx = blockIdx.x - band * a.strips_x;
    sweep_tile<T, CPL, ST, WALLS, FORCE, AM>(a.t, band, sx * Strip<CPL, Stencil<ST>::H>::S, sx == a.strips_x - 1);
}

// Rows per wavefront when the caller leaves the choice open (fastest at 8192^2): FP32
// 3-point 8, FP32 5-point 16, LW-ACM 4, FP16 storage 16, FP64 6.  fdlbm_autotune measures
// instead.
int default_rows(const FdArgs &a)
{
    if (a.dtype == FDLBM_F64) return 6;
    if (is_f16(a.dtype)) return 16;
    if (a.stencil == 1) return 4;
    return a.stencil == 5 ? 16 : 8;
}

template <typename T, int CPL, int ST, bool WALLS, bool FORCE, int AM>
hipError_t run(const FdArgs &fa, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    using C = typename Storage<T>::C;
    using G = Strip<CPL, Stencil<ST>::H>;
    SweepArgs<T> a;
    const T *in = static_cast<const T *>(src);
    T *out = static_cast<T *>(dst);
    a.t.dr = in + fd_elem(0, 0, 0, fa.nx);
    a.t.jx = in + fd_elem(0, 0, 1, fa.nx);
    a.t.jy = in + fd_elem(0, 0, 2, fa.nx);
    a.t.odr = out + fd_elem(0, 0, 0, fa.nx);
    a.t.ojx = out + fd_elem(0, 0, 1, fa.nx);
    a.t.ojy = out + fd_elem(0, 0, 2, fa.nx);
    a.t.nx = fa.nx;
    a.t.ny = fa.ny;
    // rows per wavefront (>= 2, see the tile body)
    a.t.rows = tile_rows >= 2 ? tile_rows : default_rows(fa);
    a.t.k = make_coef<C>(ST, fa.s_xx, fa.s_e, fa.fx, fa.fy);
    a.t.gr = ghost_rules<C>(fa.xi);
    a.t.seed = fa.seed;
    a.strips_x = (fa.nx + G::S - 1) / G::S;
    const int nbands = (fa.ny + WV * a.t.rows - 1) / (WV * a.t.rows);
    hipLaunchKernelGGL((fd_sweep_kernel<T, CPL, ST, WALLS, FORCE, AM>), a.strips_x * nbands, 64 * WV, 0, s, a);
    return hipGetLastError();
}

template <typename T, int CPL, int ST, bool WALLS>
hipError_t dispatch_force(const FdArgs &a, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    // a lane's columns as one aligned vector access where nx is a multiple of CPL; else one
    // element-aligned vector access (FP32, FP64) or one access per column (FP16)
    // (LW-ACM, stencil 1, has no body force)
    const bool force = ST != 1 && (a.fx != 0.0 || a.fy != 0.0);
    if (a.nx % CPL == 0) {
        if constexpr (ST != 1)
            if (force) return run<T, CPL, ST, WALLS, true, AM_VEC>(a, tile_rows, src, dst, s);
        return run<T, CPL, ST, WALLS, false, AM_VEC>(a, tile_rows, src, dst, s);
    }
    if constexpr (CPL > 1) {
        constexpr int AM = sizeof(T) >= 4 ? AM_UNAL : AM_COL;
        if constexpr (ST != 1)
            if (force) return run<T, CPL, ST, WALLS, true, AM>(a, tile_rows, src, dst, s);
        return run<T, CPL, ST, WALLS, false, AM>(a, tile_rows, src, dst, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int CPL>
hipError_t dispatch_cpl(const FdArgs &a, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    if (a.stencil == 1) return dispatch_force<T, CPL, 1, false>(a, tile_rows, src, dst, s);  // LW-ACM, periodic
    if (a.stencil == 3)
        return a.walls ? dispatch_force<T, CPL, 3, true>(a, tile_rows, src, dst, s)
                       : dispatch_force<T, CPL, 3, false>(a, tile_rows, src, dst, s);
    if constexpr (CPL >= 2)
        return a.walls ? dispatch_force<T, CPL, 5, true>(a, tile_rows, src, dst, s)
                       : dispatch_force<T, CPL, 5, false>(a, tile_rows, src, dst, s);
    return hipErrorInvalidValue;
}

// Columns per lane (measured at 8192^2): FP32 and FP16 4 (16- and 8-byte accesses), FP64
// 2 (16-byte accesses), also where nx is not a multiple (element-aligned vector accesses),
// except FP16 at even widths, which keeps aligned 4-byte accesses of 2 columns (its odd
// widths access each column on its own).  1 column per lane is available for 3-point
// differences and LW-ACM only.
int choose_cpl(const FdArgs &a, int lane_cols)
{
    if (lane_cols > 0) return lane_cols;
    if (a.dtype == FDLBM_F64) return 2;
    if (is_f16(a.dtype) && a.nx % 4 == 2) return 2;
    return 4;
}

template <typename T>
hipError_t dispatch(const FdArgs &a, int tile_rows, int lane_cols, const void *src, void *dst, hipStream_t s)
{
    switch (choose_cpl(a, lane_cols)) {
    case 1: return dispatch_cpl<T, 1>(a, tile_rows, src, dst, s);
    case 2: return dispatch_cpl<T, 2>(a, tile_rows, src, dst, s);
    case 4:
        if constexpr (sizeof(T) != 8) return dispatch_cpl<T, 4>(a, tile_rows, src, dst, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool fd_sweep_supported(const FdArgs &a, int lane_cols)
{
    const int cpl = choose_cpl(a, lane_cols);
    const bool f64 = a.dtype == FDLBM_F64;
    if (a.stencil != 1 && a.stencil != 3 && a.stencil != 5) return false;
    if (a.stencil == 1 && (a.walls || a.fx != 0.0 || a.fy != 0.0)) return false;  // LW-ACM: periodic, no force
    if (cpl == 1) return a.stencil != 5;
    if (cpl == 4 && f64) return false;
    return cpl == 2 || cpl == 4;
}

hipError_t launch_fd_sweep(const FdArgs &a, int tile_rows, int lane_cols, const void *src, void *dst, hipStream_t s)
{
    switch (a.dtype) {
    case FDLBM_F64: return dispatch<double>(a, tile_rows, lane_cols, src, dst, s);
    case FDLBM_F32: return dispatch<float>(a, tile_rows, lane_cols, src, dst, s);
    case FDLBM_F16DEV_SR: return dispatch<HalfSR>(a, tile_rows, lane_cols, src, dst, s);
    default: return dispatch<__half>(a, tile_rows, lane_cols, src, dst, s);
    }
}

}  // namespace fdlbm
