// FD-LBM step, reference path (two passes through a scratch buffer).
//
// Pass 1 computes, for every node that sends a population into the fluid, the nine
// post-collision populations of section 2 and writes them to nine planes; pass 2 gathers
// the propagated populations (eq. 2) and adds their difference from the node's own to the
// stored (drho, jx, jy).  It moves about four times the bytes of the fused kernel and
// exists as the plain GPU rendering that the fused kernel must match bit for bit; both
// use fd_node_fstar() (lw_node_g() for the LW-ACM step), row_sum(), same_row_part(),
// fd_partial() and fd_finish().
#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Value of (drho, J) at node (i, j) with the boundary rules: x periodic; y periodic, or,
// with walls, a ghost node takes the rule of ghost_rules() (linear extrapolation with zero
// velocity on the wall; at xi = 1/2 it mirrors the fluid node at the same distance from the
// wall, drho even and J odd).
template <typename T, bool WALLS> struct View {
    using C = typename Storage<T>::C;
    const T *st;  // row-interleaved state (fd_elem)
    int nx, ny;
    GhostRules<C> gr;
    __device__ __forceinline__ void load3(int i, int j, C &r, C &x, C &y) const
    {
        r = Storage<T>::load(st[fd_elem(i, j, 0, nx)]);
        x = Storage<T>::load(st[fd_elem(i, j, 1, nx)]);
        y = Storage<T>::load(st[fd_elem(i, j, 2, nx)]);
    }
    __device__ __forceinline__ void at(int i, int j, C &r, C &x, C &y) const
    {
        i = wrap(wrap(i, nx), nx);
        if (WALLS && (j < 0 || j >= ny)) {
            const GhostRule<C> q = ghost_rule(gr, j < 0 ? -j : j - ny + 1);
            const int ja = j < 0 ? q.sa : ny - 1 - q.sa;
            C ra, xa, ya;
            load3(i, ja, ra, xa, ya);
            r = q.car * ra;
            x = q.caj * xa;
            y = q.caj * ya;
            if (q.sb >= 0) {
                const int jb = j < 0 ? q.sb : ny - 1 - q.sb;
                C rb, xb, yb;
                load3(i, jb, rb, xb, yb);
                r = r + q.cbr * rb;
                x = x + q.cbj * xb;
                y = y + q.cbj * yb;
            }
            return;
        }
        if (!WALLS) j = wrap(wrap(j, ny), ny);
        load3(i, j, r, x, y);
    }
};

template <typename T, int ST, bool WALLS, bool FORCE>
__global__ void __launch_bounds__(256) fd_ref_fstar(View<T, WALLS> v, FdCoef<typename Storage<T>::C> k, int row0,
                                                    int nrows, typename Storage<T>::C *__restrict__ fstar)
{
    using C = typename Storage<T>::C;
    constexpr int H = Stencil<ST>::H;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int rr = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= v.nx || rr >= nrows) return;
    const int j = row0 + rr;
    const size_t plane = (size_t)nrows * (size_t)v.nx;
    const size_t p = (size_t)rr * (size_t)v.nx + (size_t)i;
    if constexpr (ST == 1) {  // LW-ACM: the populations g of the node alone
        C r, x, y, f[9];
        v.at(i, j, r, x, y);
        lw_node_g<C>(r, x, y, k.lin, f);
#pragma unroll
        for (int q = 0; q < 9; ++q) fstar[q * plane + p] = f[q];
        return;
    }

    // values along the x and y axes through the node, offsets -2..2 (index o + 2)
    C rX[5], xX[5], yX[5], rY[5], xY[5], yY[5];
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
        if (o < -H || o > H) {
            rX[o + 2] = xX[o + 2] = yX[o + 2] = rY[o + 2] = xY[o + 2] = yY[o + 2] = C(0);
            continue;
        }
        v.at(i + o, j, rX[o + 2], xX[o + 2], yX[o + 2]);
        v.at(i, j + o, rY[o + 2], xY[o + 2], yY[o + 2]);
    }
    using S = Stencil<ST>;
    C d[10];
    d[0] = S::diff(rX[0], rX[1], rX[3], rX[4]);
    d[1] = S::diff(rY[0], rY[1], rY[3], rY[4]);
    d[2] = S::diff(xX[0], xX[1], xX[3], xX[4]);
    d[3] = S::diff(yY[0], yY[1], yY[3], yY[4]);
    d[4] = S::diff(yX[0], yX[1], yX[3], yX[4]);
    d[5] = S::diff(xY[0], xY[1], xY[3], xY[4]);
    // products of J_a = J + F/2
    C P[5], Rx[5], Ry[5], Q[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        const C ax = plus_force<FORCE>(xX[o], k.hfx), ay = plus_force<FORCE>(yX[o], k.hfy);
        const C bx = plus_force<FORCE>(xY[o], k.hfx), by = plus_force<FORCE>(yY[o], k.hfy);
        P[o] = ax * ax;
        Rx[o] = ax * ay;
        Ry[o] = bx * by;
        Q[o] = by * by;
    }
    d[6] = S::diff(P[0], P[1], P[3], P[4]);
    d[7] = S::diff(Ry[0], Ry[1], Ry[3], Ry[4]);
    d[8] = S::diff(Rx[0], Rx[1], Rx[3], Rx[4]);
    d[9] = S::diff(Q[0], Q[1], Q[3], Q[4]);

    C f[9];
    fd_node_fstar<C, FORCE>(rX[2], plus_force<FORCE>(xX[2], k.hfx), plus_force<FORCE>(yX[2], k.hfy), d, k, f);
#pragma unroll
    for (int q = 0; q < 9; ++q) fstar[q * plane + p] = f[q];
}

template <typename T, bool WALLS, bool FORCE>
__global__ void __launch_bounds__(256) fd_ref_gather(const typename Storage<T>::C *__restrict__ fstar,
                                                     const T *__restrict__ in, FdCoef<typename Storage<T>::C> k,
                                                     int nx, int ny, int row0, int nrows, T *__restrict__ out,
                                                     uint32_t seed)
{
    using C = typename Storage<T>::C;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t plane = (size_t)nrows * (size_t)nx;
    auto F = [&](int q, int di, int dj) -> C {
        int ii = wrap(i + di, nx);
        int jj = j + dj;
        if (!WALLS) jj = wrap(jj, ny);
        const int rr = jj - row0;  // walls: row0 = -1, so rows -1..ny map to 0..ny+1
        return fstar[q * plane + (size_t)rr * (size_t)nx + (size_t)ii];
    };
    // arriving minus own, per source row: same row, row below, row above
    C pc, pcx;
    same_row_part<C>(F(1, -1, 0) - F(1, 0, 0), F(3, 1, 0) - F(3, 0, 0), pc, pcx);
    const C pu = row_sum(F(2, 0, -1), F(5, -1, -1), F(6, 1, -1)) - row_sum(F(2, 0, 0), F(5, 0, 0), F(6, 0, 0));
    const C pux = (F(5, -1, -1) - F(6, 1, -1)) - (F(5, 0, 0) - F(6, 0, 0));
    const C pd = row_sum(F(4, 0, 1), F(8, -1, 1), F(7, 1, 1)) - row_sum(F(4, 0, 0), F(8, 0, 0), F(7, 0, 0));
    const C pdx = (F(8, -1, 1) - F(7, 1, 1)) - (F(8, 0, 0) - F(7, 0, 0));
    const size_t p = (size_t)j * (size_t)nx + (size_t)i;  // node index
    C r, x, y;
    fd_finish<C, FORCE>(fd_partial<C>(pc, pcx, pu, pux), pd, pdx, Storage<T>::load(in[fd_elem(i, j, 0, nx)]),
                        Storage<T>::load(in[fd_elem(i, j, 1, nx)]), Storage<T>::load(in[fd_elem(i, j, 2, nx)]), k.dfx,
                        k.dfy, r, x, y);
    // rounded for storage (stochastically for HalfSR: the same bits as the sweep kernel)
    uint32_t rb[3] = {0u, 0u, 0u};
    if constexpr (Storage<T>::STOCHASTIC) sr_draw(uint32_t(p), seed, rb);
    out[fd_elem(i, j, 0, nx)] = Storage<T>::store_r(r, rb[0]);
    out[fd_elem(i, j, 1, nx)] = Storage<T>::store_r(x, rb[1]);
    out[fd_elem(i, j, 2, nx)] = Storage<T>::store_r(y, rb[2]);
}

template <typename T> FdCoef<typename Storage<T>::C> make_coef(const FdArgs &a)
{
    using C = typename Storage<T>::C;
    const double scale = a.stencil == 3 ? Stencil<3>::SCALE : Stencil<5>::SCALE;
    FdCoef<C> k;
    const double ke = 2.0 * scale * (1.0 - 1.0 / a.s_e);
    k.eax = C(-ke / 36.0);
    k.edg = C(ke / 18.0);
    k.e0 = C(-ke / 9.0);
    k.kxx = C(scale * (1.0 - 1.0 / a.s_xx));
    k.kxx2 = C(2.0 * scale * (1.0 - 1.0 / a.s_xx));
    k.hfx = C(0.5 * a.fx);
    k.hfy = C(0.5 * a.fy);
    k.qfx = C(0.25 * a.fx);
    k.qfy = C(0.25 * a.fy);
    k.dfx = C(a.fx);
    k.dfy = C(a.fy);
    k.lin = C(2.0 / a.s_xx - 1.0);
    return k;
}

template <typename T, int ST, bool WALLS, bool FORCE>
hipError_t run(const FdArgs &a, const void *src, void *dst, void *fstar, hipStream_t s)
{
    using C = typename Storage<T>::C;
    const T *in = static_cast<const T *>(src);
    T *out = static_cast<T *>(dst);
    auto k = make_coef<T>(a);
    View<T, WALLS> v{in, a.nx, a.ny, ghost_rules<C>(a.xi)};
    const int row0 = WALLS ? -1 : 0, nrows = WALLS ? a.ny + 2 : a.ny;
    dim3 blk(64, 4);
    dim3 g1((a.nx + 63) / 64, (nrows + 3) / 4);
    hipLaunchKernelGGL((fd_ref_fstar<T, ST, WALLS, FORCE>), g1, blk, 0, s, v, k, row0, nrows, static_cast<C *>(fstar));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((a.nx + 63) / 64, (a.ny + 3) / 4);
    hipLaunchKernelGGL((fd_ref_gather<T, WALLS, FORCE>), g2, blk, 0, s, static_cast<const C *>(fstar), in, k, a.nx, a.ny,
                       row0, nrows, out, a.seed);
    return hipGetLastError();
}

template <typename T, int ST, bool WALLS>
hipError_t dispatch_force(const FdArgs &a, const void *src, void *dst, void *fstar, hipStream_t s)
{
    if (a.fx != 0.0 || a.fy != 0.0) return run<T, ST, WALLS, true>(a, src, dst, fstar, s);
    return run<T, ST, WALLS, false>(a, src, dst, fstar, s);
}

template <typename T>
hipError_t dispatch_stencil(const FdArgs &a, const void *src, void *dst, void *fstar, hipStream_t s)
{
    if (a.stencil == 1) return run<T, 1, false, false>(a, src, dst, fstar, s);  // LW-ACM, periodic
    if (a.stencil == 3)
        return a.walls ? dispatch_force<T, 3, true>(a, src, dst, fstar, s)
                       : dispatch_force<T, 3, false>(a, src, dst, fstar, s);
    return a.walls ? dispatch_force<T, 5, true>(a, src, dst, fstar, s) : dispatch_force<T, 5, false>(a, src, dst, fstar, s);
}

}  // namespace

size_t fd_reference_scratch_bytes(const FdArgs &a)
{
    const size_t rows = (size_t)a.ny + (a.walls ? 2 : 0);
    return 9 * rows * (size_t)a.nx * compute_bytes(a.dtype);
}

hipError_t launch_fd_reference(const FdArgs &a, const void *src, void *dst, void *fstar, hipStream_t s)
{
    switch (a.dtype) {
    case FDLBM_F64: return dispatch_stencil<double>(a, src, dst, fstar, s);
    case FDLBM_F32: return dispatch_stencil<float>(a, src, dst, fstar, s);
    case FDLBM_F16DEV_SR: return dispatch_stencil<HalfSR>(a, src, dst, fstar, s);
    default: return dispatch_stencil<__half>(a, src, dst, fstar, s);
    }
}

}  // namespace fdlbm
