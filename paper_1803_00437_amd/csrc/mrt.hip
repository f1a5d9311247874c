// MRT D2Q9 stream-collide step (section 1, eqs. 1-2; equilibria and rates of the table
// in section 1-a), the scheme the FD-LBM is compared against.
//
// Storage: the nine deviations f_k - w_k from the rest populations, row-interleaved (row j
// of population k at element (9 j + k) nx, pop_elem): the nine rows a node row reads are
// adjacent in memory, and so are the rows it writes.  Two kernels:
// one thread per node (mrt_kernel), and the vectorised sweep over lane groups of columns
// (mrt_sweep_kernel, the default).  Each relaxes the non-conserved moments of a node and
// pushes f*_k to x + e_k in the other buffer.  A population whose destination lies beyond
// a wall returns with the opposite velocity: halfway bounce-back (the wall half-way
// between the last fluid row and the next one, section 3-c), or the interpolated
// bounce-back of Bouzidi et al. for a wall at another distance xi, in both kernels (they
// agree bit for bit).  Algorithmic traffic: 9 values read + 9 written per node.
#include "fd_sweep_body.hpp"
#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {

template <typename C> struct MrtCoef {
    C se, sxx, sq, seps;
    C hfx, hfy, fx, fy;
};

// m = M f for the deviations (rows rho, Jx, Jy, E, XX, XY, qx, qy, eps of section 1).
template <typename C> __device__ __forceinline__ void moments(const C (&f)[9], C (&m)[9])
{
    const C ax = (f[1] + f[2]) + (f[3] + f[4]);
    const C dg = (f[5] + f[6]) + (f[7] + f[8]);
    const C x13 = f[1] - f[3], y24 = f[2] - f[4];
    const C dxp = (f[5] - f[6]) - (f[7] - f[8]);  // sum e_x over diagonals
    const C dyp = (f[5] + f[6]) - (f[7] + f[8]);  // sum e_y over diagonals
    m[0] = (f[0] + ax) + dg;
    m[1] = x13 + dxp;
    m[2] = y24 + dyp;
    m[3] = fmac(C(-4), f[0], fmac(C(2), dg, -ax));
    m[4] = (f[1] + f[3]) - (f[2] + f[4]);
    m[5] = (f[5] + f[7]) - (f[6] + f[8]);
    m[6] = fmac(C(-2), x13, dxp);
    m[7] = fmac(C(-2), y24, dyp);
    m[8] = fmac(C(4), f[0], fmac(C(-2), ax, dg));
}

// f = M^{-1} m, M^{-1} = M^T diag(1/9, 1/6, 1/6, 1/36, 1/4, 1/4, 1/12, 1/12, 1/36).
template <typename C> __device__ __forceinline__ void populations(const C (&m)[9], C (&f)[9])
{
    const C r9 = m[0] * C(1.0 / 9.0);
    const C e36 = m[3] * C(1.0 / 36.0), p36 = m[8] * C(1.0 / 36.0);
    f[0] = fmac(C(-4), e36, fmac(C(4), p36, r9));
    const C ax = fmac(C(-2), p36, r9 - e36);            // rho/9 - E/36 - eps/18
    const C dg = fmac(C(2), e36, r9 + p36);             // rho/9 + E/18 + eps/36
    const C xx = m[4] * C(0.25), xy = m[5] * C(0.25);
    const C jx6 = m[1] * C(1.0 / 6.0), jy6 = m[2] * C(1.0 / 6.0);
    const C qx6 = m[6] * C(1.0 / 6.0), qy6 = m[7] * C(1.0 / 6.0);
    const C ux = jx6 - qx6, uy = jy6 - qy6;             // axis: J/6 - q/6 (M_q = -2e on axes)
    const C vx = fmac(qx6, C(0.5), jx6), vy = fmac(qy6, C(0.5), jy6);  // diagonal: J/6 + q/12
    f[1] = (ax + xx) + ux;
    f[3] = (ax + xx) - ux;
    f[2] = (ax - xx) + uy;
    f[4] = (ax - xx) - uy;
    f[5] = (dg + xy) + (vx + vy);
    f[7] = (dg + xy) - (vx + vy);
    f[6] = (dg - xy) + (vy - vx);
    f[8] = (dg - xy) - (vy - vx);
}

// f += M^{-1} d for a moment increment d that leaves the mass unchanged (d[0] is not read).
// Adding the small change to the stored deviations, instead of rebuilding f from the
// relaxed moments, keeps the FP32 rounding relative to the change rather than to f: in a
// slow steady flow the rebuilt form's rounding biases every step the same way.
template <typename C> __device__ __forceinline__ void add_increment(const C (&d)[9], C (&f)[9])
{
    const C e36 = d[3] * C(1.0 / 36.0), p36 = d[8] * C(1.0 / 36.0);
    f[0] = f[0] + C(4) * (p36 - e36);
    const C ax = -fmac(C(2), p36, e36);                 // -E/36 - eps/18
    const C dg = fmac(C(2), e36, p36);                  // E/18 + eps/36
    const C xx = d[4] * C(0.25), xy = d[5] * C(0.25);
    const C jx6 = d[1] * C(1.0 / 6.0), jy6 = d[2] * C(1.0 / 6.0);
    const C qx6 = d[6] * C(1.0 / 6.0), qy6 = d[7] * C(1.0 / 6.0);
    const C ux = jx6 - qx6, uy = jy6 - qy6;
    const C vx = fmac(qx6, C(0.5), jx6), vy = fmac(qy6, C(0.5), jy6);
    f[1] = f[1] + ((ax + xx) + ux);
    f[3] = f[3] + ((ax + xx) - ux);
    f[2] = f[2] + ((ax - xx) + uy);
    f[4] = f[4] + ((ax - xx) - uy);
    f[5] = f[5] + ((dg + xy) + (vx + vy));
    f[7] = f[7] + ((dg + xy) - (vx + vy));
    f[6] = f[6] + ((dg - xy) + (vy - vx));
    f[8] = f[8] + ((dg - xy) - (vy - vx));
}

// Equilibrium moments of section 1-a as deviations from the rest moments.
template <typename C>
__device__ __forceinline__ void equilibrium(C dr, C jx, C jy, C &E, C &XX, C &XY, C &qx, C &qy, C &eps)
{
    const C rinv = recip(C(1) + dr);
    const C p = jx * jx, q = jy * jy;
    const C K3 = C(3) * ((p + q) * rinv);
    E = fmac(C(-2), dr, K3);
    XX = (p - q) * rinv;
    XY = (jx * jy) * rinv;
    qx = -jx;
    qy = -jy;
    eps = dr - K3;
}

// Collision of one node: moments, relaxation of the non-conserved ones toward the
// equilibria (eq. 1) with the force split half before and half after (Strang), and the
// post-collision populations f* = f + M^{-1} (m* - m).  Every MRT kernel calls this, so
// all of them agree bit for bit.
template <typename C> __device__ __forceinline__ void collide(C (&f)[9], const MrtCoef<C> &k)
{
    C m[9];
    moments<C>(f, m);
    // Strang splitting: half the force before the collision ...
    const C jax = m[1] + k.hfx, jay = m[2] + k.hfy;
    C E, XX, XY, qx, qy, eps;
    equilibrium<C>(m[0], jax, jay, E, XX, XY, qx, qy, eps);
    C d[9];
    d[0] = C(0);
    // ... the whole force over the step (the other half after the collision) ...
    d[1] = k.fx;
    d[2] = k.fy;
    // ... and eq. 1 for the non-conserved moments
    d[3] = k.se * (E - m[3]);
    d[4] = k.sxx * (XX - m[4]);
    d[5] = k.sxx * (XY - m[5]);
    d[6] = k.sq * (qx - m[6]);
    d[7] = k.sq * (qy - m[7]);
    d[8] = k.seps * (eps - m[8]);
    add_increment<C>(d, f);
}

// Reference MRT step: one thread per node.  With walls, a population whose destination
// lies beyond a wall returns to its node with the opposite velocity.  The wall cuts that
// link at the fraction xi of its length (walls at y = -xi and ny - 1 + xi), and the
// returning population is the linear interpolation of Bouzidi, Firdaouss and Lallemand:
//   xi <  1/2:  f_kbar(x) = 2 xi f*_k(x) + (1 - 2 xi) f*_k(x - e_k)
//   xi >= 1/2:  f_kbar(x) = f*_k(x) / (2 xi) + (2 xi - 1) / (2 xi) f*_kbar(x)
// which is halfway bounce-back at xi = 1/2.  For xi < 1/2 the thread collides the node
// behind it, x - e_k, once more.
template <typename T, bool WALLS>
__global__ void __launch_bounds__(256) mrt_kernel(const T *__restrict__ in, T *__restrict__ out, int nx, int ny,
                                                  MrtCoef<typename Storage<T>::C> k, typename Storage<T>::C xi)
{
    using C = typename Storage<T>::C;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= nx || j >= ny) return;
    C f[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = Storage<T>::load(in[pop_elem(i, j, q, nx)]);
    collide<C>(f, k);
    // propagation, eq. 2 (push)
    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    int jp = j + 1, jm = j - 1;
    if (!WALLS) {
        if (jp == ny) jp = 0;
        if (jm < 0) jm = ny - 1;
    }
    // post-collision population q at node (ii, jj), collided again (interpolated bounce-back)
    auto post_at = [&](int ii, int jj, int q) -> C {
        ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
        C g[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) g[r] = Storage<T>::load(in[pop_elem(ii, jj, r, nx)]);
        collide<C>(g, k);
        C v = g[0];
#pragma unroll
        for (int r = 1; r < 9; ++r)
            if (r == q) v = g[r];
        return v;
    };
    // population kq leaving toward the wall along (ex, ey), returning as kb
    auto back = [&](int kq, int kb, int ex, int ey) -> C {
        if (xi == C(0.5)) return f[kq];
        if (xi > C(0.5)) return f[kq] / (C(2) * xi) + (C(2) * xi - C(1)) / (C(2) * xi) * f[kb];
        return C(2) * xi * f[kq] + (C(1) - C(2) * xi) * post_at(i - ex, j - ey, kq);
    };
    out[pop_elem(i, j, 0, nx)] = Storage<T>::store(f[0]);
    out[pop_elem(ip, j, 1, nx)] = Storage<T>::store(f[1]);
    out[pop_elem(im, j, 3, nx)] = Storage<T>::store(f[3]);
    if (!WALLS || jp < ny) {
        out[pop_elem(i, jp, 2, nx)] = Storage<T>::store(f[2]);
        out[pop_elem(ip, jp, 5, nx)] = Storage<T>::store(f[5]);
        out[pop_elem(im, jp, 6, nx)] = Storage<T>::store(f[6]);
    } else {  // bounce-back at the upper wall
        out[pop_elem(i, j, 4, nx)] = Storage<T>::store(back(2, 4, 0, 1));
        out[pop_elem(i, j, 7, nx)] = Storage<T>::store(back(5, 7, 1, 1));
        out[pop_elem(i, j, 8, nx)] = Storage<T>::store(back(6, 8, -1, 1));
    }
    if (!WALLS || jm >= 0) {
        out[pop_elem(i, jm, 4, nx)] = Storage<T>::store(f[4]);
        out[pop_elem(im, jm, 7, nx)] = Storage<T>::store(f[7]);
        out[pop_elem(ip, jm, 8, nx)] = Storage<T>::store(f[8]);
    } else {  // bounce-back at the lower wall
        out[pop_elem(i, j, 2, nx)] = Storage<T>::store(back(4, 2, 0, -1));
        out[pop_elem(i, j, 5, nx)] = Storage<T>::store(back(7, 5, -1, -1));
        out[pop_elem(i, j, 6, nx)] = Storage<T>::store(back(8, 6, 1, -1));
    }
}

// Vectorised MRT step.  A wavefront owns 64*CPL consecutive columns (CPL per lane, one
// aligned vector access per population row) of R rows.  After the collision, the
// populations moving along +x / -x are shifted by one column across lanes with DPP
// whole-wave shifts, so every store is an aligned vector too; the outermost lane on each
// side has no neighbour to take from and only feeds its neighbour, so strips overlap by
// one lane on each side.  Populations moving along y go to the row above or below (or
// bounce back at a wall).  Wavefronts are dealt out row band after row band.
//
// The nine population rows of the next grid row are loaded while the current one is collided (two row
// buffers, the loop unrolled by two so that they alternate without copies).  Loads and
// stores go through range-checked buffer resources: the halo lanes' stores and the
// prefetch past the last row use an offset beyond the row and are dropped, so every row
// issues the same memory operations without branches.
//
// WALL: 0 periodic in y; 1 walls half-way between rows (halfway bounce-back); 2 walls at a
// distance xi (interpolated bounce-back, the same expressions as mrt_kernel; for xi < 1/2
// the row next to the wall row is loaded and collided once more for f*_k(x - e_k), the
// populations at x - e_k coming from the neighbouring lane with the same DPP shifts).
template <typename T, int CPL, int WALL>
__global__ void __launch_bounds__(256) mrt_sweep_kernel(const T *__restrict__ in, T *__restrict__ out, int nx, int ny,
                                                        int rows, int strips_x, int ntiles,
                                                        MrtCoef<typename Storage<T>::C> k, typename Storage<T>::C xi)
{
    constexpr bool WALLS = WALL != 0;
    using C = typename Storage<T>::C;
    using namespace sweep;
    constexpr int S = 64 * CPL - 2 * CPL;  // stored columns per strip
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (tile >= ntiles) return;  // uniform over the wavefront
    const int band = tile / strips_x, sx = tile - band * strips_x;
    const int xl = sx * S - CPL + CPL * lane;  // first column of this lane (unwrapped)
    const unsigned col = ((xl % nx) + nx) % nx;
    const bool store_ok = lane >= 1 && lane <= 62 && xl < nx;
    const unsigned voff = col * (unsigned)sizeof(T);
    const unsigned soff = store_ok ? voff : OFF_NONE;  // halo lanes do not store
    const int y0 = band * rows, y1 = min(y0 + rows, ny);

    auto load_row = [&](int y, bool use, Group<T, CPL>(&g)[9]) {
        const int yy = min(y, ny - 1);
#pragma unroll
        for (int q = 0; q < 9; ++q)
            g[q] = buf_load_group<T, CPL>(row_rsrc(in + pop_elem(0, 0, q, nx), yy, 9 * nx, nx), use ? voff : OFF_NONE);
    };
    auto put = [&](int q, int y, const Group<T, CPL> &g) {
        buf_store_group<T, CPL>(row_rsrc(out + pop_elem(0, 0, q, nx), y, 9 * nx, nx), soff, g);
    };
    // post-collision populations of row yy (the row next to a wall, collided once more)
    auto collide_row = [&](int yy, C(&h)[CPL][9]) {
        Group<T, CPL> g[9];
        load_row(yy, true, g);
#pragma unroll
        for (int q = 0; q < 9; ++q)
#pragma unroll
            for (int c = 0; c < CPL; ++c) h[c][q] = Storage<T>::load(g[q].v[c]);
#pragma unroll
        for (int c = 0; c < CPL; ++c) collide<C>(h[c], k);
    };
    // populations returning from a wall into this row: kq leaves along (ex, ey) (ey = +1 at
    // the top wall, -1 at the bottom one) and returns as kb; ynb is the row behind the node
    auto bounce = [&](const C(&f)[CPL][9], int kq, int kb, int ex, int ynb, Group<T, CPL> &b) {
        if (WALL == 1 || xi == C(0.5)) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) b.v[c] = Storage<T>::store(f[c][kq]);
        } else if (xi > C(0.5)) {
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                b.v[c] = Storage<T>::store(f[c][kq] / (C(2) * xi) + (C(2) * xi - C(1)) / (C(2) * xi) * f[c][kb]);
        } else if constexpr (WALL == 2) {
            C h[CPL][9];
            collide_row(ynb, h);
            // f*_kq at x - e_kq: column - ex, i.e. from the left for ex = +1, the right for -1
            const C edge = ex > 0 ? from_left(h[CPL - 1][kq]) : ex < 0 ? from_right(h[0][kq]) : C(0);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const C behind = ex == 0 ? h[c][kq]
                                 : ex > 0 ? (c > 0 ? h[c > 0 ? c - 1 : 0][kq] : edge)
                                          : (c < CPL - 1 ? h[c < CPL - 1 ? c + 1 : 0][kq] : edge);
                b.v[c] = Storage<T>::store(C(2) * xi * f[c][kq] + (C(1) - C(2) * xi) * behind);
            }
        }
    };
    // collide row y (populations in `cur`) and push its post-collision populations
    auto process = [&](int y, const Group<T, CPL>(&cur)[9]) {
        C f[CPL][9];
#pragma unroll
        for (int q = 0; q < 9; ++q)
#pragma unroll
            for (int c = 0; c < CPL; ++c) f[c][q] = Storage<T>::load(cur[q].v[c]);
#pragma unroll
        for (int c = 0; c < CPL; ++c) collide<C>(f[c], k);
        // destination rows (wave-uniform); with walls a population leaving the channel
        // returns to its own node with the opposite velocity
        int yp = y + 1, ym = y - 1;
        const bool top_wall = WALLS && yp == ny, bottom_wall = WALLS && ym < 0;
        if (!WALLS) {
            if (yp == ny) yp = 0;
            if (ym < 0) ym = ny - 1;
        }
        Group<T, CPL> g[9];
        // velocities (0,0), (0,+1), (0,-1) keep their column
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            g[0].v[c] = Storage<T>::store(f[c][0]);
            g[2].v[c] = Storage<T>::store(f[c][2]);
            g[4].v[c] = Storage<T>::store(f[c][4]);
        }
        // +x movers (1, 5, 8) arrive from the column on the left, -x movers (3, 6, 7) from
        // the column on the right
        const int rq[3] = {1, 5, 8}, lq[3] = {3, 6, 7};
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const C fl = from_left(f[CPL - 1][rq[t]]), fr = from_right(f[0][lq[t]]);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                g[rq[t]].v[c] = Storage<T>::store(c > 0 ? f[c > 0 ? c - 1 : 0][rq[t]] : fl);
                g[lq[t]].v[c] = Storage<T>::store(c < CPL - 1 ? f[c < CPL - 1 ? c + 1 : 0][lq[t]] : fr);
            }
        }
        put(0, y, g[0]);
        put(1, y, g[1]);
        put(3, y, g[3]);
        if (top_wall) {
            // the upward movers return into this row's downward populations, unshifted
            Group<T, CPL> b2, b5, b6;
            bounce(f, 2, 4, 0, y - 1, b2);
            bounce(f, 5, 7, 1, y - 1, b5);
            bounce(f, 6, 8, -1, y - 1, b6);
            put(4, y, b2);
            put(7, y, b5);
            put(8, y, b6);
        } else {
            put(2, yp, g[2]);
            put(5, yp, g[5]);
            put(6, yp, g[6]);
        }
        if (bottom_wall) {
            Group<T, CPL> b4, b7, b8;
            bounce(f, 4, 2, 0, y + 1, b4);
            bounce(f, 7, 5, -1, y + 1, b7);
            bounce(f, 8, 6, 1, y + 1, b8);
            put(2, y, b4);
            put(5, y, b7);
            put(6, y, b8);
        } else {
            put(4, ym, g[4]);
            put(7, ym, g[7]);
            put(8, ym, g[8]);
        }
    };

    Group<T, CPL> A[9], B[9];
    load_row(y0, true, A);
    for (int y = y0; y < y1; y += 2) {
        load_row(y + 1, y + 1 < y1, B);
        process(y, A);
        if (y + 1 >= y1) break;
        load_row(y + 2, y + 2 < y1, A);
        process(y + 1, B);
    }
}

// Equilibrium populations of host-order FP64 planes (drho, Jx, Jy; node (i, j) at j nx + i),
// stored row-interleaved; one block row of columns per grid row.
template <typename T>
__global__ void __launch_bounds__(256) mrt_init_kernel(const double *__restrict__ dr, const double *__restrict__ jx,
                                                       const double *__restrict__ jy, T *__restrict__ pop, int nx, int ny)
{
    using C = typename Storage<T>::C;
    for (int j = blockIdx.x; j < ny; j += gridDim.x)
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            const size_t p = (size_t)j * (size_t)nx + (size_t)i;
            C m[9], f[9];
            m[0] = C(dr[p]);
            m[1] = C(jx[p]);
            m[2] = C(jy[p]);
            equilibrium<C>(m[0], m[1], m[2], m[3], m[4], m[5], m[6], m[7], m[8]);
            populations<C>(m, f);
#pragma unroll
            for (int q = 0; q < 9; ++q) pop[pop_elem(i, j, q, nx)] = Storage<T>::store(f[q]);
        }
}

// Conserved moments of the stored populations, summed in FP64 whatever the storage dtype,
// into host-order planes.
template <typename T>
__global__ void __launch_bounds__(256) mrt_moments_kernel(const T *__restrict__ pop, double *__restrict__ dr,
                                                          double *__restrict__ jx, double *__restrict__ jy, int nx,
                                                          int ny)
{
    for (int j = blockIdx.x; j < ny; j += gridDim.x)
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            const size_t p = (size_t)j * (size_t)nx + (size_t)i;
            double f[9], m[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) f[q] = double(Storage<T>::load(pop[pop_elem(i, j, q, nx)]));
            moments<double>(f, m);
            dr[p] = m[0];
            jx[p] = m[1];
            jy[p] = m[2];
        }
}

template <typename T, int CPL>
hipError_t run_sweep(const MrtArgs &a, MrtCoef<typename Storage<T>::C> k, const void *src, void *dst, hipStream_t s)
{
    constexpr int S = 64 * CPL - 2 * CPL;
    const int rows = a.tile_rows > 0 ? a.tile_rows : 1;  // 1 measured best at 8192^2 (1 % over 2)
    const int strips_x = (a.nx + S - 1) / S;
    const int ntiles = strips_x * ((a.ny + rows - 1) / rows);
    const int blocks = (ntiles + 3) / 4;
    using C = typename Storage<T>::C;
    if (a.walls && a.xi != 0.5)
        hipLaunchKernelGGL((mrt_sweep_kernel<T, CPL, 2>), blocks, 256, 0, s, static_cast<const T *>(src),
                           static_cast<T *>(dst), a.nx, a.ny, rows, strips_x, ntiles, k, C(a.xi));
    else if (a.walls)
        hipLaunchKernelGGL((mrt_sweep_kernel<T, CPL, 1>), blocks, 256, 0, s, static_cast<const T *>(src),
                           static_cast<T *>(dst), a.nx, a.ny, rows, strips_x, ntiles, k, C(0.5));
    else
        hipLaunchKernelGGL((mrt_sweep_kernel<T, CPL, 0>), blocks, 256, 0, s, static_cast<const T *>(src),
                           static_cast<T *>(dst), a.nx, a.ny, rows, strips_x, ntiles, k, C(0.5));
    return hipGetLastError();
}

template <typename T> hipError_t run(const MrtArgs &a, const void *src, void *dst, hipStream_t s)
{
    using C = typename Storage<T>::C;
    MrtCoef<C> k{C(a.s_e), C(a.s_xx), C(a.s_q), C(a.s_eps), C(0.5 * a.fx), C(0.5 * a.fy), C(a.fx), C(a.fy)};
    if (a.kernel != FDLBM_KERNEL_REFERENCE) {
        constexpr int CPL = sizeof(T) == 8 ? 2 : 4;
        if (a.nx % CPL == 0) return run_sweep<T, CPL>(a, k, src, dst, s);
        if (a.nx % 2 == 0) return run_sweep<T, 2>(a, k, src, dst, s);
        return run_sweep<T, 1>(a, k, src, dst, s);
    }
    dim3 blk(64, 4), grd((a.nx + 63) / 64, (a.ny + 3) / 4);
    if (a.walls)
        hipLaunchKernelGGL((mrt_kernel<T, true>), grd, blk, 0, s, static_cast<const T *>(src), static_cast<T *>(dst),
                           a.nx, a.ny, k, C(a.xi));
    else
        hipLaunchKernelGGL((mrt_kernel<T, false>), grd, blk, 0, s, static_cast<const T *>(src), static_cast<T *>(dst),
                           a.nx, a.ny, k, C(0.5));
    return hipGetLastError();
}

inline unsigned rows_grid(int ny) { return (unsigned)(ny < 65536 ? ny : 65536); }

}  // namespace

hipError_t launch_mrt(const MrtArgs &a, const void *src, void *dst, hipStream_t s)
{
    return a.dtype == FDLBM_F64 ? run<double>(a, src, dst, s) : run<float>(a, src, dst, s);
}

hipError_t launch_mrt_init(int dtype, const double *dr, const double *jx, const double *jy, void *pop, int nx, int ny,
                           hipStream_t s)
{
    if (dtype == FDLBM_F64)
        hipLaunchKernelGGL(mrt_init_kernel<double>, rows_grid(ny), 256, 0, s, dr, jx, jy, static_cast<double *>(pop), nx,
                           ny);
    else
        hipLaunchKernelGGL(mrt_init_kernel<float>, rows_grid(ny), 256, 0, s, dr, jx, jy, static_cast<float *>(pop), nx,
                           ny);
    return hipGetLastError();
}

hipError_t launch_mrt_moments(int dtype, const void *pop, double *dr, double *jx, double *jy, int nx, int ny,
                              hipStream_t s)
{
    if (dtype == FDLBM_F64)
        hipLaunchKernelGGL(mrt_moments_kernel<double>, rows_grid(ny), 256, 0, s, static_cast<const double *>(pop), dr,
                           jx, jy, nx, ny);
    else
        hipLaunchKernelGGL(mrt_moments_kernel<float>, rows_grid(ny), 256, 0, s, static_cast<const float *>(pop), dr,
                           jx, jy, nx, ny);
    return hipGetLastError();
}

}  // namespace fdlbm
