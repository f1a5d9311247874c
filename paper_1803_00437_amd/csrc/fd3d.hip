// FD-LBM step on the D3Q19 lattice (section 2's construction in three dimensions; the
// per-node arithmetic is in fd3d_device.hpp).  Periodic grid nx * ny * nz, state as four
// planes (drho, Jx, Jy, Jz), node (x, y, z) at (z*ny + y)*nx + x.
//
// Reference path: d3_ref_fstar writes the 18 moving post-collision populations of every node
// to scratch planes, d3_ref_gather forms the new state from them.
//
// Sweep path (d3_sweep_kernel), one fused pass per step:
//   * a wavefront holds 64 consecutive columns of one row, one column per lane; the two
//     lanes at each end are halo (the 3-point differences and the propagation each reach one
//     column), so a wavefront updates 60 columns; x-neighbours come from the adjacent lanes
//     through DPP whole-wave shifts;
//   * a block stacks WY wavefronts on consecutive rows; the first and last are halo rows
//     (they form post-collision populations only, for the rows inside); y-neighbours are
//     exchanged through LDS, twice per plane: the stored fields of the plane (for the
//     y-differences) and the x-shifted group sums sent to the row above and below;
//   * the block sweeps TZ planes along z; each lane keeps its column's fields of three
//     planes in registers (plus one loaded ahead), and the partial update of the plane below
//     until the plane above has been formed;
//   * measured at 512^3 (FP32): 12 rows per block and 64 planes run fastest (86 000 MLUPS);
//     16 rows leave one block per compute unit (68 000), 8 rows spend a third of the work on
//     halo rows (83 000), 14 rows split 4/4/3/3 over the SIMDs so that a second block does not
//     fit (69 000); unrolling the plane loop to rename the window instead of copying it raised
//     the registers past six wavefronts per SIMD and ran 5-17 % slower;
//   * every index wraps (periodic grid), so a grid narrower than a tile is covered by lanes,
//     rows or planes that repeat: they compute and store the same bits.  The last strip, row
//     band and plane band are shifted back to end at the grid's edge, so tiles overlap there
//     instead of running past it (overlapping nodes are stored twice with the same bits).
#include "fd3d_device.hpp"
#include "fd_sweep_body.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace d3 {

__device__ __forceinline__ int wrapi(int i, int n)
{
    i %= n;
    return i < 0 ? i + n : i;
}

// ----------------------------------------------------------------- reference path ----

template <typename T>
__global__ __launch_bounds__(256) void d3_ref_fstar(const T *__restrict__ st, T *__restrict__ fs, int nx, int ny, int nz,
                                                    Coef3<T> k)
{
    using C = T;
    const size_t n = (size_t)nx * ny * nz, plane = (size_t)nx * ny;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny), kz = (int)(p / plane);
        const size_t o[3][2] = {
            {(size_t)kz * plane + (size_t)j * nx + wrapi(i + 1, nx), (size_t)kz * plane + (size_t)j * nx + wrapi(i - 1, nx)},
            {(size_t)kz * plane + (size_t)wrapi(j + 1, ny) * nx + i, (size_t)kz * plane + (size_t)wrapi(j - 1, ny) * nx + i},
            {(size_t)wrapi(kz + 1, nz) * plane + (size_t)j * nx + i, (size_t)wrapi(kz - 1, nz) * plane + (size_t)j * nx + i}};
        C v[4], nb[3][2][4];
        for (int f = 0; f < 4; ++f) {
            v[f] = st[f * n + p];
            for (int a = 0; a < 3; ++a)
                for (int s = 0; s < 2; ++s) nb[a][s][f] = st[f * n + o[a][s]];
        }
        const C j3[3] = {v[1], v[2], v[3]};
        C gr[3], dj[3][3], dpa[3][3];
        for (int a = 0; a < 3; ++a) {
            gr[a] = nb[a][0][0] - nb[a][1][0];
            for (int b = 0; b < 3; ++b) dj[a][b] = nb[a][0][1 + b] - nb[a][1][1 + b];
            // D_a of the products J_b J_a (b = x, y, z) at the two neighbours along a: along x the
            // difference of the two rounded products (the sweep forms each column's products once
            // and shifts them between lanes), along y and z one product fused into the difference
            for (int b = 0; b < 3; ++b)
                dpa[a][b] = a == 0 ? nb[a][0][1 + b] * nb[a][0][1 + a] - nb[a][1][1 + b] * nb[a][1][1 + a]
                                   : d3_pdiff(nb[a][0][1 + b], nb[a][0][1 + a], nb[a][1][1 + b], nb[a][1][1 + a]);
        }
        const C dp[3] = {d3_flux(dpa[0][0], dpa[1][0], dpa[2][0]), d3_flux(dpa[0][1], dpa[1][1], dpa[2][1]),
                         d3_flux(dpa[0][2], dpa[1][2], dpa[2][2])};
        C f[Q];
        d3_fstar<C>(v[0], j3, gr, dj, dp, k, f);
        for (int q = 1; q < Q; ++q) fs[(size_t)(q - 1) * n + p] = f[q];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void d3_ref_gather(const T *__restrict__ st, const T *__restrict__ fs,
                                                     T *__restrict__ out, int nx, int ny, int nz)
{
    using C = T;
    const size_t n = (size_t)nx * ny * nz, plane = (size_t)nx * ny;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny), kz = (int)(p / plane);
        auto F = [&](int q, int di, int dj, int dk) -> C {
            const size_t at = (size_t)wrapi(kz + dk, nz) * plane + (size_t)wrapi(j + dj, ny) * nx + wrapi(i + di, nx);
            return fs[(size_t)(q - 1) * n + at];
        };
        auto own = [&](int q) -> C { return fs[(size_t)(q - 1) * n + p]; };
        // from the plane below: group (0,1) = f5, f11 (from x-1), f14 (from x+1); f15, f18
        const C a11 = F(11, -1, 0, -1), a14 = F(14, 1, 0, -1);
        const C dS01 = d3_sum(F(5, 0, 0, -1), a11, a14) - d3_sum(own(5), own(11), own(14));
        const C dX01 = (a11 - a14) - (own(11) - own(14));
        const D3Part<C> lo = d3_lo(dS01, dX01, F(15, 0, -1, -1) - own(15), F(18, 0, 1, -1) - own(18));
        // same plane: f1, f2 along the row; group (1,0) from the row below, (-1,0) from above
        const C e1 = F(1, -1, 0, 0) - own(1), e2 = F(2, 1, 0, 0) - own(2);
        const C b7 = F(7, -1, -1, 0), b10 = F(10, 1, -1, 0);
        const C dS10 = d3_sum(F(3, 0, -1, 0), b7, b10) - d3_sum(own(3), own(7), own(10));
        const C dX10 = (b7 - b10) - (own(7) - own(10));
        const C c9 = F(9, -1, 1, 0), c8 = F(8, 1, 1, 0);
        const C dSm10 = d3_sum(F(4, 0, 1, 0), c9, c8) - d3_sum(own(4), own(9), own(8));
        const C dXm10 = (c9 - c8) - (own(9) - own(8));
        const D3Part<C> part = d3_lo_mid(lo, e1, e2, dS10, dX10, dSm10, dXm10);
        // from the plane above: group (0,-1) = f6, f13 (from x-1), f12 (from x+1); f17, f16
        const C h13 = F(13, -1, 0, 1), h12 = F(12, 1, 0, 1);
        const C dS0m1 = d3_sum(F(6, 0, 0, 1), h13, h12) - d3_sum(own(6), own(13), own(12));
        const C dX0m1 = (h13 - h12) - (own(13) - own(12));
        C r, x, y, z;
        d3_finish(part, dS0m1, dX0m1, F(17, 0, -1, 1) - own(17), F(16, 0, 1, 1) - own(16), st[p], st[n + p],
                  st[2 * n + p], st[3 * n + p], r, x, y, z);
        out[p] = r;
        out[n + p] = x;
        out[2 * n + p] = y;
        out[3 * n + p] = z;
    }
}

// --------------------------------------------------------------------- sweep path ----

constexpr int LANES = 64, XU = LANES - 4;  // columns per wavefront, of which updated

template <typename T, int WY>
__global__ __launch_bounds__(LANES *WY) void d3_sweep_kernel(const T *__restrict__ st, T *__restrict__ out, int nx,
                                                             int ny, int nz, int tz, Coef3<T> k)
{
    using C = T;
    using sweep::from_left;
    using sweep::from_right;
    constexpr int YU = WY - 2;  // rows updated per block
    __shared__ C lds_f[WY][4][LANES];   // the fields of the current plane, per row
    __shared__ C lds_g[WY][8][LANES];   // sums sent to the row above (0..3) and below (4..7)

    const int lane = threadIdx.x & (LANES - 1);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const size_t n = (size_t)nx * ny * nz, plane = (size_t)nx * ny;

    int x0 = blockIdx.x * XU;
    if (x0 + XU > nx) x0 = nx > XU ? nx - XU : 0;
    int y0 = blockIdx.y * YU;
    if (y0 + YU > ny) y0 = ny > YU ? ny - YU : 0;
    int z0 = blockIdx.z * tz;
    if (z0 + tz > nz) z0 = nz > tz ? nz - tz : 0;

    const int col = wrapi(x0 - 2 + lane, nx);
    const bool halo_lo = w == 0, halo_hi = w == WY - 1;
    const bool store_lane = lane >= 2 && lane < LANES - 2 && !halo_lo && !halo_hi;
    // Accesses go through one buffer resource per field plane (scalar base and size), so the
    // per-lane part of every address is a 32-bit byte offset fixed for the whole sweep: this
    // row, the outer row of a halo wave, and this row for the stores (beyond the plane, where
    // the hardware drops the store, for the halo lanes and rows).
    const unsigned off_row = (unsigned)(((size_t)wrapi(y0 - 1 + w, ny) * nx + col) * sizeof(T));
    const unsigned off_out = (unsigned)(((size_t)wrapi(halo_lo ? y0 - 2 : y0 + WY - 1, ny) * nx + col) * sizeof(T));
    const unsigned off_st = store_lane ? off_row : sweep::OFF_NONE;
    using Ops = sweep::BufOps<sizeof(T)>;
    auto rsrc = [&](const T *base, int f, int pz) {
        const unsigned long long r = reinterpret_cast<unsigned long long>(base + (size_t)f * n + (size_t)pz * plane);
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)r);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(r >> 32));
        void *b = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
        return __builtin_amdgcn_make_buffer_rsrc(b, 0, (int)(plane * sizeof(T)), sweep::RSRC_WORD3);
    };
    auto load4 = [&](unsigned off, int pz, C (&d)[4]) {  // pz wrapped by the caller
        for (int f = 0; f < 4; ++f) d[f] = __builtin_bit_cast(T, Ops::load(rsrc(st, f, pz), off));
    };

    // window: planes p-1, p, p+1 of this row; nxt: plane p+2; outer row (halo waves): plane p
    C win[3][4], nxt[4], orow[4], onxt[4];
    load4(off_row, wrapi(z0 - 2, nz), win[0]);
    load4(off_row, wrapi(z0 - 1, nz), win[1]);
    load4(off_row, wrapi(z0, nz), win[2]);
    for (int f = 0; f < 4; ++f) orow[f] = onxt[f] = C(0);
    if (halo_lo || halo_hi) load4(off_out, wrapi(z0 - 1, nz), orow);
    auto next_plane = [&](int z) { return z + 1 == nz ? 0 : z + 1; };
    int zn = wrapi(z0 + 1, nz);  // plane p+2: this row's next load
    int zo = wrapi(z0, nz);      // plane p+1: the outer row's next load
    int zs = wrapi(z0 - 2, nz);  // plane p-1: completed in this iteration

    // carried between planes: arrivals for the plane above (group (0,1) and f15, f18 from the
    // neighbouring rows) and, for the plane below, its partial update and own sums of the
    // groups that come down from this plane
    C a01s = 0, a01x = 0, a15 = 0, a18 = 0;
    D3Part<C> part{0, 0, 0, 0};
    C o0m1s = 0, o0m1x = 0, o17 = 0, o16 = 0;

    for (int it = 0; it < tz + 2; ++it) {
        load4(off_row, zn, nxt);  // plane p + 2 (p = z0 - 1 + it: the plane formed now)
        if (halo_lo || halo_hi) load4(off_out, zo, onxt);

        for (int f = 0; f < 4; ++f) lds_f[w][f][lane] = win[1][f];
        __syncthreads();
        C up[4], dn[4];
        for (int f = 0; f < 4; ++f) {
            up[f] = halo_hi ? orow[f] : lds_f[halo_hi ? w : w + 1][f][lane];
            dn[f] = halo_lo ? orow[f] : lds_f[halo_lo ? w : w - 1][f][lane];
        }

        // differences along x (lanes), y (LDS rows) and z (window planes)
        const C *c = win[1];
        const C jj[3] = {c[1], c[2], c[3]};
        C gr[3], dj[3][3];
        gr[0] = from_right(c[0]) - from_left(c[0]);
        gr[1] = up[0] - dn[0];
        gr[2] = win[2][0] - win[0][0];
        for (int b = 0; b < 3; ++b) {
            dj[0][b] = from_right(c[1 + b]) - from_left(c[1 + b]);
            dj[1][b] = up[1 + b] - dn[1 + b];
            dj[2][b] = win[2][1 + b] - win[0][1 + b];
        }
        C dp[3];
        for (int b = 0; b < 3; ++b) {
            const C px = c[1 + b] * c[1];  // J_b J_x of this column, for the neighbours' x-differences
            const C dx = from_right(px) - from_left(px);
            const C dy = d3_pdiff(up[1 + b], up[2], dn[1 + b], dn[2]);
            const C dz = d3_pdiff(win[2][1 + b], win[2][3], win[0][1 + b], win[0][3]);
            dp[b] = d3_flux(dx, dy, dz);
        }
        C f[Q];
        d3_fstar<C>(c[0], jj, gr, dj, dp, k, f);

        // x-shifted group sums that leave this row
        const C l7 = from_left(f[7]), r10 = from_right(f[10]);
        const C l9 = from_left(f[9]), r8 = from_right(f[8]);
        lds_g[w][0][lane] = d3_sum(f[3], l7, r10);  // (1,0) to the row above
        lds_g[w][1][lane] = l7 - r10;
        lds_g[w][2][lane] = f[15];  // (1,1): row above, plane above
        lds_g[w][3][lane] = f[17];  // (1,-1): row above, plane below
        lds_g[w][4][lane] = d3_sum(f[4], l9, r8);  // (-1,0) to the row below
        lds_g[w][5][lane] = l9 - r8;
        lds_g[w][6][lane] = f[16];  // (-1,-1): row below, plane below
        lds_g[w][7][lane] = f[18];  // (-1,1): row below, plane above
        // A halo row only sends: its own update is never stored, so it skips it (the branch is
        // uniform in each wavefront; every wavefront still meets both barriers).
        const bool inner = !halo_lo && !halo_hi;
        C s01 = 0, x01 = 0, s0m1 = 0, x0m1 = 0, e1 = 0, e2 = 0;
        if (inner) {
            const C l11 = from_left(f[11]), r14 = from_right(f[14]);
            const C l13 = from_left(f[13]), r12 = from_right(f[12]);
            s01 = d3_sum(f[5], l11, r14);  // (0,1): this row, plane above
            x01 = l11 - r14;
            s0m1 = d3_sum(f[6], l13, r12);  // (0,-1): this row, plane below
            x0m1 = l13 - r12;
            e1 = from_left(f[1]) - f[1];
            e2 = from_right(f[2]) - f[2];
        }
        __syncthreads();
        if (inner) {
            const C in10s = lds_g[w - 1][0][lane], in10x = lds_g[w - 1][1][lane];
            const C in15 = lds_g[w - 1][2][lane], in17 = lds_g[w - 1][3][lane];
            const C inm10s = lds_g[w + 1][4][lane], inm10x = lds_g[w + 1][5][lane];
            const C in16 = lds_g[w + 1][6][lane], in18 = lds_g[w + 1][7][lane];

            // the plane below (p - 1) is complete: its arrivals from plane p are in
            if (it >= 2) {
                C r, x, y, z;
                d3_finish(part, s0m1 - o0m1s, x0m1 - o0m1x, in17 - o17, in16 - o16, win[0][0], win[0][1], win[0][2],
                          win[0][3], r, x, y, z);
                const C v[4] = {r, x, y, z};
                for (int f = 0; f < 4; ++f)
                    Ops::store(__builtin_bit_cast(typename Ops::W, v[f]), rsrc(out, f, zs), off_st);
            }
            // this plane: arrivals from the plane below (carried) and from this plane
            const D3Part<C> lo =
                d3_lo(a01s - d3_sum(f[5], f[11], f[14]), a01x - (f[11] - f[14]), a15 - f[15], a18 - f[18]);
            part = d3_lo_mid(lo, e1, e2, in10s - d3_sum(f[3], f[7], f[10]), in10x - (f[7] - f[10]),
                             inm10s - d3_sum(f[4], f[9], f[8]), inm10x - (f[9] - f[8]));
            o0m1s = d3_sum(f[6], f[13], f[12]);
            o0m1x = f[13] - f[12];
            o17 = f[17];
            o16 = f[16];
            a01s = s01;
            a01x = x01;
            a15 = in15;
            a18 = in18;
        }
        zn = next_plane(zn);
        zo = next_plane(zo);
        zs = next_plane(zs);
        for (int q = 0; q < 4; ++q) {
            win[0][q] = win[1][q];
            win[1][q] = win[2][q];
            win[2][q] = nxt[q];
            orow[q] = onxt[q];
        }
    }
}

// ------------------------------------------------------------------- diagnostics ----

constexpr int DTPB = 256, DIAG3 = 8;

template <typename T>
__global__ __launch_bounds__(DTPB) void d3_diag_partials(const T *__restrict__ st, size_t n, double *__restrict__ part)
{
    __shared__ double sh[DIAG3][DTPB];
    double a[DIAG3] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (size_t p = (size_t)blockIdx.x * DTPB + threadIdx.x; p < n; p += (size_t)gridDim.x * DTPB) {
        const double r = st[p], x = st[n + p], y = st[2 * n + p], z = st[3 * n + p];
        const double j2 = x * x + y * y + z * z;
        if (!(__builtin_isfinite(r) && __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z))) {
            a[6] += 1.0;
            continue;
        }
        a[0] += r;
        a[1] += x;
        a[2] += y;
        a[3] += z;
        a[4] += 0.5 * j2 / (1.0 + r);
        a[5] = fmax(a[5], sqrt(j2));
    }
    for (int q = 0; q < DIAG3; ++q) sh[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int s = DTPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < DIAG3; ++q)
                sh[q][threadIdx.x] = q == 5 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + s])
                                            : sh[q][threadIdx.x] + sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < DIAG3) part[(size_t)blockIdx.x * DIAG3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(DTPB) void d3_diag_final(const double *__restrict__ part, int blocks, double *__restrict__ out)
{
    __shared__ double sh[DIAG3][DTPB];
    double a[DIAG3] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < blocks; b += DTPB)
        for (int q = 0; q < DIAG3; ++q) a[q] = q == 5 ? fmax(a[q], part[(size_t)b * DIAG3 + q]) : a[q] + part[(size_t)b * DIAG3 + q];
    for (int q = 0; q < DIAG3; ++q) sh[q][threadIdx.x] = a[q];
    __syncthreads();
    for (int s = DTPB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int q = 0; q < DIAG3; ++q)
                sh[q][threadIdx.x] = q == 5 ? fmax(sh[q][threadIdx.x], sh[q][threadIdx.x + s])
                                            : sh[q][threadIdx.x] + sh[q][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < DIAG3) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace d3

// ------------------------------------------------------------------------ launches ----

namespace {
unsigned ref_blocks(size_t n)
{
    const size_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? b : 65536);
}
}  // namespace

hipError_t launch_d3_reference(int dtype, const void *in, void *out, void *fstar, int nx, int ny, int nz, double s_nu,
                               double s_e, hipStream_t s)
{
    const size_t n = (size_t)nx * ny * nz;
    if (dtype == FDLBM_F64) {
        hipLaunchKernelGGL(d3::d3_ref_fstar<double>, ref_blocks(n), 256, 0, s, (const double *)in, (double *)fstar, nx,
                           ny, nz, d3::coef3<double>(s_nu, s_e));
        hipLaunchKernelGGL(d3::d3_ref_gather<double>, ref_blocks(n), 256, 0, s, (const double *)in,
                           (const double *)fstar, (double *)out, nx, ny, nz);
    } else {
        hipLaunchKernelGGL(d3::d3_ref_fstar<float>, ref_blocks(n), 256, 0, s, (const float *)in, (float *)fstar, nx, ny,
                           nz, d3::coef3<float>(s_nu, s_e));
        hipLaunchKernelGGL(d3::d3_ref_gather<float>, ref_blocks(n), 256, 0, s, (const float *)in, (const float *)fstar,
                           (float *)out, nx, ny, nz);
    }
    return hipGetLastError();
}

// Grid of the sweep: strips of 60 columns, bands of WY - 2 rows, bands of tz planes.
Dim3Grid d3_sweep_grid(int nx, int ny, int nz, int wy, int tz)
{
    const int yu = wy - 2;
    return Dim3Grid{(nx + d3::XU - 1) / d3::XU, (ny + yu - 1) / yu, (nz + tz - 1) / tz};
}

hipError_t launch_d3_sweep(int dtype, const void *in, void *out, int nx, int ny, int nz, double s_nu, double s_e,
                           int wy, int tz, hipStream_t s)
{
    const Dim3Grid g = d3_sweep_grid(nx, ny, nz, wy, tz);
    const dim3 grid(g.x, g.y, g.z);
    if (dtype == FDLBM_F64) {
        const auto k = d3::coef3<double>(s_nu, s_e);
        if (wy == 8)
            hipLaunchKernelGGL((d3::d3_sweep_kernel<double, 8>), grid, 64 * 8, 0, s, (const double *)in, (double *)out,
                               nx, ny, nz, tz, k);
        else if (wy == 12)
            hipLaunchKernelGGL((d3::d3_sweep_kernel<double, 12>), grid, 64 * 12, 0, s, (const double *)in,
                               (double *)out, nx, ny, nz, tz, k);
        else
            hipLaunchKernelGGL((d3::d3_sweep_kernel<double, 16>), grid, 64 * 16, 0, s, (const double *)in,
                               (double *)out, nx, ny, nz, tz, k);
    } else {
        const auto k = d3::coef3<float>(s_nu, s_e);
        if (wy == 8)
            hipLaunchKernelGGL((d3::d3_sweep_kernel<float, 8>), grid, 64 * 8, 0, s, (const float *)in, (float *)out, nx,
                               ny, nz, tz, k);
        else if (wy == 12)
            hipLaunchKernelGGL((d3::d3_sweep_kernel<float, 12>), grid, 64 * 12, 0, s, (const float *)in, (float *)out,
                               nx, ny, nz, tz, k);
        else
            hipLaunchKernelGGL((d3::d3_sweep_kernel<float, 16>), grid, 64 * 16, 0, s, (const float *)in, (float *)out,
                               nx, ny, nz, tz, k);
    }
    return hipGetLastError();
}

int d3_diag_blocks(size_t n)
{
    const size_t b = (n + d3::DTPB - 1) / d3::DTPB;
    return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_d3_diagnostics(int dtype, const void *state, size_t n, double *partials, double *out, hipStream_t s)
{
    const int blocks = d3_diag_blocks(n);
    if (dtype == FDLBM_F64)
        hipLaunchKernelGGL(d3::d3_diag_partials<double>, blocks, d3::DTPB, 0, s, (const double *)state, n, partials);
    else
        hipLaunchKernelGGL(d3::d3_diag_partials<float>, blocks, d3::DTPB, 0, s, (const float *)state, n, partials);
    hipLaunchKernelGGL(d3::d3_diag_final, 1, d3::DTPB, 0, s, (const double *)partials, blocks, out);
    return hipGetLastError();
}

}  // namespace fdlbm
