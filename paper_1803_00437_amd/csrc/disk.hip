// Curved no-slip wall around a disk (section 3-b): the ghost-node table, built on the host
// once per context, and the kernel that fills ghost and rest nodes before each periodic
// step (FD-LBM, LW-ACM); for MRT D2Q9, the boundary-link table and the kernels that apply
// the interpolated bounce-back of Bouzidi et al. after each periodic step and return the
// solid nodes to rest.
//
// Section 3-b states the principle: the nodes just outside the fluid carry a virtual-fluid
// state, extrapolated linearly with zero velocity on the wall, by an expression chosen from
// where the wall cuts the link.  The rule implemented here, the curved counterpart of the
// straight-wall ghost rows: a ghost node at r = R + d on the ray of unit vector n takes the
// state at its mirror point c + (R - d) n, momentum negated and density kept, bilinearly
// interpolated when the four nodes around the mirror point are fluid; otherwise (mirror
// point in the last cell before the wall) the momentum runs linearly from zero on the wall
// to the sample at depth 3/2, J = -(d / 1.5) J(c + (R - 1.5) n), with that sample's density.
// Ghost nodes are the non-fluid nodes within Chebyshev distance 3 of the fluid: one
// propagation link plus the two-node reach of the 5-point differences, so no fluid update
// reads anything else.  Every other node is held at rest.  A step maps a rest
// neighbourhood (all deviations zero) to exactly zero unless a body force acts, so after
// one full clearing only the ring of rest nodes within that same reach of the fluid and
// ghost nodes (periodic images included) can leave rest, and only the ring is cleared.
#include <algorithm>
#include <cmath>

#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {

namespace {

constexpr double SAMPLE_DEPTH = 1.5;
constexpr int GHOST_REACH = 3;

struct Disk {
    double cx, cy, r;
    bool fluid(long i, long j) const { return std::hypot(double(i) - cx, double(j) - cy) < r; }
};

// fluid columns [lo, hi] of row j (lo > hi: none); the disk is convex, so they are contiguous
void fluid_span(const Disk &d, int j, long *lo, long *hi)
{
    const double dy = double(j) - d.cy;
    *lo = 1;
    *hi = 0;
    if (!(std::fabs(dy) < d.r)) return;
    const double half = std::sqrt(d.r * d.r - dy * dy);
    long a = (long)std::floor(d.cx - half), b = (long)std::ceil(d.cx + half);
    // settle the ends with the exact membership test
    while (d.fluid(a - 1, j)) --a;
    while (a <= b && !d.fluid(a, j)) ++a;
    while (d.fluid(b + 1, j)) ++b;
    while (b >= a && !d.fluid(b, j)) --b;
    *lo = a;
    *hi = b;
}

}  // namespace

bool build_disk_table(int nx, int ny, double cx, double cy, double r, DiskTable *out)
{
    if (!(std::isfinite(cx) && std::isfinite(cy) && std::isfinite(r)) || !(r > SAMPLE_DEPTH)) return false;
    if (size_t(nx) * size_t(ny) >= (size_t(1) << 31)) return false;  // 32-bit node indices
    // every fluid node (r < R) then lies in [GHOST_REACH, n - 1 - GHOST_REACH] on both axes
    if (!(cx - r >= GHOST_REACH - 1 && cx + r <= nx - GHOST_REACH && cy - r >= GHOST_REACH - 1 &&
          cy + r <= ny - GHOST_REACH))
        return false;
    const Disk d{cx, cy, r};
    std::vector<long> flo(ny), fhi(ny);
    size_t nfluid = 0;
    for (int j = 0; j < ny; ++j) {
        fluid_span(d, j, &flo[j], &fhi[j]);
        if (flo[j] <= fhi[j]) {
            if (flo[j] < GHOST_REACH || fhi[j] > nx - 1 - GHOST_REACH) return false;
            if (j < GHOST_REACH || j > ny - 1 - GHOST_REACH) return false;
            nfluid += size_t(fhi[j] - flo[j] + 1);
        }
    }
    if (nfluid == 0) return false;
    DiskTable t;
    t.nfluid = nfluid;
    t.span.assign(2 * size_t(ny), 0);
    auto cell = [&](double px, double py, int32_t *src, double *wx, double *wy) {
        const long i0 = (long)std::floor(px), j0 = (long)std::floor(py);
        if (!(d.fluid(i0, j0) && d.fluid(i0 + 1, j0) && d.fluid(i0, j0 + 1) && d.fluid(i0 + 1, j0 + 1))) return false;
        *src = int32_t(j0 * nx + i0);
        *wx = px - double(i0);
        *wy = py - double(j0);
        return true;
    };
    for (int j = 0; j < ny; ++j) {
        // Chebyshev dilation of the fluid by GHOST_REACH, row by row
        long a = nx, b = -1;
        for (int k = j - GHOST_REACH; k <= j + GHOST_REACH; ++k) {
            if (k < 0 || k >= ny || flo[k] > fhi[k]) continue;
            a = std::min(a, flo[k] - GHOST_REACH);
            b = std::max(b, fhi[k] + GHOST_REACH);
        }
        t.span[2 * size_t(j)] = int32_t(a);
        t.span[2 * size_t(j) + 1] = int32_t(b);
        for (long i = a; i <= b; ++i) {
            if (i >= flo[j] && i <= fhi[j]) continue;
            const double rr = std::hypot(double(i) - cx, double(j) - cy);
            const double ux = (double(i) - cx) / rr, uy = (double(j) - cy) / rr;
            const double delta = rr - r;
            int32_t src;
            double wx, wy, sj = -1.0;
            if (!cell(cx + (r - delta) * ux, cy + (r - delta) * uy, &src, &wx, &wy)) {
                if (!cell(cx + (r - SAMPLE_DEPTH) * ux, cy + (r - SAMPLE_DEPTH) * uy, &src, &wx, &wy)) return false;
                sj = -delta / SAMPLE_DEPTH;
            }
            t.dst.push_back(int32_t(long(j) * nx + i));
            t.src.push_back(src);
            t.w.push_back(wx);
            t.w.push_back(wy);
            t.w.push_back(sj);
        }
    }
    // ring: rest nodes within GHOST_REACH (the step's reach) of a fluid or ghost node,
    // across the periodic edges as well
    std::vector<long> rlo(ny, 0), rhi(ny, -1);
    std::vector<char> dirty(ny, 0);
    for (int k = 0; k < ny; ++k) {
        const long a = t.span[2 * size_t(k)], b = t.span[2 * size_t(k) + 1];
        if (a > b) continue;
        for (int dj = -GHOST_REACH; dj <= GHOST_REACH; ++dj) {
            const int j = ((k + dj) % ny + ny) % ny;
            if (!dirty[j]) {
                rlo[j] = a - GHOST_REACH;
                rhi[j] = b + GHOST_REACH;
                dirty[j] = 1;
            } else {
                rlo[j] = std::min(rlo[j], a - GHOST_REACH);
                rhi[j] = std::max(rhi[j], b + GHOST_REACH);
            }
        }
    }
    for (int j = 0; j < ny; ++j) {
        if (!dirty[j]) continue;
        const long a = t.span[2 * size_t(j)], b = t.span[2 * size_t(j) + 1];
        const long hi = std::min(rhi[j], rlo[j] + nx - 1);  // at most one whole row
        for (long c = rlo[j]; c <= hi; ++c) {
            const long i = (c % nx + nx) % nx;
            if (i >= a && i <= b) continue;
            t.ring.push_back(int32_t(long(j) * nx + i));
        }
    }
    // MRT D2Q9: the boundary links, every (fluid node x, direction k) whose x + e_k is solid.
    // The wall cuts the link at x + q e_k with |x + q e_k - c| = R, the root in (0, 1] of
    // a q^2 + b q + c0 = 0 (x inside, x + e_k outside).
    static const int EXk[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}, EYk[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    t.fspan.assign(2 * size_t(ny), 0);
    for (int j = 0; j < ny; ++j) {
        t.fspan[2 * size_t(j)] = int32_t(flo[j]);
        t.fspan[2 * size_t(j) + 1] = int32_t(fhi[j]);
        for (long i = flo[j]; i <= fhi[j]; ++i)
            for (int k = 1; k < 9; ++k) {
                if (d.fluid(i + EXk[k], j + EYk[k])) continue;
                const double px = double(i) - cx, py = double(j) - cy;
                const double a = double(EXk[k] * EXk[k] + EYk[k] * EYk[k]);
                const double b = 2.0 * (px * EXk[k] + py * EYk[k]);
                const double c0 = px * px + py * py - r * r;
                double q = (-b + std::sqrt(b * b - 4.0 * a * c0)) / (2.0 * a);
                if (!(q > 0.0)) return false;
                q = std::min(q, 1.0);
                const bool back = d.fluid(i - EXk[k], j - EYk[k]);
                t.link_node.push_back(int32_t(long(j) * nx + i));
                t.link_kb.push_back(int32_t(k | (back ? 16 : 0)));
                t.link_q.push_back(q);
                t.solid_ring.push_back(int32_t((long(j) + EYk[k]) * nx + i + EXk[k]));
            }
    }
    std::sort(t.solid_ring.begin(), t.solid_ring.end());
    t.solid_ring.erase(std::unique(t.solid_ring.begin(), t.solid_ring.end()), t.solid_ring.end());
    *out = std::move(t);
    return true;
}

namespace {

constexpr int TPB = 256;

// threads [0, nghost): one ghost node each; then either one thread per ring node (set to
// rest), or, for a full clearing, one thread per CLEAR_COLS columns of a row, which sets the
// nodes outside the row's fluid-or-ghost span to rest.  Ghost threads read fluid nodes only
// and write ghost nodes only, so the fill works in place.
constexpr int CLEAR_COLS = 8;

template <typename T>
__global__ __launch_bounds__(TPB) void disk_fill_kernel(DiskFill f, T *state, int full)
{
    using S = Storage<T>;
    using C = typename S::C;
    const size_t t = size_t(blockIdx.x) * TPB + threadIdx.x;
    const size_t nx = size_t(f.nx);
    // element of field p at a node index (j nx + i) of the row-interleaved state (fd_elem)
    auto elem = [&](size_t node, int p) { return fd_elem(node % nx, node / nx, p, nx); };
    if (t < size_t(f.nghost)) {
        const size_t s = size_t(f.src[t]), dst = size_t(f.dst[t]);
        const C wx = C(f.w[3 * t]), wy = C(f.w[3 * t + 1]), sj = C(f.w[3 * t + 2]);
        const C ux = C(1) - wx, uy = C(1) - wy;
        for (int p = 0; p < 3; ++p) {
            const T *a = state + elem(s, p);  // the cell's corners: +1 the next column, +3 nx the next row
            const C lower = ux * S::load(a[0]) + wx * S::load(a[1]);
            const C upper = ux * S::load(a[3 * nx]) + wx * S::load(a[3 * nx + 1]);
            const C v = uy * lower + wy * upper;
            state[elem(dst, p)] = S::store(p == 0 ? v : sj * v);
        }
        return;
    }
    const size_t u = t - size_t(f.nghost);
    if (!full) {
        if (u >= size_t(f.nring)) return;
        const size_t node = size_t(f.ring[u]);
        for (int p = 0; p < 3; ++p) state[elem(node, p)] = S::store(C(0));
        return;
    }
    const size_t per_row = (size_t(f.nx) + CLEAR_COLS - 1) / CLEAR_COLS;
    if (u >= per_row * size_t(f.ny)) return;
    const int j = int(u / per_row);
    const int i0 = int(u - size_t(j) * per_row) * CLEAR_COLS;
    const int a = f.span[2 * j], b = f.span[2 * j + 1];
    for (int i = i0; i < min(i0 + CLEAR_COLS, f.nx); ++i) {
        if (i >= a && i <= b) continue;
        for (int p = 0; p < 3; ++p) state[fd_elem(i, j, p, nx)] = S::store(C(0));
    }
}

// MRT: one thread per boundary link.  The population re-entering the fluid node x along
// k' = -e_k is rebuilt from post-collision values still present in the streamed grid:
// f*_k(x) at the solid node x + e_k, f*_k(x - e_k) at x itself, f*_k'(x) at x - e_k:
//   q <  1/2:  2q f*_k(x) + (1 - 2q) f*_k(x - e_k)   (halfway bounce-back if x - e_k is solid)
//   q >= 1/2:  f*_k(x) / (2q) + (2q - 1)/(2q) f*_k'(x)
// No thread writes what another reads (the writes go to fluid nodes, direction k', which
// no link reads), so the links run in any order, in place.
template <typename T> __global__ __launch_bounds__(TPB) void mrt_disk_links_kernel(MrtDisk d, T *pop)
{
    using S = Storage<T>;
    using C = typename S::C;
    const int t = int(blockIdx.x) * TPB + int(threadIdx.x);
    if (t >= d.nlinks) return;
    const int kb = d.kb[t], k = kb & 15;
    const bool back = (kb >> 4) != 0;
    const int opp = k <= 4 ? ((k + 1) & 3) + 1 : ((k - 3) & 3) + 5;  // 1<->3, 2<->4, 5<->7, 6<->8
    const int ex = (k == 1 || k == 5 || k == 8) - (k == 3 || k == 6 || k == 7);
    const int ey = (k == 2 || k == 5 || k == 6) - (k == 4 || k == 7 || k == 8);
    const size_t nx = size_t(d.nx);
    // element of population p at a node index (j nx + i) of the row-interleaved state
    auto at = [&](long node, int p) { return pop_elem(size_t(node) % nx, size_t(node) / nx, p, nx); };
    const long node = d.node[t];
    const long off = long(ex) + long(ey) * long(d.nx);
    const C fi_x = S::load(pop[at(node + off, k)]);
    const C fb_x = S::load(pop[at(node - off, opp)]);
    const C fi_back = S::load(pop[at(node, k)]);
    const C q = C(d.q[t]);
    C v;
    if (q < C(0.5))
        v = back ? C(2) * q * fi_x + (C(1) - C(2) * q) * fi_back : fi_x;
    else
        v = fi_x / (C(2) * q) + (C(2) * q - C(1)) / (C(2) * q) * fb_x;
    pop[at(node, opp)] = S::store(v);
}

// MRT: solid nodes to rest (all nine deviations zero): the ring the links reach, or, for a
// full clearing, every node outside its row's fluid span (CLEAR_COLS columns per thread).
template <typename T> __global__ __launch_bounds__(TPB) void mrt_disk_clear_kernel(MrtDisk d, T *pop, int full)
{
    using S = Storage<T>;
    using C = typename S::C;
    const size_t t = size_t(blockIdx.x) * TPB + threadIdx.x;
    const size_t nx = size_t(d.nx);
    if (!full) {
        if (t >= size_t(d.nring)) return;
        const size_t node = size_t(d.ring[t]);
        for (int p = 0; p < 9; ++p) pop[pop_elem(node % nx, node / nx, p, nx)] = S::store(C(0));
        return;
    }
    const size_t per_row = (size_t(d.nx) + CLEAR_COLS - 1) / CLEAR_COLS;
    if (t >= per_row * size_t(d.ny)) return;
    const int j = int(t / per_row);
    const int i0 = int(t - size_t(j) * per_row) * CLEAR_COLS;
    const int a = d.fspan[2 * j], b = d.fspan[2 * j + 1];
    for (int i = i0; i < min(i0 + CLEAR_COLS, d.nx); ++i) {
        if (i >= a && i <= b) continue;
        for (int p = 0; p < 9; ++p) pop[pop_elem(i, j, p, nx)] = S::store(C(0));
    }
}

template <typename T> hipError_t mrt_disk_run(const MrtDisk &d, T *pop, bool full, hipStream_t s)
{
    if (d.nlinks > 0) {
        hipLaunchKernelGGL(mrt_disk_links_kernel<T>, dim3(unsigned((d.nlinks + TPB - 1) / TPB)), TPB, 0, s, d, pop);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const size_t per_row = (size_t(d.nx) + CLEAR_COLS - 1) / CLEAR_COLS;
    const size_t threads = full ? per_row * size_t(d.ny) : size_t(d.nring);
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(mrt_disk_clear_kernel<T>, dim3(unsigned((threads + TPB - 1) / TPB)), TPB, 0, s, d, pop,
                       full ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mrt_disk(const MrtDisk &d, int dtype, void *pop, bool full, hipStream_t s)
{
    switch (dtype) {
    case FDLBM_F64: return mrt_disk_run<double>(d, static_cast<double *>(pop), full, s);
    case FDLBM_F32: return mrt_disk_run<float>(d, static_cast<float *>(pop), full, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_disk_fill(const DiskFill &f, int dtype, void *state, bool full, hipStream_t s)
{
    const size_t per_row = (size_t(f.nx) + CLEAR_COLS - 1) / CLEAR_COLS;
    const size_t threads = size_t(f.nghost) + (full ? per_row * size_t(f.ny) : size_t(f.nring));
    const dim3 grid(unsigned((threads + TPB - 1) / TPB));
    const int fl = full ? 1 : 0;
    switch (dtype) {
    case FDLBM_F64: hipLaunchKernelGGL(disk_fill_kernel<double>, grid, TPB, 0, s, f, (double *)state, fl); break;
    case FDLBM_F32: hipLaunchKernelGGL(disk_fill_kernel<float>, grid, TPB, 0, s, f, (float *)state, fl); break;
    default: hipLaunchKernelGGL(disk_fill_kernel<__half>, grid, TPB, 0, s, f, (__half *)state, fl); break;
    }
    return hipGetLastError();
}

}  // namespace fdlbm
