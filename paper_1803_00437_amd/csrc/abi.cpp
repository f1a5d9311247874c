// C ABI of the FD-LBM / MRT D2Q9 library (declarations and contracts in include/fdlbm.h).
// Host code only: validation, scratch layout, stream-ordered launches of the kernels in
// the other translation units, and FP64 host <-> device staging.
#include <cmath>
#include <vector>
#include <cstdio>
#include <cstring>
#include <new>

#include "fdlbm_device.hpp"
#include "internal.hpp"

using namespace fdlbm;

namespace {

thread_local char g_err[512] = "";

int device_error(hipError_t e, const char *what)
{
    std::snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return FDLBM_EDEVICE;
}

#define HIPCHK(call, what)                                 \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return device_error(e_, what); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool rate_ok(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

// rows per wavefront (FD-LBM sweep) or per tile (MRT sweep): beyond this a tile is taller
// than any grid the kernels' index arithmetic is sized for
constexpr int MAX_TILE_ROWS = 1024;

double quartic(double s_xx) { return 1.0 / (0.5 + 1.0 / (6.0 * (1.0 / s_xx - 0.5))); }

struct Layout {
    size_t partials, out, mode, staging, fstar;
    size_t disk_dst, disk_src, disk_w, disk_span, disk_ring;  // ghost-node table (FDLBM_BC_DISK)
    size_t mdisk_node, mdisk_kb, mdisk_q, mdisk_ring, mdisk_fspan;  // MRT boundary links (FDLBM_BC_DISK)
    size_t total;
};

// FD-LBM and LW-ACM store (drho, Jx, Jy) and run on the FD-LBM kernels; MRT stores populations
bool three_words(int scheme) { return scheme != FDLBM_SCHEME_MRT; }

// distance of the walls beyond the first and last rows (0 selects 1/2)
double wall_xi(const fdlbm_params &p) { return p.wall_xi == 0.0 ? 0.5 : p.wall_xi; }

FdArgs fd_args(const fdlbm_params &p)
{
    const int stencil = p.scheme == FDLBM_SCHEME_LWACM ? LWACM_STENCIL : p.stencil;
    return FdArgs{p.nx, p.ny, stencil, p.bc == FDLBM_BC_WALLS_Y ? 1 : 0, p.dtype, p.s_xx, p.s_e, p.force_x, p.force_y,
                  wall_xi(p)};
}

// the disk's ghost-node table; false if the disk does not fit (checked by validate)
bool disk_table(const fdlbm_params &p, DiskTable *t)
{
    return build_disk_table(p.nx, p.ny, p.disk_cx, p.disk_cy, p.disk_r, t);
}

bool uses_reference(const fdlbm_params &p)
{
    if (!three_words(p.scheme)) return false;
    if (p.kernel == FDLBM_KERNEL_REFERENCE) return true;
    return !fd_sweep_supported(fd_args(p), p.lane_cols);
}

int validate(const fdlbm_params *p)
{
    if (!p) return FDLBM_EINVAL;
    if (p->scheme != FDLBM_SCHEME_FD && p->scheme != FDLBM_SCHEME_MRT && p->scheme != FDLBM_SCHEME_LWACM)
        return FDLBM_EINVAL;
    if (p->bc != FDLBM_BC_PERIODIC && p->bc != FDLBM_BC_WALLS_Y && p->bc != FDLBM_BC_DISK) return FDLBM_EINVAL;
    if (p->nx < 8 || p->nx > (1 << 20)) return FDLBM_EINVAL;
    if (p->ny < (p->bc == FDLBM_BC_WALLS_Y ? 4 : 8) || p->ny > (1 << 20)) return FDLBM_EINVAL;
    if ((size_t)p->nx * (size_t)p->ny > (size_t(1) << 32)) return FDLBM_EINVAL;
    if (!rate_ok(p->s_xx) || !rate_ok(p->s_e)) return FDLBM_EINVAL;
    if (!std::isfinite(p->force_x) || !std::isfinite(p->force_y)) return FDLBM_EINVAL;
    if (p->bc == FDLBM_BC_WALLS_Y && !(wall_xi(*p) > 0.0 && wall_xi(*p) <= 1.0)) return FDLBM_EINVAL;
    if (p->kernel < FDLBM_KERNEL_AUTO || p->kernel > FDLBM_KERNEL_SWEEP) return FDLBM_EINVAL;
    if (p->tile_rows < 0 || p->tile_rows > MAX_TILE_ROWS || p->check_every < 0) return FDLBM_EINVAL;
    if (three_words(p->scheme)) {
        if (p->scheme == FDLBM_SCHEME_FD && p->stencil != 3 && p->stencil != 5)
            return FDLBM_EINVAL;  // the 9-point form is unstable on {1,1}
        if (p->scheme == FDLBM_SCHEME_LWACM &&
            (p->bc == FDLBM_BC_WALLS_Y || p->force_x != 0.0 || p->force_y != 0.0))
            return FDLBM_EINVAL;  // section 1-b: a periodic step without force (the disk only adds ghost nodes)
        if (p->bc == FDLBM_BC_DISK) {
            DiskTable t;
            if (!disk_table(*p, &t)) return FDLBM_EINVAL;
        }
        if (p->dtype != FDLBM_F64 && p->dtype != FDLBM_F32 && !is_f16(p->dtype)) return FDLBM_EINVAL;
        if (p->lane_cols != 0 && p->lane_cols != 1 && p->lane_cols != 2 && p->lane_cols != 4) return FDLBM_EINVAL;
        if (p->kernel == FDLBM_KERNEL_SWEEP && !fd_sweep_supported(fd_args(*p), p->lane_cols)) return FDLBM_EINVAL;
    } else {
        if (p->bc == FDLBM_BC_DISK) {
            DiskTable t;
            if (!disk_table(*p, &t)) return FDLBM_EINVAL;
        }
        if (p->dtype != FDLBM_F64 && p->dtype != FDLBM_F32) return FDLBM_EINVAL;
        if (!rate_ok(p->s_eps)) return FDLBM_EINVAL;
        if (!p->quartic && !rate_ok(p->s_q)) return FDLBM_EINVAL;
    }
    return FDLBM_OK;
}

Layout layout(const fdlbm_params &p)
{
    const size_t n = (size_t)p.nx * (size_t)p.ny;
    Layout L;
    size_t off = 0;
    L.partials = off;
    off += align256(sizeof(double) * DIAG_BLOCKS * DIAG_SLOTS);
    L.out = off;
    off += align256(sizeof(double) * DIAG_SLOTS);
    L.mode = off;
    off += align256(sizeof(double) * 2 * n);
    // staging (set/get) and the reference path's f* planes are never live at once
    const size_t staging = align256(sizeof(double) * (p.scheme == FDLBM_SCHEME_MRT ? 9 : 3) * n);
    const size_t fstar = uses_reference(p) ? align256(fd_reference_scratch_bytes(fd_args(p))) : 0;
    L.staging = off;
    L.fstar = off;
    off += staging > fstar ? staging : fstar;
    size_t ng = 0, nr = 0, nl = 0, nsr = 0;
    const bool mrt_disk = p.bc == FDLBM_BC_DISK && !three_words(p.scheme);
    if (p.bc == FDLBM_BC_DISK) {
        DiskTable t;
        if (disk_table(p, &t)) {
            ng = three_words(p.scheme) ? t.dst.size() : 0;
            nr = three_words(p.scheme) ? t.ring.size() : 0;
            nl = mrt_disk ? t.link_node.size() : 0;
            nsr = mrt_disk ? t.solid_ring.size() : 0;
        }
    }
    L.disk_dst = off;
    off += align256(sizeof(int32_t) * ng);
    L.disk_src = off;
    off += align256(sizeof(int32_t) * ng);
    L.disk_w = off;
    off += align256(sizeof(double) * 3 * ng);
    L.disk_span = off;
    off += p.bc == FDLBM_BC_DISK && three_words(p.scheme) ? align256(sizeof(int32_t) * 2 * size_t(p.ny)) : 0;
    L.disk_ring = off;
    off += align256(sizeof(int32_t) * nr);
    L.mdisk_node = off;
    off += align256(sizeof(int32_t) * nl);
    L.mdisk_kb = off;
    off += align256(sizeof(int32_t) * nl);
    L.mdisk_q = off;
    off += align256(sizeof(double) * nl);
    L.mdisk_ring = off;
    off += align256(sizeof(int32_t) * nsr);
    L.mdisk_fspan = off;
    off += mrt_disk ? align256(sizeof(int32_t) * 2 * size_t(p.ny)) : 0;
    L.total = off;
    return L;
}

// Runs an entry point's body so that no C++ exception crosses the C ABI: host allocation
// failure (std::bad_alloc from the tables) becomes FDLBM_ENOMEM, anything else FDLBM_EINVAL.
template <typename Body> int guarded(Body &&body)
{
    try {
        return body();
    } catch (const std::bad_alloc &) {
        return FDLBM_ENOMEM;
    } catch (...) {
        return FDLBM_EINVAL;
    }
}

}  // namespace

struct fdlbm_ctx {
    fdlbm_params p;
    double s_q;  // effective MRT s_q
    int device;
    char *buf[2];
    int cur;
    char *scratch;
    Layout L;
    hipStream_t stream;
    int64_t steps;
    bool mode_set;
    DiskFill disk;   // FDLBM_BC_DISK: the ghost-node table in the scratch buffer
    MrtDisk mdisk;   // FDLBM_BC_DISK, MRT: the boundary-link table in the scratch buffer
    bool disk_full;  // the next fill sets every rest node to rest (the state was just set)

    size_t n() const { return (size_t)p.nx * (size_t)p.ny; }
    double *sd(size_t off) const { return reinterpret_cast<double *>(scratch + off); }
};

extern "C" {

int fdlbm_workspace_bytes(const fdlbm_params *p, size_t *state_bytes, size_t *scratch_bytes)
{
    return guarded([&]() -> int {
        int rc = validate(p);
        if (rc) return rc;
        const size_t n = (size_t)p->nx * (size_t)p->ny;
        if (state_bytes) *state_bytes = align256((p->scheme == FDLBM_SCHEME_MRT ? 9 : 3) * n * dtype_bytes(p->dtype));
        if (scratch_bytes) *scratch_bytes = layout(*p).total;
        return FDLBM_OK;
    });
}

int fdlbm_create(const fdlbm_params *p, void *state_a, void *state_b, void *scratch, size_t scratch_bytes,
                 void *hip_stream, fdlbm_ctx **out)
{
    return guarded([&]() -> int {
        int rc = validate(p);
        if (rc) return rc;
        if (!out || !state_a || !state_b || !scratch || state_a == state_b) return FDLBM_EINVAL;
        if (((uintptr_t)state_a | (uintptr_t)state_b | (uintptr_t)scratch) & 255) return FDLBM_EINVAL;
        Layout L = layout(*p);
        if (scratch_bytes < L.total) return FDLBM_ENOMEM;
        fdlbm_ctx *c = new (std::nothrow) fdlbm_ctx;
        if (!c) return FDLBM_ENOMEM;
        c->p = *p;
        c->s_q = p->scheme == FDLBM_SCHEME_MRT && p->quartic ? quartic(p->s_xx) : p->s_q;
        c->buf[0] = static_cast<char *>(state_a);
        c->buf[1] = static_cast<char *>(state_b);
        c->cur = 0;
        c->scratch = static_cast<char *>(scratch);
        c->L = L;
        c->stream = static_cast<hipStream_t>(hip_stream);
        c->steps = 0;
        c->mode_set = false;
        c->disk = DiskFill{p->nx, p->ny, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
        c->mdisk = MrtDisk{p->nx, p->ny, 0, 0, nullptr, nullptr, nullptr, nullptr, nullptr};
        c->disk_full = true;
        hipError_t e = hipGetDevice(&c->device);
        size_t sb = 0;
        fdlbm_workspace_bytes(p, &sb, nullptr);
        if (e == hipSuccess) e = hipMemsetAsync(state_a, 0, sb, c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(state_b, 0, sb, c->stream);
        DiskTable t;  // outlives the uploads: the stream is synchronised below
        if (e == hipSuccess && p->bc == FDLBM_BC_DISK && !three_words(p->scheme)) {
            if (!disk_table(*p, &t)) {
                delete c;
                return FDLBM_EINVAL;
            }
            char *sc = c->scratch;
            const size_t nl = t.link_node.size(), nsr = t.solid_ring.size();
            c->mdisk.nlinks = int(nl);
            c->mdisk.nring = int(nsr);
            c->mdisk.node = reinterpret_cast<const int32_t *>(sc + L.mdisk_node);
            c->mdisk.kb = reinterpret_cast<const int32_t *>(sc + L.mdisk_kb);
            c->mdisk.q = reinterpret_cast<const double *>(sc + L.mdisk_q);
            c->mdisk.ring = reinterpret_cast<const int32_t *>(sc + L.mdisk_ring);
            c->mdisk.fspan = reinterpret_cast<const int32_t *>(sc + L.mdisk_fspan);
            if (nl) e = hipMemcpyAsync(sc + L.mdisk_node, t.link_node.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice,
                                       c->stream);
            if (e == hipSuccess && nl)
                e = hipMemcpyAsync(sc + L.mdisk_kb, t.link_kb.data(), nl * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess && nl)
                e = hipMemcpyAsync(sc + L.mdisk_q, t.link_q.data(), nl * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess && nsr)
                e = hipMemcpyAsync(sc + L.mdisk_ring, t.solid_ring.data(), nsr * sizeof(int32_t), hipMemcpyHostToDevice,
                                   c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sc + L.mdisk_fspan, t.fspan.data(), t.fspan.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, c->stream);
        } else if (e == hipSuccess && p->bc == FDLBM_BC_DISK) {
            if (!disk_table(*p, &t)) {
                delete c;
                return FDLBM_EINVAL;
            }
            char *sc = c->scratch;
            c->disk.nghost = int(t.dst.size());
            c->disk.dst = reinterpret_cast<const int32_t *>(sc + L.disk_dst);
            c->disk.src = reinterpret_cast<const int32_t *>(sc + L.disk_src);
            c->disk.w = reinterpret_cast<const double *>(sc + L.disk_w);
            c->disk.span = reinterpret_cast<const int32_t *>(sc + L.disk_span);
            c->disk.nring = int(t.ring.size());
            c->disk.ring = reinterpret_cast<const int32_t *>(sc + L.disk_ring);
            const size_t ng = t.dst.size(), nr = t.ring.size();
            if (ng) e = hipMemcpyAsync(sc + L.disk_dst, t.dst.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess && ng)
                e = hipMemcpyAsync(sc + L.disk_src, t.src.data(), ng * sizeof(int32_t), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess && ng)
                e = hipMemcpyAsync(sc + L.disk_w, t.w.data(), 3 * ng * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(sc + L.disk_span, t.span.data(), t.span.size() * sizeof(int32_t),
                                   hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess && nr)
                e = hipMemcpyAsync(sc + L.disk_ring, t.ring.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice,
                                   c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) {
            delete c;
            return device_error(e, "fdlbm_create");
        }
        *out = c;
        return FDLBM_OK;
    });
}

void fdlbm_destroy(fdlbm_ctx *c) { delete c; }

int64_t fdlbm_step_count(const fdlbm_ctx *c) { return c ? c->steps : -1; }

int fdlbm_set_step_count(fdlbm_ctx *c, int64_t steps)
{
    if (!c || steps < 0) return FDLBM_EINVAL;
    c->steps = steps;
    return FDLBM_OK;
}

int fdlbm_set_state(fdlbm_ctx *c, const double *drho, const double *jx, const double *jy)
{
    if (!c || !drho || !jx || !jy) return FDLBM_EINVAL;
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n(), nb = n * sizeof(double);
    double *st = c->sd(c->L.staging);
    HIPCHK(hipMemcpyAsync(st, drho, nb, hipMemcpyHostToDevice, c->stream), "set_state upload");
    HIPCHK(hipMemcpyAsync(st + n, jx, nb, hipMemcpyHostToDevice, c->stream), "set_state upload");
    HIPCHK(hipMemcpyAsync(st + 2 * n, jy, nb, hipMemcpyHostToDevice, c->stream), "set_state upload");
    if (three_words(c->p.scheme))
        HIPCHK(launch_pack_rows(c->p.dtype, 3, st, c->buf[c->cur], c->p.nx, c->p.ny, c->stream), "pack");
    else
        HIPCHK(launch_mrt_init(c->p.dtype, st, st + n, st + 2 * n, c->buf[c->cur], c->p.nx, c->p.ny, c->stream), "mrt_init");
    HIPCHK(hipStreamSynchronize(c->stream), "set_state");
    c->steps = 0;
    c->disk_full = true;
    return FDLBM_OK;
}

int fdlbm_get_state(fdlbm_ctx *c, double *drho, double *jx, double *jy)
{
    if (!c || !drho || !jx || !jy) return FDLBM_EINVAL;
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n(), nb = n * sizeof(double);
    double *st = c->sd(c->L.staging);
    if (three_words(c->p.scheme))
        HIPCHK(launch_unpack_rows(c->p.dtype, 3, c->buf[c->cur], st, c->p.nx, c->p.ny, c->stream), "unpack");
    else
        HIPCHK(launch_mrt_moments(c->p.dtype, c->buf[c->cur], st, st + n, st + 2 * n, c->p.nx, c->p.ny, c->stream), "mrt_moments");
    HIPCHK(hipMemcpyAsync(drho, st, nb, hipMemcpyDeviceToHost, c->stream), "get_state download");
    HIPCHK(hipMemcpyAsync(jx, st + n, nb, hipMemcpyDeviceToHost, c->stream), "get_state download");
    HIPCHK(hipMemcpyAsync(jy, st + 2 * n, nb, hipMemcpyDeviceToHost, c->stream), "get_state download");
    HIPCHK(hipStreamSynchronize(c->stream), "get_state");
    return FDLBM_OK;
}

int fdlbm_set_populations(fdlbm_ctx *c, const double *df)
{
    if (!c || !df || c->p.scheme != FDLBM_SCHEME_MRT) return FDLBM_EINVAL;
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n();
    double *st = c->sd(c->L.staging);
    HIPCHK(hipMemcpyAsync(st, df, 9 * n * sizeof(double), hipMemcpyHostToDevice, c->stream), "set_populations");
    HIPCHK(launch_pack_rows(c->p.dtype, 9, st, c->buf[c->cur], c->p.nx, c->p.ny, c->stream), "pack");
    HIPCHK(hipStreamSynchronize(c->stream), "set_populations");
    c->steps = 0;
    c->disk_full = true;
    return FDLBM_OK;
}

int fdlbm_get_populations(fdlbm_ctx *c, double *df)
{
    if (!c || !df || c->p.scheme != FDLBM_SCHEME_MRT) return FDLBM_EINVAL;
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n();
    double *st = c->sd(c->L.staging);
    HIPCHK(launch_unpack_rows(c->p.dtype, 9, c->buf[c->cur], st, c->p.nx, c->p.ny, c->stream), "unpack");
    HIPCHK(hipMemcpyAsync(df, st, 9 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "get_populations");
    HIPCHK(hipStreamSynchronize(c->stream), "get_populations");
    return FDLBM_OK;
}

static int run_diag(fdlbm_ctx *c, double out[DIAG_SLOTS])
{
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n();
    const double *m = c->mode_set ? c->sd(c->L.mode) : nullptr;
    HIPCHK(launch_diag(c->p.scheme, c->p.dtype, c->buf[c->cur], c->p.nx, c->p.ny, m, m ? m + n : nullptr,
                       c->sd(c->L.partials), c->sd(c->L.out), c->stream),
           "diagnostics");
    HIPCHK(hipMemcpyAsync(out, c->sd(c->L.out), DIAG_SLOTS * sizeof(double), hipMemcpyDeviceToHost, c->stream),
           "diagnostics download");
    HIPCHK(hipStreamSynchronize(c->stream), "diagnostics");
    return FDLBM_OK;
}

static int advance(fdlbm_ctx *c, int64_t nsteps)
{
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const bool fd = three_words(c->p.scheme);
    const bool ref = uses_reference(c->p);
    FdArgs fa = fd_args(c->p);
    const MrtArgs ma{c->p.nx, c->p.ny, c->p.bc == FDLBM_BC_WALLS_Y ? 1 : 0, c->p.dtype, c->p.s_e, c->p.s_xx, c->s_q,
                     c->p.s_eps, c->p.force_x, c->p.force_y, c->p.kernel, c->p.tile_rows, wall_xi(c->p)};
    for (int64_t s = 0; s < nsteps; ++s) {
        // stochastic rounding draws fresh bits every step, reproducibly from the step count
        fa.seed = pcg_hash(uint32_t(c->steps));
        void *src = c->buf[c->cur], *dst = c->buf[c->cur ^ 1];
        // the curved wall: ghost and rest nodes from the fluid, in place, before the step;
        // every rest node after the state was set or under a body force (which moves the
        // rest nodes too), else only the ring the previous step could reach
        const bool disk_full = c->disk_full || c->p.force_x != 0.0 || c->p.force_y != 0.0;
        if (c->p.bc == FDLBM_BC_DISK && fd) {
            HIPCHK(launch_disk_fill(c->disk, c->p.dtype, src, disk_full, c->stream), "disk fill launch");
            c->disk_full = false;
        }
        hipError_t e;
        if (!fd)
            e = launch_mrt(ma, src, dst, c->stream);
        else if (ref)
            e = launch_fd_reference(fa, src, dst, c->scratch + c->L.fstar, c->stream);
        else
            e = launch_fd_sweep(fa, c->p.tile_rows, c->p.lane_cols, src, dst, c->stream);
        if (e != hipSuccess)
            return device_error(e, c->p.scheme == FDLBM_SCHEME_FD    ? "fdlbm_step launch"
                                   : c->p.scheme == FDLBM_SCHEME_MRT ? "mrt_step launch"
                                                                      : "lwacm_step launch");
        // MRT in the disk: the wall acts on the streamed populations, after the step; the
        // solid nodes the links reach go back to rest (every solid node after the state was
        // set or under a body force)
        if (c->p.bc == FDLBM_BC_DISK && !fd) {
            HIPCHK(launch_mrt_disk(c->mdisk, c->p.dtype, dst, disk_full, c->stream), "mrt disk launch");
            c->disk_full = false;
        }
        c->cur ^= 1;
        ++c->steps;
        if (c->p.check_every > 0 && c->steps % c->p.check_every == 0) {
            double d[DIAG_SLOTS];
            int rc = run_diag(c, d);
            if (rc) return rc;
            if (d[7] > 0) return FDLBM_EUNSTABLE;
        }
    }
    return FDLBM_OK;
}

int fdlbm_step(fdlbm_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0 || c->p.scheme != FDLBM_SCHEME_FD) return FDLBM_EINVAL;
    return advance(c, nsteps);
}

int mrt_step(fdlbm_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0 || c->p.scheme != FDLBM_SCHEME_MRT) return FDLBM_EINVAL;
    return advance(c, nsteps);
}

int lwacm_step(fdlbm_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0 || c->p.scheme != FDLBM_SCHEME_LWACM) return FDLBM_EINVAL;
    return advance(c, nsteps);
}

int fdlbm_diagnostics(fdlbm_ctx *c, fdlbm_diag *out)
{
    if (!c || !out) return FDLBM_EINVAL;
    double d[DIAG_SLOTS];
    int rc = run_diag(c, d);
    if (rc) return rc;
    out->mass = d[0];
    out->mom_x = d[1];
    out->mom_y = d[2];
    out->kin_energy = d[3];
    out->max_abs_j = d[4];
    out->proj_num = d[5];
    out->proj_den = d[6];
    out->nonfinite = (int64_t)d[7];
    return FDLBM_OK;
}

int fdlbm_diagnostics_static(const fdlbm_params *p, const void *state, const double *j0x, const double *j0y,
                             void *hip_stream, double *out)
{
    return guarded([&]() -> int {
        int rc = validate(p);
        if (rc) return rc;
        if (!state || !out || (j0x == nullptr) != (j0y == nullptr)) return FDLBM_EINVAL;
        HIPCHK(launch_diag_static(p->scheme, p->dtype, state, p->nx, p->ny, j0x, j0y, out,
                                  static_cast<hipStream_t>(hip_stream)),
               "fdlbm_diagnostics_static");
        return FDLBM_OK;
    });
}

int fdlbm_set_mode(fdlbm_ctx *c, const double *j0x, const double *j0y)
{
    if (!c || !j0x || !j0y) return FDLBM_EINVAL;
    HIPCHK(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = c->n();
    double *m = c->sd(c->L.mode);
    HIPCHK(hipMemcpyAsync(m, j0x, n * sizeof(double), hipMemcpyHostToDevice, c->stream), "set_mode");
    HIPCHK(hipMemcpyAsync(m + n, j0y, n * sizeof(double), hipMemcpyHostToDevice, c->stream), "set_mode");
    HIPCHK(hipStreamSynchronize(c->stream), "set_mode");
    c->mode_set = true;
    return FDLBM_OK;
}

int fdlbm_mode_projection(fdlbm_ctx *c, double *out)
{
    if (!c || !out || !c->mode_set) return FDLBM_EINVAL;
    double d[DIAG_SLOTS];
    int rc = run_diag(c, d);
    if (rc) return rc;
    if (!(d[6] > 0)) return FDLBM_EINVAL;
    *out = d[5] / d[6];
    return FDLBM_OK;
}

int fdlbm_autotune(fdlbm_ctx *c, int32_t reps, int32_t *out_lane_cols, int32_t *out_tile_rows, double *out_ms)
{
    return guarded([&]() -> int {
        if (!c || reps < 1 || reps > 10000) return FDLBM_EINVAL;
        HIPCHK(hipSetDevice(c->device), "hipSetDevice");
        const bool fd = three_words(c->p.scheme);
        const FdArgs fa = fd_args(c->p);
        const bool ref = fd ? uses_reference(c->p) : c->p.kernel == FDLBM_KERNEL_REFERENCE;
        // candidate shapes: (lane_cols, tile_rows); the reference kernels have none to choose
        struct Shape {
            int cols, rows;
        };
        std::vector<Shape> cand;
        if (ref) {
            cand.push_back({c->p.lane_cols, c->p.tile_rows});
        } else if (fd) {
            for (int cols : {1, 2, 4})
                if (fd_sweep_supported(fa, cols))
                    for (int rows : {4, 6, 8, 12, 16, 24}) cand.push_back({cols, rows});
        } else {
            for (int rows : {1, 2, 4, 8, 16}) cand.push_back({0, rows});
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        // every timed launch reads the current state and writes the spare buffer, which the
        // next step overwrites: the state does not advance
        void *src = c->buf[c->cur], *dst = c->buf[c->cur ^ 1];
        auto launch = [&](const Shape &sh) -> hipError_t {
            if (fd && ref) return launch_fd_reference(fa, src, dst, c->scratch + c->L.fstar, c->stream);
            if (fd) return launch_fd_sweep(fa, sh.rows, sh.cols, src, dst, c->stream);
            const MrtArgs ma{c->p.nx, c->p.ny, c->p.bc == FDLBM_BC_WALLS_Y ? 1 : 0, c->p.dtype, c->p.s_e, c->p.s_xx, c->s_q,
                             c->p.s_eps, c->p.force_x, c->p.force_y, c->p.kernel, sh.rows, wall_xi(c->p)};
            return launch_mrt(ma, src, dst, c->stream);
        };
        Shape best{0, 0};
        float best_ms = 0.0f;
        for (const Shape &sh : cand) {
            if (e == hipSuccess) e = launch(sh);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(sh);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            if (best_ms == 0.0f || ms < best_ms) {
                best_ms = ms;
                best = sh;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (e != hipSuccess) return device_error(e, "fdlbm_autotune");
        if (!ref) {
            c->p.lane_cols = best.cols;
            c->p.tile_rows = best.rows;
        }
        if (out_lane_cols) *out_lane_cols = best.cols;
        if (out_tile_rows) *out_tile_rows = best.rows;
        if (out_ms) *out_ms = (double)best_ms / reps;
        return FDLBM_OK;
    });
}

int fdlbm_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) & 15) return FDLBM_EINVAL;
    HIPCHK(launch_device_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream)), "fdlbm_device_copy");
    return FDLBM_OK;
}

const char *fdlbm_strerror(int code)
{
    switch (code) {
    case FDLBM_OK: return "ok";
    case FDLBM_EINVAL: return "invalid argument";
    case FDLBM_ENOMEM: return "buffer smaller than fdlbm_workspace_bytes requires";
    case FDLBM_EDEVICE: return "HIP runtime error (see fdlbm_last_error)";
    case FDLBM_EUNSTABLE: return "non-finite value in the state";
    default: return "unknown error";
    }
}

const char *fdlbm_last_error(void) { return g_err; }

double fdlbm_rate_from_viscosity(double nu) { return 1.0 / (0.5 + 3.0 * nu); }

double fdlbm_quartic_s_q(double s_xx) { return quartic(s_xx); }

}  // extern "C"
