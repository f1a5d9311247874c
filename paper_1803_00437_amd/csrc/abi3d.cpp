// C ABI of the D3Q19 FD-LBM step (declarations and contracts in include/fdlbm3d.h).
// Host code only: validation, scratch layout and stream-ordered launches of fd3d.hip.
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "fdlbm3d.h"
#include "internal.hpp"

using namespace fdlbm;

namespace {

thread_local char g_err3[512] = "";

int device_error3(hipError_t e, const char *what)
{
    std::snprintf(g_err3, sizeof g_err3, "%s: %s", what, hipGetErrorString(e));
    return FDLBM_EDEVICE;
}

#define HIPCHK3(call, what)                                   \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return device_error3(e_, what); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
bool rate_ok(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

constexpr int DIAG3_SLOTS = 8;

struct Layout3 {
    size_t staging, partials, out, fstar, total;
};

// default tile (measured at 512^3): FP32 12 rows x 64 planes (86 000 MLUPS), FP64 12 rows x 32
// planes (43 600)
int tile_rows(const fdlbm3d_params &p) { return p.tile_rows != 0 ? p.tile_rows : 12; }
int tile_planes(const fdlbm3d_params &p) { return p.tile_planes != 0 ? p.tile_planes : p.dtype == FDLBM_F64 ? 32 : 64; }
size_t nodes(const fdlbm3d_params &p) { return (size_t)p.nx * (size_t)p.ny * (size_t)p.nz; }
size_t elem(const fdlbm3d_params &p) { return p.dtype == FDLBM_F64 ? 8 : 4; }

int validate3(const fdlbm3d_params *p)
{
    if (!p) return FDLBM_EINVAL;
    for (int v : {p->nx, p->ny, p->nz})
        if (v < 3 || v > (1 << 20)) return FDLBM_EINVAL;
    if (nodes(*p) >= (size_t(1) << 40)) return FDLBM_EINVAL;
    if (p->dtype != FDLBM_F64 && p->dtype != FDLBM_F32) return FDLBM_EINVAL;
    // the sweep kernel addresses a field plane through a buffer resource whose size and
    // per-lane offsets are 32-bit byte counts: one plane must stay below 2^31 bytes
    if ((size_t)p->nx * (size_t)p->ny * elem(*p) >= (size_t(1) << 31)) return FDLBM_EINVAL;
    if (!rate_ok(p->s_nu) || !rate_ok(p->s_e)) return FDLBM_EINVAL;
    if (p->kernel != FDLBM_KERNEL_AUTO && p->kernel != FDLBM_KERNEL_REFERENCE && p->kernel != FDLBM_KERNEL_SWEEP)
        return FDLBM_EINVAL;
    if (p->tile_rows != 0 && p->tile_rows != 8 && p->tile_rows != 12 && p->tile_rows != 16) return FDLBM_EINVAL;
    if (p->tile_planes < 0 || p->tile_planes > 4096) return FDLBM_EINVAL;
    const Dim3Grid g = d3_sweep_grid(p->nx, p->ny, p->nz, tile_rows(*p), tile_planes(*p));
    if (g.y > 65535 || g.z > 65535) return FDLBM_EINVAL;
    return FDLBM_OK;
}

Layout3 layout3(const fdlbm3d_params &p)
{
    Layout3 L{};
    const size_t n = nodes(p);
    size_t o = 0;
    L.staging = o;
    o += align256(4 * n * sizeof(double));
    L.partials = o;
    o += align256((size_t)d3_diag_blocks(n) * DIAG3_SLOTS * sizeof(double));
    L.out = o;
    o += align256(DIAG3_SLOTS * sizeof(double));
    L.fstar = o;
    if (p.kernel == FDLBM_KERNEL_REFERENCE) o += align256(18 * n * elem(p));
    L.total = o;
    return L;
}

}  // namespace

struct fdlbm3d_ctx {
    fdlbm3d_params p{};
    Layout3 L{};
    void *buf[2] = {nullptr, nullptr};
    char *scratch = nullptr;
    hipStream_t stream = nullptr;
    int device = 0;
    int cur = 0;
    int64_t steps = 0;
    double *sd(size_t off) const { return reinterpret_cast<double *>(scratch + off); }
};

extern "C" {

int fdlbm3d_workspace_bytes(const fdlbm3d_params *p, size_t *state_bytes, size_t *scratch_bytes)
{
    const int v = validate3(p);
    if (v != FDLBM_OK) return v;
    if (state_bytes) *state_bytes = align256(4 * nodes(*p) * elem(*p));
    if (scratch_bytes) *scratch_bytes = layout3(*p).total;
    return FDLBM_OK;
}

int fdlbm3d_create(const fdlbm3d_params *p, void *state_a, void *state_b, void *scratch, size_t scratch_bytes,
                   void *hip_stream, fdlbm3d_ctx **out)
{
    if (!out) return FDLBM_EINVAL;
    *out = nullptr;
    const int v = validate3(p);
    if (v != FDLBM_OK) return v;
    if (!state_a || !state_b || !scratch || state_a == state_b) return FDLBM_EINVAL;
    for (const void *b : {state_a, state_b, scratch})
        if ((reinterpret_cast<uintptr_t>(b) & 255) != 0) return FDLBM_EINVAL;
    const Layout3 L = layout3(*p);
    if (scratch_bytes < L.total) return FDLBM_ENOMEM;
    fdlbm3d_ctx *c = new (std::nothrow) fdlbm3d_ctx;
    if (!c) return FDLBM_ENOMEM;
    c->p = *p;
    c->L = L;
    c->buf[0] = state_a;
    c->buf[1] = state_b;
    c->scratch = static_cast<char *>(scratch);
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMemsetAsync(state_a, 0, align256(4 * nodes(*p) * elem(*p)), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return device_error3(e, "fdlbm3d_create");
    }
    *out = c;
    return FDLBM_OK;
}

void fdlbm3d_destroy(fdlbm3d_ctx *c) { delete c; }

int64_t fdlbm3d_step_count(const fdlbm3d_ctx *c) { return c ? c->steps : -1; }

int fdlbm3d_set_state(fdlbm3d_ctx *c, const double *drho, const double *jx, const double *jy, const double *jz)
{
    if (!c || !drho || !jx || !jy || !jz) return FDLBM_EINVAL;
    HIPCHK3(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = nodes(c->p), nb = n * sizeof(double);
    double *st = c->sd(c->L.staging);
    const double *src[4] = {drho, jx, jy, jz};
    for (int f = 0; f < 4; ++f)
        HIPCHK3(hipMemcpyAsync(st + f * n, src[f], nb, hipMemcpyHostToDevice, c->stream), "set_state upload");
    HIPCHK3(launch_pack(c->p.dtype, st, c->buf[c->cur], 4 * n, c->stream), "pack");
    HIPCHK3(hipStreamSynchronize(c->stream), "set_state");
    c->steps = 0;
    return FDLBM_OK;
}

int fdlbm3d_get_state(fdlbm3d_ctx *c, double *drho, double *jx, double *jy, double *jz)
{
    if (!c || !drho || !jx || !jy || !jz) return FDLBM_EINVAL;
    HIPCHK3(hipSetDevice(c->device), "hipSetDevice");
    const size_t n = nodes(c->p), nb = n * sizeof(double);
    double *st = c->sd(c->L.staging);
    HIPCHK3(launch_unpack(c->p.dtype, c->buf[c->cur], st, 4 * n, c->stream), "unpack");
    double *dst[4] = {drho, jx, jy, jz};
    for (int f = 0; f < 4; ++f)
        HIPCHK3(hipMemcpyAsync(dst[f], st + f * n, nb, hipMemcpyDeviceToHost, c->stream), "get_state download");
    HIPCHK3(hipStreamSynchronize(c->stream), "get_state");
    return FDLBM_OK;
}

int fdlbm3d_step(fdlbm3d_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 0) return FDLBM_EINVAL;
    HIPCHK3(hipSetDevice(c->device), "hipSetDevice");
    const fdlbm3d_params &p = c->p;
    for (int64_t s = 0; s < nsteps; ++s) {
        const void *in = c->buf[c->cur];
        void *out = c->buf[1 - c->cur];
        if (p.kernel == FDLBM_KERNEL_REFERENCE)
            HIPCHK3(launch_d3_reference(p.dtype, in, out, c->scratch + c->L.fstar, p.nx, p.ny, p.nz, p.s_nu, p.s_e,
                                        c->stream),
                    "d3 reference step");
        else
            HIPCHK3(launch_d3_sweep(p.dtype, in, out, p.nx, p.ny, p.nz, p.s_nu, p.s_e, tile_rows(p), tile_planes(p),
                                    c->stream),
                    "d3 sweep step");
        c->cur = 1 - c->cur;
        ++c->steps;
    }
    return FDLBM_OK;
}

int fdlbm3d_diagnostics(fdlbm3d_ctx *c, fdlbm3d_diag *out)
{
    if (!c || !out) return FDLBM_EINVAL;
    HIPCHK3(hipSetDevice(c->device), "hipSetDevice");
    double h[DIAG3_SLOTS];
    HIPCHK3(launch_d3_diagnostics(c->p.dtype, c->buf[c->cur], nodes(c->p), c->sd(c->L.partials), c->sd(c->L.out),
                                  c->stream),
            "d3 diagnostics");
    HIPCHK3(hipMemcpyAsync(h, c->sd(c->L.out), sizeof h, hipMemcpyDeviceToHost, c->stream), "diagnostics download");
    HIPCHK3(hipStreamSynchronize(c->stream), "diagnostics");
    out->mass = h[0];
    out->mom_x = h[1];
    out->mom_y = h[2];
    out->mom_z = h[3];
    out->kin_energy = h[4];
    out->max_abs_j = h[5];
    out->nonfinite = (int64_t)h[6];
    return FDLBM_OK;
}

int fdlbm3d_autotune(fdlbm3d_ctx *c, int32_t reps, int32_t *out_rows, int32_t *out_planes, double *out_ms)
{
    if (!c || reps < 1 || reps > 10000) return FDLBM_EINVAL;
    HIPCHK3(hipSetDevice(c->device), "hipSetDevice");
    fdlbm3d_params &p = c->p;
    struct Shape {
        int rows, planes;
    };
    std::vector<Shape> cand;
    if (p.kernel == FDLBM_KERNEL_REFERENCE) {
        cand.push_back({p.tile_rows, p.tile_planes});
    } else {
        for (int rows : {8, 12, 16})
            for (int planes : {16, 32, 64, 128}) {
                const Dim3Grid g = d3_sweep_grid(p.nx, p.ny, p.nz, rows, planes);
                if (g.y <= 65535 && g.z <= 65535) cand.push_back({rows, planes});
            }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // every timed launch reads the current state and writes the spare buffer, which the next
    // step overwrites: the state does not advance
    const void *src = c->buf[c->cur];
    void *dst = c->buf[1 - c->cur];
    auto launch = [&](const Shape &sh) -> hipError_t {
        if (p.kernel == FDLBM_KERNEL_REFERENCE)
            return launch_d3_reference(p.dtype, src, dst, c->scratch + c->L.fstar, p.nx, p.ny, p.nz, p.s_nu, p.s_e,
                                       c->stream);
        return launch_d3_sweep(p.dtype, src, dst, p.nx, p.ny, p.nz, p.s_nu, p.s_e, sh.rows, sh.planes, c->stream);
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
    if (e != hipSuccess) return device_error3(e, "fdlbm3d_autotune");
    if (p.kernel != FDLBM_KERNEL_REFERENCE) {
        p.tile_rows = best.rows;
        p.tile_planes = best.planes;
    }
    if (out_rows) *out_rows = tile_rows(p);
    if (out_planes) *out_planes = tile_planes(p);
    if (out_ms) *out_ms = (double)best_ms / reps;
    return FDLBM_OK;
}

const char *fdlbm3d_last_error(void) { return g_err3; }

}  // extern "C"
