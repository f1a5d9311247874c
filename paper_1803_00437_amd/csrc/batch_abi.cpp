// C ABI of the batched FD-LBM path (declarations and contracts in include/fdlbm.h):
// layout of many independent grids in two caller-owned state buffers, the tile and chunk
// tables, stream-ordered launches, and the HIP graphs that replay a chunk of steps plus
// one A(t) sample.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "internal.hpp"

using namespace fdlbm;

namespace {

thread_local char g_berr[512] = "";

int batch_device_error(hipError_t e, const char *what)
{
    std::snprintf(g_berr, sizeof g_berr, "%s: %s", what, hipGetErrorString(e));
    return FDLBM_EDEVICE;
}

#define BHIPCHK(call, what)                                        \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess) return batch_device_error(e_, what); \
    } while (0)

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
size_t al64(size_t x) { return (x + 63) & ~size_t(63); }
bool rate_in_range(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

constexpr int BATCH_ROWS = 8;               // rows per wavefront unless tuned
constexpr int BATCH_TUNE_ROWS[] = {4, 6, 8, 12, 16};  // candidates of fdlbm_batch_autotune
constexpr int BATCH_MIN_ROWS = 4;           // the block table is sized for the smallest

struct Plan {
    std::vector<BatchInstance> inst;
    std::vector<BatchBlock> blocks;
    std::vector<BatchChunk> chunks;
    int class_begin[BATCH_CLASSES] = {}, class_blocks[BATCH_CLASSES] = {};
    size_t state_elems = 0, mode_elems = 0, max_n = 0;
    // scratch offsets (bytes)
    size_t o_inst, o_blocks, o_chunks, o_partials, o_counter, o_amps, o_mode, o_staging, total;
};

int validate(const fdlbm_instance *in, int32_t count, int32_t dtype, int32_t max_samples)
{
    if (!in || count < 1 || count > (1 << 20) || max_samples < 0) return FDLBM_EINVAL;
    if (dtype != FDLBM_F64 && dtype != FDLBM_F32 && dtype != FDLBM_F16DEV) return FDLBM_EINVAL;
    for (int i = 0; i < count; ++i) {
        if (in[i].nx < 8 || in[i].ny < 8 || in[i].nx > (1 << 16) || in[i].ny > (1 << 16)) return FDLBM_EINVAL;
        if (!rate_in_range(in[i].s_xx) || !rate_in_range(in[i].s_e)) return FDLBM_EINVAL;
    }
    return FDLBM_OK;
}

// Lane class of an instance (BATCH_CLASSES): aligned vector accesses of the widest lane
// group where its width allows; else FP16 at even widths keeps aligned accesses of two
// columns, and every other width takes class 2 (measured on the 512-instance workload:
// FP32 2 mod 4 widths are faster in class 2 than at two columns per lane).
int instance_class(int nx, int dtype)
{
    const int w = dtype == FDLBM_F64 ? 2 : 4;
    if (nx % w == 0) return 0;
    if (dtype == FDLBM_F16DEV && nx % 2 == 0) return 1;
    return 2;
}

// Tiles of every instance for `rows` rows per wavefront: the instances' band counts and
// the block table, grouped by lane-group class (one launch each) and, within a class,
// largest grids first so that the last blocks to start are small ones.
void tile_tables(Plan &P, int rows)
{
    const int RB = batch_rows_per_block(rows);
    for (BatchInstance &I : P.inst) I.nbands = (I.ny + RB - 1) / RB;
    const int count = (int)P.inst.size();
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const BatchInstance &A = P.inst[a], &B = P.inst[b];
        if (A.cls != B.cls) return A.cls < B.cls;
        return (size_t)A.nx * A.ny > (size_t)B.nx * B.ny;
    });
    P.blocks.clear();
    for (int c = 0; c < BATCH_CLASSES; ++c) P.class_blocks[c] = 0;
    for (int i : order) {
        const int tiles = P.inst[i].strips_x * P.inst[i].nbands;
        P.class_blocks[P.inst[i].cls] += tiles;
        for (int t = 0; t < tiles; ++t) P.blocks.push_back(BatchBlock{i, t});
    }
    for (int c = 0, begin = 0; c < BATCH_CLASSES; ++c) {
        P.class_begin[c] = begin;
        begin += P.class_blocks[c];
    }
}

// Point a launch description at the block table the plan holds.
void use_tables(BatchLaunch &L, const Plan &P, int rows)
{
    L.rows = rows;
    L.nblocks = (int)P.blocks.size();
    for (int c = 0; c < BATCH_CLASSES; ++c) {
        L.class_begin[c] = P.class_begin[c];
        L.class_blocks[c] = P.class_blocks[c];
    }
}

Plan plan(const fdlbm_instance *in, int32_t count, int32_t dtype, int32_t max_samples)
{
    Plan P;
    P.inst.resize(count);
    int chunk0 = 0;
    for (int i = 0; i < count; ++i) {
        BatchInstance &I = P.inst[i];
        const size_t n = (size_t)in[i].nx * (size_t)in[i].ny;
        I.offset = P.state_elems;
        P.state_elems = al64(P.state_elems + 3 * n);
        I.mode_offset = P.mode_elems;
        P.mode_elems = al64(P.mode_elems + 2 * n);
        I.nx = in[i].nx;
        I.ny = in[i].ny;
        I.cls = instance_class(I.nx, dtype);
        const int S = batch_strip_stride(batch_class_cpl(I.cls, dtype));
        I.strips_x = (I.nx + S - 1) / S;
        I.first_chunk = chunk0;
        I.nchunks = (int)((n + BATCH_CHUNK - 1) / BATCH_CHUNK);
        chunk0 += I.nchunks;
        I.ke = 0.5 * (1.0 - 1.0 / in[i].s_e);
        I.kxx = 0.5 * (1.0 - 1.0 / in[i].s_xx);
        P.max_n = std::max(P.max_n, n);
        for (int c = 0; c < I.nchunks; ++c) P.chunks.push_back(BatchChunk{i, c});
    }
    // the block table is sized for the smallest tile height a tuning run may choose
    tile_tables(P, BATCH_MIN_ROWS);
    const size_t max_blocks = P.blocks.size();
    tile_tables(P, BATCH_ROWS);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += al256(bytes);
        return o;
    };
    P.o_inst = take(sizeof(BatchInstance) * P.inst.size());
    P.o_blocks = take(sizeof(BatchBlock) * max_blocks);
    P.o_chunks = take(sizeof(BatchChunk) * P.chunks.size());
    P.o_partials = take(2 * sizeof(double) * P.chunks.size());
    P.o_counter = take(sizeof(int));
    P.o_amps = take(sizeof(double) * (size_t)count * (size_t)std::max(max_samples, 1));
    P.o_mode = take(dtype_bytes(dtype) * P.mode_elems);
    P.o_staging = take(3 * sizeof(double) * P.max_n);
    P.total = off;
    return P;
}

struct GraphEntry {
    int sample_every, parity;
    hipGraphExec_t exec;
};

}  // namespace

struct fdlbm_batch {
    Plan P;
    int dtype, count, max_samples, device;
    hipStream_t stream;
    char *buf[2];
    int cur;
    char *scratch;
    BatchLaunch L;
    int64_t steps;
    std::vector<GraphEntry> graphs;
};

namespace {

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

int launch_chunk(fdlbm_batch *b, int steps, bool sample)
{
    for (int s = 0; s < steps; ++s) {
        BHIPCHK(launch_batch_step(b->L, b->buf[b->cur], b->buf[b->cur ^ 1], b->stream), "batch step launch");
        b->cur ^= 1;
    }
    if (sample) BHIPCHK(launch_batch_sample(b->L, b->buf[b->cur], b->stream), "batch sample launch");
    return FDLBM_OK;
}

}  // namespace

extern "C" {

int fdlbm_batch_workspace_bytes(const fdlbm_instance *instances, int32_t count, int32_t dtype, int32_t max_samples,
                                size_t *state_bytes, size_t *scratch_bytes)
{
    return guarded([&]() -> int {
        int rc = validate(instances, count, dtype, max_samples);
        if (rc) return rc;
        Plan P = plan(instances, count, dtype, max_samples);
        if (state_bytes) *state_bytes = al256(P.state_elems * dtype_bytes(dtype));
        if (scratch_bytes) *scratch_bytes = P.total;
        return FDLBM_OK;
    });
}

int fdlbm_batch_create(const fdlbm_instance *instances, int32_t count, int32_t dtype, int32_t max_samples,
                       void *state_a, void *state_b, void *scratch, size_t scratch_bytes, void *hip_stream,
                       fdlbm_batch **out)
{
    return guarded([&]() -> int {
        int rc = validate(instances, count, dtype, max_samples);
        if (rc) return rc;
        if (!out || !state_a || !state_b || !scratch || state_a == state_b) return FDLBM_EINVAL;
        if (((uintptr_t)state_a | (uintptr_t)state_b | (uintptr_t)scratch) & 255) return FDLBM_EINVAL;
        fdlbm_batch *b = new (std::nothrow) fdlbm_batch;
        if (!b) return FDLBM_ENOMEM;
        b->P = plan(instances, count, dtype, max_samples);
        if (scratch_bytes < b->P.total) {
            delete b;
            return FDLBM_ENOMEM;
        }
        b->dtype = dtype;
        b->count = count;
        b->max_samples = max_samples;
        b->stream = static_cast<hipStream_t>(hip_stream);
        b->buf[0] = static_cast<char *>(state_a);
        b->buf[1] = static_cast<char *>(state_b);
        b->cur = 0;
        b->scratch = static_cast<char *>(scratch);
        b->steps = 0;
        const Plan &P = b->P;
        BatchLaunch &L = b->L;
        L.dtype = dtype;
        L.count = count;
        use_tables(L, P, BATCH_ROWS);
        L.nchunks = (int)P.chunks.size();
        L.max_samples = max_samples;
        L.inst = reinterpret_cast<const BatchInstance *>(b->scratch + P.o_inst);
        L.blocks = reinterpret_cast<const BatchBlock *>(b->scratch + P.o_blocks);
        L.chunks = reinterpret_cast<const BatchChunk *>(b->scratch + P.o_chunks);
        L.mode = b->scratch + P.o_mode;
        L.partials = reinterpret_cast<double *>(b->scratch + P.o_partials);
        L.counter = reinterpret_cast<int *>(b->scratch + P.o_counter);
        L.amps = reinterpret_cast<double *>(b->scratch + P.o_amps);
        hipError_t e = hipGetDevice(&b->device);
        const size_t sb = al256(P.state_elems * dtype_bytes(dtype));
        if (e == hipSuccess) e = hipMemcpyAsync(b->scratch + P.o_inst, P.inst.data(), sizeof(BatchInstance) * P.inst.size(),
                                                hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b->scratch + P.o_blocks, P.blocks.data(), sizeof(BatchBlock) * P.blocks.size(),
                                                hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(b->scratch + P.o_chunks, P.chunks.data(), sizeof(BatchChunk) * P.chunks.size(),
                                                hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(state_a, 0, sb, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(state_b, 0, sb, b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->scratch + P.o_counter, 0, sizeof(int), b->stream);
        if (e == hipSuccess) e = hipMemsetAsync(b->scratch + P.o_mode, 0, dtype_bytes(dtype) * P.mode_elems, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) {
            delete b;
            return batch_device_error(e, "fdlbm_batch_create");
        }
        *out = b;
        return FDLBM_OK;
    });
}

void fdlbm_batch_destroy(fdlbm_batch *b)
{
    if (!b) return;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    delete b;
}

int fdlbm_batch_set_state(fdlbm_batch *b, int32_t i, const double *drho, const double *jx, const double *jy)
{
    if (!b || i < 0 || i >= b->count || !drho || !jx || !jy) return FDLBM_EINVAL;
    BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
    const BatchInstance &I = b->P.inst[i];
    const size_t n = (size_t)I.nx * (size_t)I.ny, nb = n * sizeof(double), db = dtype_bytes(b->dtype);
    double *st = reinterpret_cast<double *>(b->scratch + b->P.o_staging);
    BHIPCHK(hipMemcpyAsync(st, drho, nb, hipMemcpyHostToDevice, b->stream), "batch set_state upload");
    BHIPCHK(hipMemcpyAsync(st + n, jx, nb, hipMemcpyHostToDevice, b->stream), "batch set_state upload");
    BHIPCHK(hipMemcpyAsync(st + 2 * n, jy, nb, hipMemcpyHostToDevice, b->stream), "batch set_state upload");
    BHIPCHK(launch_pack_rows(b->dtype, 3, st, b->buf[b->cur] + I.offset * db, I.nx, I.ny, b->stream), "batch pack");
    // the correlation reference J0 is this state's momentum, as stored
    BHIPCHK(launch_pack(b->dtype, st + n, b->scratch + b->P.o_mode + I.mode_offset * db, 2 * n, b->stream),
            "batch pack mode");
    BHIPCHK(hipMemsetAsync(b->L.counter, 0, sizeof(int), b->stream), "batch reset samples");
    BHIPCHK(hipStreamSynchronize(b->stream), "batch set_state");
    b->steps = 0;
    return FDLBM_OK;
}

int fdlbm_batch_get_state(fdlbm_batch *b, int32_t i, double *drho, double *jx, double *jy)
{
    if (!b || i < 0 || i >= b->count || !drho || !jx || !jy) return FDLBM_EINVAL;
    BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
    const BatchInstance &I = b->P.inst[i];
    const size_t n = (size_t)I.nx * (size_t)I.ny, nb = n * sizeof(double), db = dtype_bytes(b->dtype);
    double *st = reinterpret_cast<double *>(b->scratch + b->P.o_staging);
    BHIPCHK(launch_unpack_rows(b->dtype, 3, b->buf[b->cur] + I.offset * db, st, I.nx, I.ny, b->stream), "batch unpack");
    BHIPCHK(hipMemcpyAsync(drho, st, nb, hipMemcpyDeviceToHost, b->stream), "batch get_state download");
    BHIPCHK(hipMemcpyAsync(jx, st + n, nb, hipMemcpyDeviceToHost, b->stream), "batch get_state download");
    BHIPCHK(hipMemcpyAsync(jy, st + 2 * n, nb, hipMemcpyDeviceToHost, b->stream), "batch get_state download");
    BHIPCHK(hipStreamSynchronize(b->stream), "batch get_state");
    return FDLBM_OK;
}

int fdlbm_batch_autotune(fdlbm_batch *b, int32_t reps, int32_t *out_rows, double *out_ms)
{
    return guarded([&]() -> int {
        if (!b || reps < 1 || reps > 10000) return FDLBM_EINVAL;
        BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
        // upload the tile tables for `rows` rows per wavefront and point the launch at them
        auto use_rows = [&](int rows) -> hipError_t {
            tile_tables(b->P, rows);
            hipError_t e = hipMemcpyAsync(b->scratch + b->P.o_inst, b->P.inst.data(),
                                          sizeof(BatchInstance) * b->P.inst.size(), hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->scratch + b->P.o_blocks, b->P.blocks.data(), sizeof(BatchBlock) * b->P.blocks.size(),
                                   hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
            use_tables(b->L, b->P, rows);
            return e;
        };
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        // timed launches read the current state and write the spare buffer: no step is taken
        void *src = b->buf[b->cur], *dst = b->buf[b->cur ^ 1];
        int best = b->L.rows;
        float best_ms = 0.0f;
        for (int rows : BATCH_TUNE_ROWS) {
            if (e == hipSuccess) e = use_rows(rows);
            if (e == hipSuccess) e = launch_batch_step(b->L, src, dst, b->stream);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch_step(b->L, src, dst, b->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            if (best_ms == 0.0f || ms < best_ms) {
                best_ms = ms;
                best = rows;
            }
        }
        if (e == hipSuccess) e = use_rows(best);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        // replays captured before hold the old grid size
        for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.exec);
        b->graphs.clear();
        if (e != hipSuccess) return batch_device_error(e, "fdlbm_batch_autotune");
        if (out_rows) *out_rows = best;
        if (out_ms) *out_ms = (double)best_ms / reps;
        return FDLBM_OK;
    });
}

int fdlbm_batch_step(fdlbm_batch *b, int64_t nsteps, int32_t sample_every, int32_t use_graph)
{
    return guarded([&]() -> int {
        if (!b || nsteps < 0 || sample_every < 0) return FDLBM_EINVAL;
        if (sample_every > 0 && nsteps % sample_every) return FDLBM_EINVAL;
        if (use_graph && (sample_every == 0 || !b->stream)) return FDLBM_EINVAL;  // capture needs a non-default stream
        BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
        if (sample_every == 0) {
            int rc = launch_chunk(b, (int)nsteps, false);
            if (rc) return rc;
            b->steps += nsteps;
            return FDLBM_OK;
        }
        for (int64_t done = 0; done < nsteps; done += sample_every) {
            if (!use_graph) {
                int rc = launch_chunk(b, sample_every, true);
                if (rc) return rc;
                continue;
            }
            hipGraphExec_t exec = nullptr;
            for (auto &g : b->graphs)
                if (g.sample_every == sample_every && g.parity == b->cur) exec = g.exec;
            if (!exec) {
                const int cur0 = b->cur;
                hipGraph_t graph = nullptr;
                BHIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "batch graph capture");
                int rc = launch_chunk(b, sample_every, true);
                hipError_t e = hipStreamEndCapture(b->stream, &graph);
                if (rc) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return rc;
                }
                if (e != hipSuccess) return batch_device_error(e, "batch graph capture");
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return batch_device_error(e, "batch graph instantiate");
                b->graphs.push_back(GraphEntry{sample_every, cur0, exec});
                b->cur = cur0;  // capture recorded the launches without running them
            }
            BHIPCHK(hipGraphLaunch(exec, b->stream), "batch graph launch");
            b->cur ^= (sample_every & 1);
        }
        b->steps += nsteps;
        return FDLBM_OK;
    });
}

int fdlbm_batch_step_per_instance(fdlbm_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return FDLBM_EINVAL;
    BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int i = 0; i < b->count; ++i) {
            const BatchInstance &I = b->P.inst[i];
            BHIPCHK(launch_batch_single(b->L, i, I.cls, I.strips_x * I.nbands, b->buf[b->cur], b->buf[b->cur ^ 1],
                                        b->stream),
                    "batch single launch");
        }
        b->cur ^= 1;
    }
    b->steps += nsteps;
    return FDLBM_OK;
}

int fdlbm_batch_amplitudes(fdlbm_batch *b, double *out, int32_t *nsamples)
{
    if (!b || !nsamples) return FDLBM_EINVAL;
    BHIPCHK(hipSetDevice(b->device), "hipSetDevice");
    int counter = 0;
    BHIPCHK(hipMemcpyAsync(&counter, b->L.counter, sizeof(int), hipMemcpyDeviceToHost, b->stream), "batch samples");
    BHIPCHK(hipStreamSynchronize(b->stream), "batch samples");
    const int n = std::min(counter, b->max_samples);
    *nsamples = n;
    if (out && b->max_samples > 0)
        BHIPCHK(hipMemcpyAsync(out, b->L.amps, sizeof(double) * (size_t)b->count * b->max_samples,
                               hipMemcpyDeviceToHost, b->stream),
                "batch amplitudes");
    BHIPCHK(hipStreamSynchronize(b->stream), "batch amplitudes");
    return FDLBM_OK;
}

int64_t fdlbm_batch_step_count(const fdlbm_batch *b) { return b ? b->steps : -1; }

const char *fdlbm_batch_last_error(void) { return g_berr; }

}  // extern "C"
