// Many independent FD-LBM grids (periodic, 3-point differences) of different sizes and
// viscosities advanced together: one launch per lane class (at most three) per time step
// covers every tile of every instance, and the FP64 correlation A(t) = <J(t), J0> / <J0, J0> of each instance with its
// initial state (section 3-a) is sampled on the device.  A chunk of steps plus one sample
// is captured once in a HIP graph and replayed.
//
// Each block looks up (instance, tile) in a table built on the host and runs the same
// tile body as the single-grid kernel, so every instance evolves exactly as it would
// alone.  Instances are grouped by lane class (vector or per-column accesses, see
// BATCH_CLASSES); each class is one launch.
#include "fd_sweep_body.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {
using namespace sweep;

constexpr int PROJ_TPB = 256;

template <typename T, int CPL, int AM>
__global__ void __launch_bounds__(64 * WV) fd_batch_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                           const BatchInstance *__restrict__ inst,
                                                           const BatchBlock *__restrict__ blocks, int rows)
{
    using C = typename Storage<T>::C;
    const BatchBlock b = blocks[blockIdx.x];
    const BatchInstance I = inst[b.instance];
    TileArgs<T> t;
    t.dr = in + I.offset;
    t.jx = t.dr + I.nx;  // row-interleaved fields (fd_elem)
    t.jy = t.dr + 2 * (size_t)I.nx;
    t.odr = out + I.offset;
    t.ojx = t.odr + I.nx;
    t.ojy = t.odr + 2 * (size_t)I.nx;
    t.nx = I.nx;
    t.ny = I.ny;
    t.rows = rows;
    t.k.eax = C(-2.0 * I.ke / 36.0);
    t.k.edg = C(2.0 * I.ke / 18.0);
    t.k.e0 = C(-2.0 * I.ke / 9.0);
    t.k.kxx = C(I.kxx);
    t.k.kxx2 = C(2.0 * I.kxx);
    t.k.hfx = t.k.hfy = t.k.qfx = t.k.qfy = t.k.dfx = t.k.dfy = C(0);
    const int band = b.tile / I.strips_x;
    const int sx = b.tile - band * I.strips_x;
    sweep_tile<T, CPL, 3, false, false, AM>(t, band, sx * Strip<CPL, 1>::S, sx == I.strips_x - 1);
}

// Single instance in the same tiling: the one-launch-per-grid path of the comparison.
template <typename T, int CPL, int AM>
__global__ void __launch_bounds__(64 * WV) fd_single_kernel(const T *__restrict__ in, T *__restrict__ out,
                                                            const BatchInstance *__restrict__ inst, int i, int rows)
{
    using C = typename Storage<T>::C;
    const BatchInstance I = inst[i];
    TileArgs<T> t;
    t.dr = in + I.offset;
    t.jx = t.dr + I.nx;  // row-interleaved fields (fd_elem)
    t.jy = t.dr + 2 * (size_t)I.nx;
    t.odr = out + I.offset;
    t.ojx = t.odr + I.nx;
    t.ojy = t.odr + 2 * (size_t)I.nx;
    t.nx = I.nx;
    t.ny = I.ny;
    t.rows = rows;
    t.k.eax = C(-2.0 * I.ke / 36.0);
    t.k.edg = C(2.0 * I.ke / 18.0);
    t.k.e0 = C(-2.0 * I.ke / 9.0);
    t.k.kxx = C(I.kxx);
    t.k.kxx2 = C(2.0 * I.kxx);
    t.k.hfx = t.k.hfy = t.k.qfx = t.k.qfy = t.k.dfx = t.k.dfy = C(0);
    const int band = blockIdx.x / I.strips_x;
    const int sx = blockIdx.x - band * I.strips_x;
    sweep_tile<T, CPL, 3, false, false, AM>(t, band, sx * Strip<CPL, 1>::S, sx == I.strips_x - 1);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Partial sums of J.J0 and J0.J0 over one chunk of one instance (FP64, fixed order).
template <typename T>
__global__ void __launch_bounds__(PROJ_TPB) proj_partials(const T *__restrict__ state, const T *__restrict__ mode,
                                                          const BatchInstance *__restrict__ inst,
                                                          const BatchChunk *__restrict__ chunks,
                                                          double *__restrict__ partials)
{
    __shared__ double lds[PROJ_TPB / 64][2];
    const BatchChunk ch = chunks[blockIdx.x];
    const BatchInstance I = inst[ch.instance];
    const size_t n = (size_t)I.nx * (size_t)I.ny;
    const size_t p0 = (size_t)ch.chunk * BATCH_CHUNK, p1 = p0 + BATCH_CHUNK < n ? p0 + BATCH_CHUNK : n;
    const T *st = state + I.offset;
    const T *mx = mode + I.mode_offset, *my = mx + n;  // the mode: two planes
    const unsigned nx = (unsigned)I.nx;
    double num = 0.0, den = 0.0;
    for (size_t p = p0 + threadIdx.x; p < p1; p += PROJ_TPB) {
        const unsigned j = (unsigned)p / nx, i = (unsigned)p - j * nx;  // an instance has < 2^32 nodes
        const double ax = double(Storage<T>::load(mx[p])), ay = double(Storage<T>::load(my[p]));
        num += double(Storage<T>::load(st[fd_elem(i, j, 1, nx)])) * ax + double(Storage<T>::load(st[fd_elem(i, j, 2, nx)])) * ay;
        den += ax * ax + ay * ay;
    }
    num = wave_sum(num);
    den = wave_sum(den);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        lds[w][0] = num;
        lds[w][1] = den;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < PROJ_TPB / 64; ++k) {
            a += lds[k][0];
            b += lds[k][1];
        }
        partials[2 * blockIdx.x] = a;
        partials[2 * blockIdx.x + 1] = b;
    }
}

// A = sum num / sum den per instance, written to sample slot *counter (dropped once the
// slots are full).
__global__ void proj_final(const BatchInstance *__restrict__ inst, int count, const double *__restrict__ partials,
                           const int *__restrict__ counter, int max_samples, double *__restrict__ amps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int s = *counter;
    if (s >= max_samples) return;
    const BatchInstance I = inst[i];
    double num = 0.0, den = 0.0;
    for (int c = 0; c < I.nchunks; ++c) {
        num += partials[2 * (I.first_chunk + c)];
        den += partials[2 * (I.first_chunk + c) + 1];
    }
    amps[(size_t)i * max_samples + s] = den > 0.0 ? num / den : 0.0;
}

__global__ void advance_counter(int *counter) { *counter += 1; }

template <typename T, int CPL, int AM>
hipError_t step_class(const BatchLaunch &L, int c, const void *src, void *dst, hipStream_t s)
{
    if (L.class_blocks[c] == 0) return hipSuccess;
    hipLaunchKernelGGL((fd_batch_kernel<T, CPL, AM>), L.class_blocks[c], 64 * WV, 0, s, static_cast<const T *>(src),
                       static_cast<T *>(dst), L.inst, L.blocks + L.class_begin[c], L.rows);
    return hipGetLastError();
}

template <typename T>
hipError_t step_all(const BatchLaunch &L, const void *src, void *dst, hipStream_t s)
{
    constexpr int W = sizeof(T) == 8 ? 2 : 4;
    constexpr int AM2 = sizeof(T) >= 4 ? AM_UNAL : AM_COL;  // class 2: any width
    hipError_t e = step_class<T, W, AM_VEC>(L, 0, src, dst, s);
    if constexpr (W == 4)
        if (e == hipSuccess) e = step_class<T, 2, AM_VEC>(L, 1, src, dst, s);
    if (e == hipSuccess) e = step_class<T, W, AM2>(L, 2, src, dst, s);
    return e;
}

template <typename T>
hipError_t step_one(const BatchLaunch &L, int i, int cls, int nblocks, const void *src, void *dst, hipStream_t s)
{
    constexpr int W = sizeof(T) == 8 ? 2 : 4;
    constexpr int AM2 = sizeof(T) >= 4 ? AM_UNAL : AM_COL;
    const T *in = static_cast<const T *>(src);
    T *out = static_cast<T *>(dst);
    if (cls == 0)
        hipLaunchKernelGGL((fd_single_kernel<T, W, AM_VEC>), nblocks, 64 * WV, 0, s, in, out, L.inst, i, L.rows);
    else if (cls == 1)
        hipLaunchKernelGGL((fd_single_kernel<T, 2, AM_VEC>), nblocks, 64 * WV, 0, s, in, out, L.inst, i, L.rows);
    else
        hipLaunchKernelGGL((fd_single_kernel<T, W, AM2>), nblocks, 64 * WV, 0, s, in, out, L.inst, i, L.rows);
    return hipGetLastError();
}

template <typename T> hipError_t sample(const BatchLaunch &L, const void *state, hipStream_t s)
{
    hipLaunchKernelGGL(proj_partials<T>, L.nchunks, PROJ_TPB, 0, s, static_cast<const T *>(state),
                       static_cast<const T *>(L.mode), L.inst, L.chunks, L.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(proj_final, (L.count + 255) / 256, 256, 0, s, L.inst, L.count, L.partials, L.counter,
                       L.max_samples, L.amps);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(advance_counter, 1, 1, 0, s, L.counter);
    return hipGetLastError();
}

}  // namespace

int batch_strip_stride(int cpl) { return cpl == 4 ? Strip<4, 1>::S : cpl == 2 ? Strip<2, 1>::S : Strip<1, 1>::S; }
int batch_rows_per_block(int rows) { return WV * rows; }

hipError_t launch_batch_step(const BatchLaunch &L, const void *src, void *dst, hipStream_t s)
{
    switch (L.dtype) {
    case FDLBM_F64: return step_all<double>(L, src, dst, s);
    case FDLBM_F32: return step_all<float>(L, src, dst, s);
    default: return step_all<__half>(L, src, dst, s);
    }
}

hipError_t launch_batch_single(const BatchLaunch &L, int i, int cls, int nblocks, const void *src, void *dst,
                               hipStream_t s)
{
    switch (L.dtype) {
    case FDLBM_F64: return step_one<double>(L, i, cls, nblocks, src, dst, s);
    case FDLBM_F32: return step_one<float>(L, i, cls, nblocks, src, dst, s);
    default: return step_one<__half>(L, i, cls, nblocks, src, dst, s);
    }
}

hipError_t launch_batch_sample(const BatchLaunch &L, const void *state, hipStream_t s)
{
    switch (L.dtype) {
    case FDLBM_F64: return sample<double>(L, state, s);
    case FDLBM_F32: return sample<float>(L, state, s);
    default: return sample<__half>(L, state, s);
    }
}

}  // namespace fdlbm
