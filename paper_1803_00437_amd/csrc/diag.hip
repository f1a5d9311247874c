// FP64 diagnostics of a state and the conversions between host-staged FP64 planes and the
// device storage dtype.
//
// The reduction is deterministic: a fixed grid of DIAG_BLOCKS blocks walks the nodes with
// a grid-stride loop, each block reduces its threads in a fixed tree (wavefront shuffles,
// then LDS) and writes one partial; a single block then reduces the partials in order.
// Quantities (section 3-a uses the correlation A(t) = <J(t), J0>/<J0, J0>):
//   [0] sum drho, [1] sum jx, [2] sum jy, [3] 1/2 sum |J|^2/rho, [4] max |J|,
//   [5] sum J.J0, [6] sum J0.J0, [7] count of nodes with a non-finite field.
#include <mutex>

#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Reduce DIAG_SLOTS values over the block; thread 0 returns the result in acc.
__device__ void block_reduce(double (&acc)[DIAG_SLOTS])
{
    __shared__ double lds[TPB / 64][DIAG_SLOTS];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < DIAG_SLOTS; ++q) acc[q] = q == 4 ? wave_max(acc[q]) : wave_sum(acc[q]);
    if (lane == 0)
        for (int q = 0; q < DIAG_SLOTS; ++q) lds[wid][q] = acc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < DIAG_SLOTS; ++q) {
            double v = lds[0][q];
            for (int w = 1; w < TPB / 64; ++w) v = q == 4 ? fmax(v, lds[w][q]) : v + lds[w][q];
            acc[q] = v;
        }
    }
}

__device__ __forceinline__ void diag_add(double (&acc)[DIAG_SLOTS], double r, double x, double y,
                                         const double *__restrict__ j0x, const double *__restrict__ j0y, size_t p)
{
    const bool finite = isfinite(r) && isfinite(x) && isfinite(y);
    if (!finite) {
        acc[7] += 1.0;
        return;
    }
    const double j2 = x * x + y * y;
    acc[0] += r;
    acc[1] += x;
    acc[2] += y;
    acc[3] += 0.5 * j2 / (1.0 + r);
    acc[4] = fmax(acc[4], sqrt(j2));
    if (j0x) {
        const double ax = j0x[p], ay = j0y[p];
        acc[5] += x * ax + y * ay;
        acc[6] += ax * ax + ay * ay;
    }
}

// The row-interleaved state, row by row (rows over the blocks, columns over the threads):
// MRT nine populations (pop_elem), FD-LBM / LW-ACM drho, Jx, Jy (fd_elem).  The mode (j0x,
// j0y) is two planes of nx*ny values.
template <typename T, bool MRT>
__global__ void __launch_bounds__(TPB) diag_partials(const T *__restrict__ st, int nx, int ny,
                                                     const double *__restrict__ j0x, const double *__restrict__ j0y,
                                                     double *__restrict__ partials)
{
    double acc[DIAG_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int j = blockIdx.x; j < ny; j += gridDim.x)
        for (int i = threadIdx.x; i < nx; i += TPB) {
            double r, x, y;
            if (MRT) {
                double f[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) f[q] = double(Storage<T>::load(st[pop_elem(i, j, q, nx)]));
                r = (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) + f[8];
                x = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
                y = ((f[2] - f[4]) + (f[5] + f[6])) - (f[7] + f[8]);
            } else {
                r = double(Storage<T>::load(st[fd_elem(i, j, 0, nx)]));
                x = double(Storage<T>::load(st[fd_elem(i, j, 1, nx)]));
                y = double(Storage<T>::load(st[fd_elem(i, j, 2, nx)]));
            }
            diag_add(acc, r, x, y, j0x, j0y, (size_t)j * (size_t)nx + (size_t)i);
        }
    block_reduce(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < DIAG_SLOTS; ++q) partials[blockIdx.x * DIAG_SLOTS + q] = acc[q];
}

__global__ void __launch_bounds__(TPB) diag_final(const double *__restrict__ partials, int nblocks,
                                                  double *__restrict__ out)
{
    double acc[DIAG_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += TPB)
        for (int q = 0; q < DIAG_SLOTS; ++q) {
            const double v = partials[b * DIAG_SLOTS + q];
            acc[q] = q == 4 ? fmax(acc[q], v) : acc[q] + v;
        }
    block_reduce(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < DIAG_SLOTS; ++q) out[q] = acc[q];
}

template <typename T>
__global__ void __launch_bounds__(TPB) pack_kernel(const double *__restrict__ in, T *__restrict__ out, size_t count)
{
    for (size_t p = blockIdx.x * (size_t)TPB + threadIdx.x; p < count; p += (size_t)gridDim.x * TPB)
        out[p] = Storage<T>::store(typename Storage<T>::C(in[p]));
}

template <typename T>
__global__ void __launch_bounds__(TPB) unpack_kernel(const T *__restrict__ in, double *__restrict__ out, size_t count)
{
    for (size_t p = blockIdx.x * (size_t)TPB + threadIdx.x; p < count; p += (size_t)gridDim.x * TPB)
        out[p] = double(Storage<T>::load(in[p]));
}

// Plain streaming copy: one 16-byte access per thread and a grid covering the whole
// buffer, with non-temporal hints (the fastest copy shape measured on MI355X; grid-stride
// loops reached only about two thirds of its bandwidth).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(TPB) copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, size_t n16)
{
    const size_t i = blockIdx.x * (size_t)TPB + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

inline unsigned grid_for(size_t n)
{
    size_t b = (n + TPB - 1) / TPB;
    return (unsigned)(b < 8192 ? (b == 0 ? 1 : b) : 8192);
}

template <typename T>
hipError_t diag_run(bool mrt, const void *state, int nx, int ny, const double *j0x, const double *j0y,
                    double *partials, double *out, hipStream_t s)
{
    const T *st = static_cast<const T *>(state);
    if (mrt)
        hipLaunchKernelGGL((diag_partials<T, true>), DIAG_BLOCKS, TPB, 0, s, st, nx, ny, j0x, j0y, partials);
    else
        hipLaunchKernelGGL((diag_partials<T, false>), DIAG_BLOCKS, TPB, 0, s, st, nx, ny, j0x, j0y, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final, 1, TPB, 0, s, partials, DIAG_BLOCKS, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_diag(int scheme, int dtype, const void *state, int nx, int ny, const double *j0x, const double *j0y,
                       double *partials, double *out, hipStream_t s)
{
    const bool mrt = scheme == FDLBM_SCHEME_MRT;
    switch (dtype) {
    case FDLBM_F64: return diag_run<double>(mrt, state, nx, ny, j0x, j0y, partials, out, s);
    case FDLBM_F32: return diag_run<float>(mrt, state, nx, ny, j0x, j0y, partials, out, s);
    default: return diag_run<__half>(mrt, state, nx, ny, j0x, j0y, partials, out, s);
    }
}

// Allocation-free diagnostics (fdlbm_diagnostics_static) --------------------------------
// The block partials of the reduction live in this file-scope array instead of a caller's
// scratch buffer: 1024 blocks x 8 doubles = 64 KiB, held on every device the library runs
// on until the process ends.  The reduction always uses DIAG_BLOCKS blocks, so the array
// fits every grid.  Host code never passes the array's name to a kernel (in host code it
// is a host-side stand-in): its device address is resolved once per device with
// hipGetSymbolAddress, with that device current, and kept in static_ptr[].
namespace {
static __device__ __align__(256) double scratch[DIAG_BLOCKS * DIAG_SLOTS];
static_assert(sizeof(double) * DIAG_BLOCKS * DIAG_SLOTS == 65536, "the static scratch is the 1024 block partials");

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex static_mu;
double *static_ptr[STATIC_MAX_DEVICES] = {};

hipError_t static_partials(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(static_mu);
    if (!static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        static_ptr[dev] = static_cast<double *>(p);
    }
    *out = static_ptr[dev];
    return hipSuccess;
}
}  // namespace

hipError_t launch_diag_static(int scheme, int dtype, const void *state, int nx, int ny, const double *j0x,
                              const double *j0y, double *out, hipStream_t s)
{
    double *partials = nullptr;
    hipError_t e = static_partials(&partials);
    if (e != hipSuccess) return e;
    // every block writes its own partial, so nothing left by an earlier call is read
    return launch_diag(scheme, dtype, state, nx, ny, j0x, j0y, partials, out, s);
}

// State of NF fields (3: drho, Jx, Jy; 9: the MRT populations): host order (NF planes of
// nx*ny FP64 values) to and from the row-interleaved storage (row_elem); one block row of
// columns per grid row.
template <typename T, int NF>
__global__ void __launch_bounds__(TPB) pack_rows_kernel(const double *__restrict__ in, T *__restrict__ out, int nx,
                                                        int ny)
{
    const size_t n = (size_t)nx * (size_t)ny;
    for (int j = blockIdx.x; j < ny; j += gridDim.x)
        for (int i = threadIdx.x; i < nx; i += TPB)
            for (int f = 0; f < NF; ++f)
                out[row_elem<NF>(i, j, f, nx)] =
                    Storage<T>::store(typename Storage<T>::C(in[f * n + (size_t)j * nx + i]));
}
template <typename T, int NF>
__global__ void __launch_bounds__(TPB) unpack_rows_kernel(const T *__restrict__ in, double *__restrict__ out, int nx,
                                                          int ny)
{
    const size_t n = (size_t)nx * (size_t)ny;
    for (int j = blockIdx.x; j < ny; j += gridDim.x)
        for (int i = threadIdx.x; i < nx; i += TPB)
            for (int f = 0; f < NF; ++f)
                out[f * n + (size_t)j * nx + i] = double(Storage<T>::load(in[row_elem<NF>(i, j, f, nx)]));
}

template <typename T, int NF> void pack_rows_t(bool to_device, const void *in, void *out, int nx, int ny, hipStream_t s)
{
    const unsigned g = (unsigned)(ny < 65536 ? ny : 65536);
    if (to_device)
        hipLaunchKernelGGL((pack_rows_kernel<T, NF>), g, TPB, 0, s, (const double *)in, (T *)out, nx, ny);
    else
        hipLaunchKernelGGL((unpack_rows_kernel<T, NF>), g, TPB, 0, s, (const T *)in, (double *)out, nx, ny);
}
template <int NF> void pack_rows_nf(int dtype, bool to_device, const void *in, void *out, int nx, int ny, hipStream_t s)
{
    switch (dtype) {
    case FDLBM_F64: pack_rows_t<double, NF>(to_device, in, out, nx, ny, s); break;
    case FDLBM_F32: pack_rows_t<float, NF>(to_device, in, out, nx, ny, s); break;
    default: pack_rows_t<__half, NF>(to_device, in, out, nx, ny, s); break;
    }
}

hipError_t launch_pack_rows(int dtype, int nf, const double *in, void *out, int nx, int ny, hipStream_t s)
{
    if (nf == 9)
        pack_rows_nf<9>(dtype, true, in, out, nx, ny, s);
    else
        pack_rows_nf<3>(dtype, true, in, out, nx, ny, s);
    return hipGetLastError();
}

hipError_t launch_unpack_rows(int dtype, int nf, const void *in, double *out, int nx, int ny, hipStream_t s)
{
    if (nf == 9)
        pack_rows_nf<9>(dtype, false, in, out, nx, ny, s);
    else
        pack_rows_nf<3>(dtype, false, in, out, nx, ny, s);
    return hipGetLastError();
}

hipError_t launch_pack(int dtype, const double *in, void *out, size_t count, hipStream_t s)
{
    switch (dtype) {
    case FDLBM_F64: hipLaunchKernelGGL(pack_kernel<double>, grid_for(count), TPB, 0, s, in, (double *)out, count); break;
    case FDLBM_F32: hipLaunchKernelGGL(pack_kernel<float>, grid_for(count), TPB, 0, s, in, (float *)out, count); break;
    default: hipLaunchKernelGGL(pack_kernel<__half>, grid_for(count), TPB, 0, s, in, (__half *)out, count); break;
    }
    return hipGetLastError();
}

hipError_t launch_unpack(int dtype, const void *in, double *out, size_t count, hipStream_t s)
{
    switch (dtype) {
    case FDLBM_F64:
        hipLaunchKernelGGL(unpack_kernel<double>, grid_for(count), TPB, 0, s, (const double *)in, out, count);
        break;
    case FDLBM_F32:
        hipLaunchKernelGGL(unpack_kernel<float>, grid_for(count), TPB, 0, s, (const float *)in, out, count);
        break;
    default:
        hipLaunchKernelGGL(unpack_kernel<__half>, grid_for(count), TPB, 0, s, (const __half *)in, out, count);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_device_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + TPB - 1) / TPB;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, (unsigned)blocks, TPB, 0, s, static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst),
                       n16);
    return hipGetLastError();
}

}  // namespace fdlbm
