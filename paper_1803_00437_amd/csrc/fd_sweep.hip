// FD-LBM step, fused sweep path: one kernel per time step, state read once and written
// once (3 values per node each way), no scratch memory.
//
// Mapping (designed for CDNA4's 64-wide wavefronts):
//   * a wavefront owns a strip of W = 64*CPL consecutive columns (CPL columns per lane,
//     loaded and stored as one vector per field) and walks down R rows of the grid;
//   * x-neighbours of a lane's outer columns come from the adjacent lanes through DPP
//     whole-wave shifts (wave_shl:1 / wave_shr:1), so no LDS and no barrier is needed;
//     the PAD outermost columns on each side of the strip only feed their neighbours, and
//     strips overlap by 2*PAD columns;
//   * y-neighbours live in a rolling window of 2h+1 input rows held in registers (h = 1
//     for 3-point and 2 for 5-point differences); the row loop is unrolled by the window
//     length so the window rotates by renaming, not by register moves;
//   * the post-collision populations of a row are exchanged along x with the same DPP
//     shifts and split into the parts that land on the row itself, on the row above and
//     on the row below; the row below's output is complete once the current row is done.
// Per node the arithmetic is fd_node_fstar() and the summation order is fd_gather()'s, so
// the result equals the reference path bit for bit.
//
// Walls (rows -1 .. -(h+1) and ny .. ny+h are ghosts): the mirror of section 3-c's
// xi = 1/2 extrapolation is applied when a row is loaded (drho even, J odd).
#include "fdlbm_device.hpp"
#include "internal.hpp"

namespace fdlbm {
namespace {

constexpr int WAVES_PER_BLOCK = 4;

// whole-wave lane shifts: shl gives lane i the value of lane i+1, shr the value of lane i-1
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL> __device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double lane_shift(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <typename C> __device__ __forceinline__ C from_right(C v) { return lane_shift<DPP_WAVE_SHL1>(v); }
template <typename C> __device__ __forceinline__ C from_left(C v) { return lane_shift<DPP_WAVE_SHR1>(v); }

// CPL consecutive stored values as one memory access.
template <typename T, int CPL> struct Group {
    T v[CPL];
};

template <typename T, int CPL> __device__ __forceinline__ Group<T, CPL> load_group(const T *p)
{
    static_assert(sizeof(Group<T, CPL>) == sizeof(T) * CPL, "packed group");
    return *reinterpret_cast<const Group<T, CPL> *>(p);
}

template <typename T, int CPL> __device__ __forceinline__ void store_group(T *p, const Group<T, CPL> &g)
{
    *reinterpret_cast<Group<T, CPL> *>(p) = g;
}

template <typename T> struct SweepArgs {
    const T *dr, *jx, *jy;
    T *odr, *ojx, *ojy;
    int nx, ny, rows, strips_x, strips_y, ntiles;
    FdCoef<typename Storage<T>::C> k;
};

template <typename T, int CPL, int ST, bool WALLS>
__global__ void __launch_bounds__(64 * WAVES_PER_BLOCK) fd_sweep_kernel(SweepArgs<T> a)
{
    using C = typename Storage<T>::C;
    using S = Stencil<ST>;
    constexpr int H = S::H;
    constexpr int NW = 2 * H + 1;                           // rows in the input window
    constexpr int W = 64 * CPL;                             // columns per strip
    constexpr int PAD = ((H + 1 + CPL - 1) / CPL) * CPL;    // halo columns per side
    constexpr int SX = W - 2 * PAD;                         // output columns per strip
    static_assert(CPL >= 2 || H == 1, "5-point differences need two columns per lane");

    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;  // uniform over the wavefront
    // consecutive tiles are stacked in y so that a wavefront's halo rows were just read
    // by its neighbour
    const int sx = tile / a.strips_y, sy = tile - sx * a.strips_y;
    const int nx = a.nx, ny = a.ny;
    const int xs = sx * SX - PAD + CPL * lane;              // first column of this lane (unwrapped)
    const int col = ((xs % nx) + nx) % nx;                  // wrapped (x periodic)
    const bool store_ok = lane >= PAD / CPL && lane < (W - PAD) / CPL && xs < nx;
    const int ybeg = sy * a.rows;
    const int yend = min(ybeg + a.rows, ny);
    const int nf = yend - ybeg + 2;                         // rows whose f* is needed: ybeg-1 .. yend
    const int row0 = ybeg - 1 - H;                          // first input row

    // source row and sign for input row j (wave-uniform)
    auto source = [&](int j, int &src, C &sgn) {
        sgn = C(1);
        if (WALLS) {
            if (j < 0) { src = -1 - j; sgn = C(-1); }
            else if (j >= ny) { src = 2 * ny - 1 - j; sgn = C(-1); }
            else src = j;
        } else {
            src = ((j % ny) + ny) % ny;
        }
    };

    // rolling window of input rows; fields: 0 drho, 1 J_a,x, 2 J_a,y (J_a = J + F/2),
    // 3 Jx^2, 4 JxJy, 5 Jy^2 (products of J_a)
    C w[6][NW][CPL];
    Group<T, CPL> pr, px, py;  // prefetched row (raw storage)
    C psg = C(1);              // its sign (-1 for a ghost row beyond a wall)

    auto fetch = [&](int j) {
        int src;
        source(j, src, psg);
        const size_t off = (size_t)src * (size_t)nx + (size_t)col;
        pr = load_group<T, CPL>(a.dr + off);
        px = load_group<T, CPL>(a.jx + off);
        py = load_group<T, CPL>(a.jy + off);
    };
    auto insert = [&](int slot) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const C r = Storage<T>::load(pr.v[c]);
            const C x = fmac(psg, Storage<T>::load(px.v[c]), a.k.hfx);
            const C y = fmac(psg, Storage<T>::load(py.v[c]), a.k.hfy);
            w[0][slot][c] = r;
            w[1][slot][c] = x;
            w[2][slot][c] = y;
            w[3][slot][c] = x * x;
            w[4][slot][c] = x * y;
            w[5][slot][c] = y * y;
        }
    };

    // prologue: the first 2H input rows, and the prefetch of the next one
#pragma unroll
    for (int q = 0; q < 2 * H; ++q) {
        fetch(row0 + q);
        insert(q);
    }
    fetch(row0 + 2 * H);

    // partial sums carried between rows (order of fd_gather): A = cen(r-1) + up(r-2),
    // AX = cenx(r-1) + upx(r-2), UP = up(r-2); UPp, UPXp = up(r-1), upx(r-1)
    C A[CPL], AX[CPL], UP[CPL], UPp[CPL], UPXp[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) A[c] = AX[c] = UP[c] = UPp[c] = UPXp[c] = C(0);

    // x-derivative fields (drho, Jx, Jy, Jx^2, JxJy) -> d[0], d[2], d[4], d[6], d[8];
    // y-derivative fields (drho, Jy, Jx, JxJy, Jy^2) -> d[1], d[3], d[5], d[7], d[9]
    constexpr int XF[5] = {0, 1, 2, 3, 4};
    constexpr int YF[5] = {0, 2, 1, 4, 5};

    for (int it0 = 0; it0 < nf; it0 += NW) {
#pragma unroll
        for (int ph = 0; ph < NW; ++ph) {
            const int it = it0 + ph;
            if (it >= nf) break;
            insert((ph + 2 * H) % NW);
            if (it + 1 < nf) fetch(row0 + it + 1 + 2 * H);

            const int cen = (ph + H) % NW;  // slot of the row whose f* is computed
            // x-neighbours of the lane's outer columns, from the adjacent lanes
            C xl1[5], xr1[5], xl2[5], xr2[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                xl1[q] = from_left(w[XF[q]][cen][CPL - 1]);
                xr1[q] = from_right(w[XF[q]][cen][0]);
                xl2[q] = H == 2 ? from_left(w[XF[q]][cen][CPL - 2]) : C(0);
                xr2[q] = H == 2 ? from_right(w[XF[q]][cen][1]) : C(0);
            }
            C f[CPL][9];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                C d[10];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const int fx = XF[q], fy = YF[q];
                    const C m1 = c > 0 ? w[fx][cen][c > 0 ? c - 1 : 0] : xl1[q];
                    const C p1 = c < CPL - 1 ? w[fx][cen][c < CPL - 1 ? c + 1 : 0] : xr1[q];
                    C m2 = C(0), p2 = C(0), ym2 = C(0), yp2 = C(0);
                    if (H == 2) {
                        m2 = c >= 2 ? w[fx][cen][c >= 2 ? c - 2 : 0] : (c == 1 ? xl1[q] : xl2[q]);
                        p2 = c + 2 < CPL ? w[fx][cen][c + 2 < CPL ? c + 2 : 0] : (c + 2 == CPL ? xr1[q] : xr2[q]);
                        ym2 = w[fy][ph % NW][c];
                        yp2 = w[fy][(ph + 2 * H) % NW][c];
                    }
                    d[2 * q] = S::diff(m2, m1, p1, p2);
                    d[2 * q + 1] = S::diff(ym2, w[fy][(ph + H - 1) % NW][c], w[fy][(ph + H + 1) % NW][c], yp2);
                }
                fd_node_fstar<C>(w[0][cen][c], w[1][cen][c], w[2][cen][c], d, a.k, f[c]);
            }
            // populations moving along +x come from the column on the left, along -x from
            // the column on the right
            const C f1l = from_left(f[CPL - 1][1]), f5l = from_left(f[CPL - 1][5]), f8l = from_left(f[CPL - 1][8]);
            const C f3r = from_right(f[0][3]), f6r = from_right(f[0][6]), f7r = from_right(f[0][7]);
            Group<T, CPL> gr, gx, gy;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int cl = c > 0 ? c - 1 : 0, cr = c < CPL - 1 ? c + 1 : 0;
                const C c1 = c > 0 ? f[cl][1] : f1l;
                const C u5 = c > 0 ? f[cl][5] : f5l;
                const C d8 = c > 0 ? f[cl][8] : f8l;
                const C c3 = c < CPL - 1 ? f[cr][3] : f3r;
                const C u6 = c < CPL - 1 ? f[cr][6] : f6r;
                const C d7 = c < CPL - 1 ? f[cr][7] : f7r;
                const C cen_ = (f[c][0] + c1) + c3, cenx = c1 - c3;
                const C up = (f[c][2] + u5) + u6, upx = u5 - u6;
                const C dn = (f[c][4] + d7) + d8, dnx = d8 - d7;
                // output row r-1 = (cen(r-1) + up(r-2)) + dn(r)
                gr.v[c] = Storage<T>::store(A[c] + dn);
                gx.v[c] = Storage<T>::store(AX[c] + dnx);
                gy.v[c] = Storage<T>::store(UP[c] - dn);
                A[c] = cen_ + UPp[c];
                AX[c] = cenx + UPXp[c];
                UP[c] = UPp[c];
                UPp[c] = up;
                UPXp[c] = upx;
            }
            // the output row ybeg - 1 + it - 1 is complete once f* of ybeg - 1 + it is known
            if (it >= 2 && store_ok) {
                const size_t off = (size_t)(ybeg + it - 2) * (size_t)nx + (size_t)col;
                store_group<T, CPL>(a.odr + off, gr);
                store_group<T, CPL>(a.ojx + off, gx);
                store_group<T, CPL>(a.ojy + off, gy);
            }
        }
    }
}

template <typename T> constexpr int cols_per_lane() { return sizeof(T) == 8 ? 2 : 4; }

template <typename T, int ST> int strip_cols()
{
    constexpr int CPL = cols_per_lane<T>();
    constexpr int H = Stencil<ST>::H;
    constexpr int PAD = ((H + 1 + CPL - 1) / CPL) * CPL;
    return 64 * CPL - 2 * PAD;
}

template <typename T, int ST, bool WALLS>
hipError_t run(const FdArgs &fa, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    using C = typename Storage<T>::C;
    constexpr int CPL = cols_per_lane<T>();
    const size_t n = (size_t)fa.nx * (size_t)fa.ny;
    SweepArgs<T> a;
    const T *in = static_cast<const T *>(src);
    T *out = static_cast<T *>(dst);
    a.dr = in;
    a.jx = in + n;
    a.jy = in + 2 * n;
    a.odr = out;
    a.ojx = out + n;
    a.ojy = out + 2 * n;
    a.nx = fa.nx;
    a.ny = fa.ny;
    a.rows = tile_rows > 0 ? tile_rows : 64;
    a.strips_x = (fa.nx + strip_cols<T, ST>() - 1) / strip_cols<T, ST>();
    a.strips_y = (fa.ny + a.rows - 1) / a.rows;
    a.ntiles = a.strips_x * a.strips_y;
    const double scale = ST == 3 ? Stencil<3>::SCALE : Stencil<5>::SCALE;
    a.k.ke = C(scale * (1.0 - 1.0 / fa.s_e));
    a.k.kxx = C(scale * (1.0 - 1.0 / fa.s_xx));
    a.k.hfx = C(0.5 * fa.fx);
    a.k.hfy = C(0.5 * fa.fy);
    a.k.qfx = C(0.25 * fa.fx);
    a.k.qfy = C(0.25 * fa.fy);
    a.k.dfx = C(fa.fx);
    a.k.dfy = C(fa.fy);
    const int blocks = (a.ntiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    hipLaunchKernelGGL((fd_sweep_kernel<T, CPL, ST, WALLS>), blocks, 64 * WAVES_PER_BLOCK, 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch(const FdArgs &a, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    if (a.stencil == 3)
        return a.walls ? run<T, 3, true>(a, tile_rows, src, dst, s) : run<T, 3, false>(a, tile_rows, src, dst, s);
    return a.walls ? run<T, 5, true>(a, tile_rows, src, dst, s) : run<T, 5, false>(a, tile_rows, src, dst, s);
}

}  // namespace

bool fd_sweep_supported(const FdArgs &a)
{
    const int cpl = a.dtype == FDLBM_F64 ? 2 : 4;
    return a.nx % cpl == 0 && (a.stencil == 3 || a.stencil == 5);
}

hipError_t launch_fd_sweep(const FdArgs &a, int tile_rows, const void *src, void *dst, hipStream_t s)
{
    switch (a.dtype) {
    case FDLBM_F64: return dispatch<double>(a, tile_rows, src, dst, s);
    case FDLBM_F32: return dispatch<float>(a, tile_rows, src, dst, s);
    default: return dispatch<__half>(a, tile_rows, src, dst, s);
    }
}

}  // namespace fdlbm
