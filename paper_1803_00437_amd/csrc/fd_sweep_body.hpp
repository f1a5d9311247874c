// Body of the fused FD-LBM sweep: one block of WV stacked wavefronts updating one tile
// (a strip of 64*CPL columns by WV*R rows) of one grid.  Shared by the single-grid kernel
// (fd_sweep.hip) and the multi-instance kernel (fd_batch.hip), so that both produce the
// same bits as the reference path.  See fd_sweep.hip for the mapping.
#pragma once

#include "fdlbm_device.hpp"

namespace fdlbm {
namespace sweep {


constexpr int WV = 4;  // wavefronts stacked per block

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

// CPL consecutive stored values as one memory access (2, 4, 8 or 16 bytes).
template <typename T, int CPL> struct Group {
    T v[CPL];
};
template <int BYTES> struct Word;
template <> struct Word<2> { using type = unsigned short; };
template <> struct Word<4> { using type = unsigned int; };
template <> struct Word<8> { typedef unsigned int type __attribute__((ext_vector_type(2))); };
template <> struct Word<16> { typedef unsigned int type __attribute__((ext_vector_type(4))); };

template <typename T, int CPL> __device__ __forceinline__ Group<T, CPL> load_group(const T *p)
{
    static_assert(sizeof(Group<T, CPL>) == sizeof(T) * CPL, "packed group");
    using Wd = typename Word<sizeof(T) * CPL>::type;
    return __builtin_bit_cast(Group<T, CPL>, *reinterpret_cast<const Wd *>(p));
}
template <typename T, int CPL> __device__ __forceinline__ void store_group(T *p, const Group<T, CPL> &g)
{
    using Wd = typename Word<sizeof(T) * CPL>::type;
    __builtin_nontemporal_store(__builtin_bit_cast(Wd, g), reinterpret_cast<Wd *>(p));
}

// Strip geometry: a strip loads W columns starting at s*S - P and stores the S = W - 2P
// columns [s*S, s*S + S), where P = h+1 rounded up to whole lanes.
template <int CPL, int H> struct Strip {
    static constexpr int W = 64 * CPL;
    static constexpr int P = ((H + 1 + CPL - 1) / CPL) * CPL;
    static constexpr int S = W - 2 * P;
};

// One grid as a tile sees it: input and output planes, size, rows per wavefront and the
// reconstruction constants.
template <typename T> struct TileArgs {
    const T *dr, *jx, *jy;
    T *odr, *ojx, *ojy;
    int nx, ny, rows;
    FdCoef<typename Storage<T>::C> k;
};

// LDS slots per wavefront, each CPL x 64 values: the row sums a wavefront publishes for its
// neighbours (populations its first f* row sends down, its last f* row sends up), and the
// parts of its own first output row that it keeps until the barrier (same-row and
// row-above differences, and its own upward row sum to subtract from what arrives).
enum { PUB_DN = 0, PUB_DNX, PUB_UP, PUB_UPX, OWN_PC, OWN_PCX, OWN_LU, OWN_LUX, OWN_PD, OWN_PDX, NSLOT };

// One tile: the block's WV wavefronts over column strip sx and row band `band` of one
// grid.  Called by every wavefront of the block (it contains a block barrier).
template <typename T, int CPL, int ST, bool WALLS, bool FORCE>
__device__ __forceinline__ void sweep_tile(const TileArgs<T> &a, int band, int sx)
{
    using C = typename Storage<T>::C;
    using S = Stencil<ST>;
    constexpr int H = S::H;
    constexpr int NW = 2 * H + 1;  // rows in the input window
    using G = Strip<CPL, H>;
    static_assert(CPL >= 2 || H == 1, "5-point differences need two columns per lane");
    __shared__ C lds[WV][NSLOT][CPL][64];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    const int xl = sx * G::S - G::P + CPL * lane;  // first column of this lane (unwrapped)
    const int col = ((xl % nx) + nx) % nx;          // wrapped (x periodic)
    const bool store_ok = CPL * lane >= G::P && CPL * lane < G::P + G::S && xl < nx;

    // rows of this wavefront: R each; a single leftover row at the end of the band is
    // absorbed by the wavefront below it, so every non-empty wavefront has >= 2 rows
    // unless the whole band has one row
    const int b0 = band * WV * a.rows, b1 = min(b0 + WV * a.rows, ny);
    const int ybeg = b0 + wv * a.rows;
    int yend = min(ybeg + a.rows, b1);
    if (b1 - yend == 1) yend = b1;
    const bool empty = ybeg >= b1 || (wv > 0 && b1 - ybeg == 1);
    const bool bottom = wv == 0;  // computes f* of row ybeg - 1 itself
    const bool top = yend == b1;  // computes f* of row yend itself
    const int rb = bottom ? ybeg - 1 : ybeg;
    const int re = top ? yend : yend - 1;
    const int nf = empty ? 0 : re - rb + 1;  // rows whose f* this wavefront computes
    const int row0 = rb - H;                 // first input row

    // rolling window of input rows: drho and J (sign-flipped on ghost rows); the products
    // of J_a = J + F/2 are formed where the derivatives need them
    C w[3][NW][CPL];
    Group<T, CPL> pr, px, py;  // prefetched row (raw storage)
    C ps = C(1);               // its sign (-1: ghost row beyond a wall)

    auto fetch = [&](int j) {
        int src = j;
        C sgn = C(1);
        if (WALLS) {
            if (j < 0) { src = -1 - j; sgn = C(-1); }
            else if (j >= ny) { src = 2 * ny - 1 - j; sgn = C(-1); }
        } else {
            src = j < 0 ? j + ny : (j >= ny ? j - ny : j);
        }
        const size_t off = (size_t)src * (size_t)nx + (size_t)col;
        pr = load_group<T, CPL>(a.dr + off);
        px = load_group<T, CPL>(a.jx + off);
        py = load_group<T, CPL>(a.jy + off);
        ps = sgn;
    };
    auto insert = [&](int wslot) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            w[0][wslot][c] = Storage<T>::load(pr.v[c]);
            w[1][wslot][c] = ps * Storage<T>::load(px.v[c]);
            w[2][wslot][c] = ps * Storage<T>::load(py.v[c]);
        }
    };

    // carried between rows, when f* of row r is being computed: QP = fd_partial of output
    // row r-1 (its same-row and row-below parts), LD, LDX = the own downward row sums of
    // row r-1, UPp, UPXp = the row sums row r-1 sends up
    FdPartial<C> QP[CPL];
    C LD[CPL], LDX[CPL], UPp[CPL], UPXp[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        QP[c].q = QP[c].qx = QP[c].pu = C(0);
        LD[c] = LDX[c] = UPp[c] = UPXp[c] = C(0);
    }

    if (nf > 0) {
        // prologue: the first 2H input rows, then the prefetch of the next one
#pragma unroll
        for (int r = 0; r < 2 * H; ++r) {
            fetch(row0 + r);
            insert(r);
        }
        fetch(row0 + 2 * H);
    }

    // x-derivative fields (drho, Jx, Jy, Jx^2, JxJy) -> d[0], d[2], d[4], d[6], d[8];
    // y-derivative fields (drho, Jy, Jx, JxJy, Jy^2) -> d[1], d[3], d[5], d[7], d[9]
    // (products of J_a).  yfield(q, slot, c): y-derivative field q of a window row.
    auto yfield = [&](int q, int slot, int c) -> C {
        const C xa = plus_force<FORCE>(w[1][slot][c], a.k.hfx), ya = plus_force<FORCE>(w[2][slot][c], a.k.hfy);
        return q == 0 ? w[0][slot][c] : q == 1 ? w[2][slot][c] : q == 2 ? w[1][slot][c] : q == 3 ? xa * ya : ya * ya;
    };

    for (int it0 = 0; it0 < nf; it0 += NW) {
#pragma unroll
        for (int ph = 0; ph < NW; ++ph) {
            const int it = it0 + ph;
            if (it >= nf) break;
            insert((ph + 2 * H) % NW);
            if (it + 1 < nf) fetch(row0 + 2 * H + it + 1);

            const int cs = (ph + H) % NW;  // window slot of the row whose f* is computed
            // x-derivative fields of this row, and the J_a of its nodes
            C xf[5][CPL], jxa[CPL], jya[CPL];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                jxa[c] = plus_force<FORCE>(w[1][cs][c], a.k.hfx);
                jya[c] = plus_force<FORCE>(w[2][cs][c], a.k.hfy);
                xf[0][c] = w[0][cs][c];
                xf[1][c] = w[1][cs][c];
                xf[2][c] = w[2][cs][c];
                xf[3][c] = jxa[c] * jxa[c];
                xf[4][c] = jxa[c] * jya[c];
            }
            // x-neighbours of the lane's outer columns, from the adjacent lanes
            C xl1[5], xr1[5], xl2[5], xr2[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                xl1[q] = from_left(xf[q][CPL - 1]);
                xr1[q] = from_right(xf[q][0]);
                xl2[q] = H == 2 ? from_left(xf[q][CPL >= 2 ? CPL - 2 : 0]) : C(0);
                xr2[q] = H == 2 ? from_right(xf[q][CPL > 1 ? 1 : 0]) : C(0);
            }
            C f[CPL][9];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                C d[10];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    const C m1 = c > 0 ? xf[q][c > 0 ? c - 1 : 0] : xl1[q];
                    const C p1 = c < CPL - 1 ? xf[q][c < CPL - 1 ? c + 1 : 0] : xr1[q];
                    C m2 = C(0), p2 = C(0), ym2 = C(0), yp2 = C(0);
                    if (H == 2) {
                        m2 = c >= 2 ? xf[q][c >= 2 ? c - 2 : 0] : (c == 1 ? xl1[q] : xl2[q]);
                        p2 = c + 2 < CPL ? xf[q][c + 2 < CPL ? c + 2 : 0] : (c + 2 == CPL ? xr1[q] : xr2[q]);
                        ym2 = yfield(q, ph % NW, c);
                        yp2 = yfield(q, (ph + 2 * H) % NW, c);
                    }
                    d[2 * q] = S::diff(m2, m1, p1, p2);
                    d[2 * q + 1] = S::diff(ym2, yfield(q, (ph + H - 1) % NW, c), yfield(q, (ph + H + 1) % NW, c), yp2);
                }
                fd_node_fstar<C, FORCE>(w[0][cs][c], jxa[c], jya[c], d, a.k, f[c]);
            }
            // populations moving along +x come from the column on the left, along -x from
            // the column on the right
            const C f1l = from_left(f[CPL - 1][1]), f5l = from_left(f[CPL - 1][5]), f8l = from_left(f[CPL - 1][8]);
            const C f3r = from_right(f[0][3]), f6r = from_right(f[0][6]), f7r = from_right(f[0][7]);
            const int os = (ph + H - 1) % NW;  // window slot of output row r - 1
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
                // row sums arriving at row r from row r, at r + 1 (up) and at r - 1 (dn)
                const C up = row_sum(f[c][2], u5, u6), upx = u5 - u6;
                const C dn = row_sum(f[c][4], d8, d7), dnx = d8 - d7;
                // the same groups of this node's own populations
                const C lu = row_sum(f[c][2], f[c][5], f[c][6]), lux = f[c][5] - f[c][6];
                const C ld = row_sum(f[c][4], f[c][8], f[c][7]), ldx = f[c][8] - f[c][7];
                C pc, pcx;
                same_row_part<C>(c1 - f[c][1], c3 - f[c][3], pc, pcx);
                const C pd = dn - LD[c], pdx = dnx - LDX[c];  // row-above part of row r - 1
                if (!bottom && it == 0) {
                    // f* of the first row: its downward sums complete the last output row
                    // of the wavefront below; its own row still lacks the upward sums of
                    // that wavefront
                    lds[wv][PUB_DN][c][lane] = dn;
                    lds[wv][PUB_DNX][c][lane] = dnx;
                    lds[wv][OWN_PC][c][lane] = pc;
                    lds[wv][OWN_PCX][c][lane] = pcx;
                    lds[wv][OWN_LU][c][lane] = lu;
                    lds[wv][OWN_LUX][c][lane] = lux;
                }
                if (!bottom && it == 1) {
                    lds[wv][OWN_PD][c][lane] = pd;
                    lds[wv][OWN_PDX][c][lane] = pdx;
                }
                // output row r - 1
                C nr, nxv, nyv;
                fd_finish<C, FORCE>(QP[c], pd, pdx, w[0][os][c], w[1][os][c], w[2][os][c], a.k.dfx, a.k.dfy, nr, nxv, nyv);
                gr.v[c] = Storage<T>::store(nr);
                gx.v[c] = Storage<T>::store(nxv);
                gy.v[c] = Storage<T>::store(nyv);
                QP[c] = fd_partial<C>(pc, pcx, UPp[c] - lu, UPXp[c] - lux);
                LD[c] = ld;
                LDX[c] = ldx;
                UPp[c] = up;
                UPXp[c] = upx;
            }
            // output row rb + it - 1 is complete once f* of rows rb + it - 2 .. rb + it are known
            if (it >= 2 && store_ok) {
                const size_t off = (size_t)(rb + it - 1) * (size_t)nx + (size_t)col;
                store_group<T, CPL>(a.odr + off, gr);
                store_group<T, CPL>(a.ojx + off, gx);
                store_group<T, CPL>(a.ojy + off, gy);
            }
        }
    }
    // stored values of the two output rows completed after the barrier (interior rows)
    Group<T, CPL> o0r, o0x, o0y, o1r, o1x, o1y;
    if (!empty && !bottom) {
        const size_t off = (size_t)ybeg * (size_t)nx + (size_t)col;
        o0r = load_group<T, CPL>(a.dr + off);
        o0x = load_group<T, CPL>(a.jx + off);
        o0y = load_group<T, CPL>(a.jy + off);
    }
    if (!empty && !top) {
        const size_t off = (size_t)(yend - 1) * (size_t)nx + (size_t)col;
        o1r = load_group<T, CPL>(a.dr + off);
        o1x = load_group<T, CPL>(a.jx + off);
        o1y = load_group<T, CPL>(a.jy + off);
    }
    if (!top && !empty) {
        // the upward sums of the last f* row complete the first output row of the
        // wavefront above
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            lds[wv][PUB_UP][c][lane] = UPp[c];
            lds[wv][PUB_UPX][c][lane] = UPXp[c];
        }
    }
    __syncthreads();
    if (empty) return;
    if (!bottom) {
        // first output row: own same-row and row-above parts, upward sums from below
        Group<T, CPL> gr, gx, gy;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const C pu = lds[wv - 1][PUB_UP][c][lane] - lds[wv][OWN_LU][c][lane];
            const C pux = lds[wv - 1][PUB_UPX][c][lane] - lds[wv][OWN_LUX][c][lane];
            C nr, nxv, nyv;
            fd_finish<C, FORCE>(fd_partial<C>(lds[wv][OWN_PC][c][lane], lds[wv][OWN_PCX][c][lane], pu, pux),
                         lds[wv][OWN_PD][c][lane], lds[wv][OWN_PDX][c][lane], Storage<T>::load(o0r.v[c]),
                         Storage<T>::load(o0x.v[c]), Storage<T>::load(o0y.v[c]), a.k.dfx, a.k.dfy, nr, nxv, nyv);
            gr.v[c] = Storage<T>::store(nr);
            gx.v[c] = Storage<T>::store(nxv);
            gy.v[c] = Storage<T>::store(nyv);
        }
        if (store_ok) {
            const size_t off = (size_t)ybeg * (size_t)nx + (size_t)col;
            store_group<T, CPL>(a.odr + off, gr);
            store_group<T, CPL>(a.ojx + off, gx);
            store_group<T, CPL>(a.ojy + off, gy);
        }
    }
    if (!top) {
        // last output row: carried parts + downward sums from the wavefront above
        Group<T, CPL> gr, gx, gy;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const C pd = lds[wv + 1][PUB_DN][c][lane] - LD[c];
            const C pdx = lds[wv + 1][PUB_DNX][c][lane] - LDX[c];
            C nr, nxv, nyv;
            fd_finish<C, FORCE>(QP[c], pd, pdx, Storage<T>::load(o1r.v[c]), Storage<T>::load(o1x.v[c]),
                         Storage<T>::load(o1y.v[c]), a.k.dfx, a.k.dfy, nr, nxv, nyv);
            gr.v[c] = Storage<T>::store(nr);
            gx.v[c] = Storage<T>::store(nxv);
            gy.v[c] = Storage<T>::store(nyv);
        }
        if (store_ok) {
            const size_t off = (size_t)(yend - 1) * (size_t)nx + (size_t)col;
            store_group<T, CPL>(a.odr + off, gr);
            store_group<T, CPL>(a.ojx + off, gx);
            store_group<T, CPL>(a.ojy + off, gy);
        }
    }
}


// Host-side strip width of a (dtype, CPL, stencil) combination.
template <int CPL, int H> constexpr int strip_stride() { return Strip<CPL, H>::S; }

template <typename C> inline FdCoef<C> make_coef(int stencil, double s_xx, double s_e, double fx, double fy)
{
    const double scale = stencil == 3 ? Stencil<3>::SCALE : Stencil<5>::SCALE;
    FdCoef<C> k;
    k.ke = C(scale * (1.0 - 1.0 / s_e));
    k.kxx = C(scale * (1.0 - 1.0 / s_xx));
    k.hfx = C(0.5 * fx);
    k.hfy = C(0.5 * fy);
    k.qfx = C(0.25 * fx);
    k.qfy = C(0.25 * fy);
    k.dfx = C(fx);
    k.dfy = C(fy);
    return k;
}

}  // namespace sweep
}  // namespace fdlbm
