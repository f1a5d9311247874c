// Body of the fused FD-LBM sweep: one block of WV stacked wavefronts updating one tile
// (a strip of 64*CPL columns by WV*R rows) of one grid.  Shared by the single-grid kernel
// (fd_sweep.hip) and the multi-instance kernel (fd_batch.hip), so that both produce the
// same bits as the reference path.  See fd_sweep.hip for the mapping.
#pragma once

#include <type_traits>

#include "fdlbm_device.hpp"

namespace fdlbm {
namespace sweep {


constexpr int WV = 4;  // wavefronts stacked per block
// Input rows loaded ahead of the row that uses them.  Two keep more bytes in flight; FP16
// storage with four columns per lane keeps one, which leaves it a third wavefront per SIMD
// (measured at 8192^2: FP32 +1.5 %, FP16 with two columns per lane +7 %, FP16 with four
// columns -3 % with two rows ahead).
template <typename T, int CPL> constexpr int prefetch_rows() { return sizeof(T) == 2 && CPL == 4 ? 1 : 2; }

// whole-wave lane shifts: shl gives lane i the value of lane i+1, shr the value of lane i-1
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL> __device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
template <int CTRL> __device__ __forceinline__ double lane_shift(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
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

// Row accesses through a buffer resource.  The hardware range-checks every buffer access
// against the resource's size: an access at OFF_NONE (beyond any row) is dropped (a load
// returns zero).  The sweep loop uses this instead of branching around its row loads and
// stores, so every iteration issues the same memory operations and the waits for the
// prefetched row never have to wait for the previous row's stores as well.
constexpr unsigned OFF_NONE = 0x80000000u;
constexpr int RSRC_WORD3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)
constexpr int NT_HINT = 2;              // non-temporal store (written once, read next step)

// Buffer resource of one row of a field: the field's first row at `field`, rows `stride`
// elements apart (3 nx in the row-interleaved state), nx elements long.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const T *field, int row, int stride, int nx)
{
    const unsigned long long r = reinterpret_cast<unsigned long long>(field + (size_t)(unsigned)row * (size_t)(unsigned)stride);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)r);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(r >> 32));
    void *base = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(base, 0, nx * (int)sizeof(T), RSRC_WORD3);
}

template <int BYTES> struct BufOps;
template <> struct BufOps<2> {
    using W = Word<2>::type;
    static __device__ __forceinline__ W load(__amdgpu_buffer_rsrc_t r, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0);
    }
    static __device__ __forceinline__ void store(W v, __amdgpu_buffer_rsrc_t r, unsigned off)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, NT_HINT);
    }
};
template <> struct BufOps<4> {
    using W = Word<4>::type;
    static __device__ __forceinline__ W load(__amdgpu_buffer_rsrc_t r, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    }
    static __device__ __forceinline__ void store(W v, __amdgpu_buffer_rsrc_t r, unsigned off)
    {
        __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, NT_HINT);
    }
};
template <> struct BufOps<8> {
    using W = Word<8>::type;
    static __device__ __forceinline__ W load(__amdgpu_buffer_rsrc_t r, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    }
    static __device__ __forceinline__ void store(W v, __amdgpu_buffer_rsrc_t r, unsigned off)
    {
        __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, NT_HINT);
    }
};
template <> struct BufOps<16> {
    using W = Word<16>::type;
    static __device__ __forceinline__ W load(__amdgpu_buffer_rsrc_t r, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    }
    static __device__ __forceinline__ void store(W v, __amdgpu_buffer_rsrc_t r, unsigned off)
    {
        __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, NT_HINT);
    }
};
template <typename T, int CPL> __device__ __forceinline__ Group<T, CPL> buf_load_group(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    return __builtin_bit_cast(Group<T, CPL>, BufOps<sizeof(T) * CPL>::load(r, off));
}
template <typename T, int CPL>
__device__ __forceinline__ void buf_store_group(__amdgpu_buffer_rsrc_t r, unsigned off, const Group<T, CPL> &g)
{
    BufOps<sizeof(T) * CPL>::store(__builtin_bit_cast(typename Word<sizeof(T) * CPL>::type, g), r, off);
}

// How a lane reaches its CPL columns of a row (x periodic):
//   AM_VEC   one access at a CPL-aligned offset (nx a multiple of CPL)
//   AM_COL   one access per column, each at its own wrapped offset (any nx)
//   AM_UNAL  one access at an element-aligned offset; a lane whose columns cross the
//            periodic edge accesses them one by one instead, behind a branch that only
//            the wavefronts holding such a lane take (any nx; 4- and 8-byte elements,
//            whose vector accesses need no more than element alignment on this GPU)
constexpr int AM_VEC = 0, AM_COL = 1, AM_UNAL = 2;

// Byte offsets of a lane's loads and stores in a row (OFF_NONE: none): [0] the vector
// access (AM_VEC, AM_UNAL), [c] or [1 + c] column c (AM_COL, AM_UNAL).  Stores leave out the
// columns the tile does not store.
template <int CPL, int AM> struct LaneCols {
    static constexpr int K = AM == AM_VEC ? 1 : AM == AM_COL ? CPL : 1 + CPL;
    unsigned ld[K], st[K];
    bool edge;   // AM_UNAL: a lane of this wavefront crosses the edge (wave-uniform)
    bool cross;  // AM_UNAL: this lane's columns cross the edge
};

template <typename T, int CPL, int AM>
__device__ __forceinline__ LaneCols<CPL, AM> make_lane_cols(int xl, int nx, bool stored)
{
    LaneCols<CPL, AM> lc;
    lc.edge = lc.cross = false;
    auto wrapped = [&](int x) { return (unsigned)(((x % nx) + nx) % nx); };
    if constexpr (AM == AM_COL) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            lc.ld[c] = wrapped(xl + c) * (unsigned)sizeof(T);
            lc.st[c] = stored && xl + c < nx ? lc.ld[c] : OFF_NONE;
        }
    } else {
        const unsigned cx = wrapped(xl);
        const bool cross = AM == AM_UNAL && cx + CPL > (unsigned)nx;  // group runs past column nx - 1
        lc.ld[0] = cross ? OFF_NONE : cx * (unsigned)sizeof(T);
        lc.st[0] = stored && xl < nx && !cross ? cx * (unsigned)sizeof(T) : OFF_NONE;
        if constexpr (AM == AM_UNAL) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const unsigned o = wrapped(xl + c) * (unsigned)sizeof(T);
                lc.ld[1 + c] = cross ? o : OFF_NONE;
                lc.st[1 + c] = cross && stored && xl + c < nx ? o : OFF_NONE;
            }
            lc.edge = __builtin_amdgcn_ballot_w64(cross) != 0;
            lc.cross = cross;
        }
    }
    return lc;
}

template <typename T, int CPL, int AM>
__device__ __forceinline__ Group<T, CPL> row_load(__amdgpu_buffer_rsrc_t r, const LaneCols<CPL, AM> &lc, bool use)
{
    using W1 = typename Word<sizeof(T)>::type;
    if constexpr (AM == AM_COL) {
        Group<T, CPL> g;
#pragma unroll
        for (int c = 0; c < CPL; ++c) g.v[c] = __builtin_bit_cast(T, BufOps<sizeof(T)>::load(r, use ? lc.ld[c] : OFF_NONE));
        return g;
    } else {
        Group<T, CPL> g = buf_load_group<T, CPL>(r, use ? lc.ld[0] : OFF_NONE);
        if constexpr (AM == AM_UNAL) {
            if (lc.edge && lc.cross) {
                // only the crossing lane is active here; its vector load read zeros
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    g.v[c] = __builtin_bit_cast(T, BufOps<sizeof(T)>::load(r, use ? lc.ld[1 + c] : OFF_NONE));
            }
        }
        return g;
    }
}

template <typename T, int CPL, int AM>
__device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, const LaneCols<CPL, AM> &lc, bool use,
                                          const Group<T, CPL> &g)
{
    using W1 = typename Word<sizeof(T)>::type;
    if constexpr (AM == AM_COL) {
#pragma unroll
        for (int c = 0; c < CPL; ++c)
            BufOps<sizeof(T)>::store(__builtin_bit_cast(W1, g.v[c]), r, use ? lc.st[c] : OFF_NONE);
    } else {
        buf_store_group<T, CPL>(r, use ? lc.st[0] : OFF_NONE, g);
        if constexpr (AM == AM_UNAL) {
            if (lc.edge && lc.cross) {
#pragma unroll
                for (int c = 0; c < CPL; ++c)
                    BufOps<sizeof(T)>::store(__builtin_bit_cast(W1, g.v[c]), r, use ? lc.st[1 + c] : OFF_NONE);
            }
        }
    }
}

// Strip geometry: a strip loads W columns starting at s*S - P and stores the S = W - 2P
// columns [s*S, s*S + S), where P = h+1 rounded up to whole lanes.
template <int CPL, int H> struct Strip {
    static constexpr int W = 64 * CPL;
    static constexpr int P = ((H + 1 + CPL - 1) / CPL) * CPL;
    static constexpr int S = W - 2 * P;
};

// One grid as a tile sees it: the first rows of the input and output fields (rows of a field
// 3 nx apart, see fd_elem), size, rows per wavefront and the
// reconstruction constants.
template <typename T> struct TileArgs {
    const T *dr, *jx, *jy;
    T *odr, *ojx, *ojy;
    int nx, ny, rows;
    FdCoef<typename Storage<T>::C> k;
    GhostRules<typename Storage<T>::C> gr;  // walls only
    uint32_t seed = 0;                      // stochastic rounding: pcg_hash of the step count
};

// Each wavefront of a block sweeps its rows in one direction: even wavefronts downward,
// odd ones upward.  Two neighbouring wavefronts then both start, or both end, at the
// boundary between them, so the rows there are loaded by both at about the same time and
// the second load is served by the caches.
//
// LDS slots per wavefront, each CPL x 64 values: the row sums its first f* row sends across
// its start side (START_*) and its last f* row across its end side (END_*), and what its
// first output row keeps until the barrier (OWN_*: the same-row part, its own sums toward
// the start side, to subtract from what arrives there, the part from the row after it,
// and its stored values, loaded long before and no longer in cache by then).
enum {
    START_S = 0, START_SX, END_S, END_SX, OWN_PC, OWN_PCX, OWN_L, OWN_LX, OWN_P2, OWN_P2X, OWN_R, OWN_X, OWN_Y, NSLOT
};

// The rows of one wavefront in direction DIR (+1: upward, -1: downward).  "Forward" sums
// go to the next row in sweep order, "backward" sums to the previous one; row r's output
// needs its same-row part, the forward sums of the row before it and the backward sums of
// the row after it, combined in the order fd_partial / fd_finish fix (same-row, below,
// above) whatever the direction.
template <int DIR, typename T, int CPL, int ST, bool WALLS, bool FORCE, int AM>
__device__ __forceinline__ void sweep_wave(const TileArgs<T> &a, typename Storage<T>::C (&lds)[WV][NSLOT][CPL][64],
                                           int wv, int lane, const LaneCols<CPL, AM> &lc, int xl, int ybeg,
                                           int yend, bool empty, bool bottom, bool top)
{
    using C = typename Storage<T>::C;
    using S = Stencil<ST>;
    constexpr int H = S::H;
    constexpr bool LW = ST == 1;   // LW-ACM: populations from the node alone
    // rows in use: the 2H + 1 the derivatives read, which include the output row when
    // H > 0; without derivatives, the f* row and the output row before it
    constexpr int NW = H > 0 ? 2 * H + 1 : 2;
    constexpr int PD = prefetch_rows<T, CPL>();
    constexpr int U = (NW + PD + 1) & ~1;  // window slots: those rows and the ones in flight, even
    const int nx = a.nx, ny = a.ny;
    // the three new values of column c of row `row`, rounded for storage (stochastically
    // for HalfSR, with the random bits of that node and step)
    auto round_out = [&](int row, int c, C nr, C nxv, C nyv, T &gr_, T &gx_, T &gy_) {
        uint32_t rb_[3] = {0u, 0u, 0u};
        if constexpr (Storage<T>::STOCHASTIC)
            sr_draw(uint32_t(row) * uint32_t(nx) + uint32_t(xl + c), a.seed, rb_);
        gr_ = Storage<T>::store_r(nr, rb_[0]);
        gx_ = Storage<T>::store_r(nxv, rb_[1]);
        gy_ = Storage<T>::store_r(nyv, rb_[2]);
    };

    const int rb = bottom ? ybeg - 1 : ybeg;  // f* rows rb .. re (the band's outer
    const int re = top ? yend : yend - 1;     // wavefronts also take the row beyond)
    const int nf = empty ? 0 : re - rb + 1;
    const bool start_edge = DIR > 0 ? bottom : top;  // start / end side on the band edge
    const bool end_edge = DIR > 0 ? top : bottom;
    const int first = DIR > 0 ? rb : re;  // first f* row in sweep order
    const int row0 = first - DIR * H;     // first input row

    // rolling window of input rows in sweep order, input row m in slot m % U: drho and J as
    // used (sign-flipped on ghost rows); the products of J_a = J + F/2 are formed where the
    // derivatives need them.  The loop below is unrolled U times, so every slot stays in the
    // same registers; U is even, so values carried from one row to the next alternate
    // between two sets of registers with no copies.  Rows stored in the arithmetic type are
    // loaded straight into their slot (RAW = U load targets); FP16 rows are loaded into one
    // prefetch group per row in flight and converted into their slot when it comes due.
    constexpr int RAW = sizeof(T) < sizeof(C) ? PD : U;
    static_assert(U % RAW == 0, "a slot's load group must not depend on the loop iteration");
    C w[3][U][CPL];
    Group<T, CPL> pr[RAW], px[RAW], py[RAW];
    // with walls, a loaded row's factors for drho and J (1, 1 in the fluid) and, for a ghost
    // row interpolated between two fluid rows, the second row and its factors
    C pca[RAW], pcj[RAW], pbr[RAW], pbj[RAW];
    int psb[RAW];

    // load input row j (mirrored or wrapped) into window slot `slot`; `use` false issues the
    // same loads, dropped
    auto fetch = [&](int j, bool use, int slot) {
        int src = j, srcb = -1;
        C ca = C(1), cj = C(1), br = C(0), bj = C(0);
        if (WALLS) {
            if (j < 0 || j >= ny) {  // ghost row beyond a wall
                const GhostRule<C> q = ghost_rule(a.gr, j < 0 ? -j : j - ny + 1);
                src = j < 0 ? q.sa : ny - 1 - q.sa;
                if (q.sb >= 0) srcb = min(max(j < 0 ? q.sb : ny - 1 - q.sb, 0), ny - 1);
                ca = q.car;
                cj = q.caj;
                br = q.cbr;
                bj = q.cbj;
            }
        } else {
            src = j < 0 ? j + ny : (j >= ny ? j - ny : j);
        }
        src = min(max(src, 0), ny - 1);
        const int r = slot % RAW;
        pr[r] = row_load<T, CPL, AM>(row_rsrc(a.dr, src, 3 * nx, nx), lc, use);
        px[r] = row_load<T, CPL, AM>(row_rsrc(a.jx, src, 3 * nx, nx), lc, use);
        py[r] = row_load<T, CPL, AM>(row_rsrc(a.jy, src, 3 * nx, nx), lc, use);
        pca[r] = ca;
        pcj[r] = cj;
        pbr[r] = br;
        pbj[r] = bj;
        psb[r] = srcb;
    };
    auto insert = [&](int slot) {
        const int r = slot % RAW;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            w[0][slot][c] = WALLS ? pca[r] * Storage<T>::load(pr[r].v[c]) : Storage<T>::load(pr[r].v[c]);
            w[1][slot][c] = WALLS ? pcj[r] * Storage<T>::load(px[r].v[c]) : Storage<T>::load(px[r].v[c]);
            w[2][slot][c] = WALLS ? pcj[r] * Storage<T>::load(py[r].v[c]) : Storage<T>::load(py[r].v[c]);
        }
        if (WALLS && psb[r] >= 0) {
            // ghost row between two fluid rows (walls at a general distance): the second
            // row is read here, a few times per sweep at most
            const Group<T, CPL> br_ = row_load<T, CPL, AM>(row_rsrc(a.dr, psb[r], 3 * nx, nx), lc, true);
            const Group<T, CPL> bx_ = row_load<T, CPL, AM>(row_rsrc(a.jx, psb[r], 3 * nx, nx), lc, true);
            const Group<T, CPL> by_ = row_load<T, CPL, AM>(row_rsrc(a.jy, psb[r], 3 * nx, nx), lc, true);
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                w[0][slot][c] = w[0][slot][c] + pbr[r] * Storage<T>::load(br_.v[c]);
                w[1][slot][c] = w[1][slot][c] + pbj[r] * Storage<T>::load(bx_.v[c]);
                w[2][slot][c] = w[2][slot][c] + pbj[r] * Storage<T>::load(by_.v[c]);
            }
        }
    };

    // carried from the previous f* row (= the output row b finished at this one):
    // FW, FWX = the forward sums it sends to the current row; LB, LBX = its own sums in the
    // backward group; upward sweep: QP = fd_partial of b; downward: PC, PCX (same-row
    // part of b) and PF, PFX (its part from the row before it, i.e. from above)
    C FW[CPL], FWX[CPL], LB[CPL], LBX[CPL];
    FdPartial<C> QP[CPL];
    C PC[CPL], PCX[CPL], PF[CPL], PFX[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        FW[c] = FWX[c] = LB[c] = LBX[c] = C(0);
        QP[c].q = QP[c].qx = QP[c].pu = C(0);
        PC[c] = PCX[c] = PF[c] = PFX[c] = C(0);
    }

    if (nf > 0) {
        // prologue: the first 2H input rows, then the prefetch of the next one
#pragma unroll
        for (int m = 0; m < 2 * H; ++m) {
            fetch(row0 + DIR * m, true, m);
            insert(m);
        }
#pragma unroll
        for (int d = 0; d < PD; ++d) fetch(row0 + DIR * (2 * H + d), d < nf, 2 * H + d);
    }

    // x-derivative fields (drho, Jx, Jy, Jx^2, JxJy) -> d[0], d[2], d[4], d[6], d[8];
    // y-derivative fields (drho, Jy, Jx, JxJy, Jy^2) -> d[1], d[3], d[5], d[7], d[9]
    // (products of J_a).  yfield(q, slot, c): y-derivative field q of a window row.
    auto yfield = [&](int q, int slot, int c) -> C {
        const C xa = plus_force<FORCE>(w[1][slot][c], a.k.hfx), ya = plus_force<FORCE>(w[2][slot][c], a.k.hfy);
        return q == 0 ? w[0][slot][c] : q == 1 ? w[2][slot][c] : q == 2 ? w[1][slot][c] : q == 3 ? xa * ya : ya * ya;
    };

    for (int it0 = 0; it0 < nf; it0 += U) {
#pragma unroll
        for (int ph = 0; ph < U; ++ph) {
            const int it = it0 + ph;
            if (it >= nf) break;
            insert((ph + 2 * H) % U);
            // input row 2H + it + PD replaces a row that no later f* row reads
            fetch(row0 + DIR * (2 * H + it + PD), it + PD < nf, (ph + 2 * H + PD) % U);

            const int cs = (ph + H) % U;  // window slot of the row r whose f* is computed
            // window slot of row r + k (k rows up the grid)
            auto sl = [&](int k) { return (ph + H + DIR * k + 2 * U) % U; };
            C f[CPL][9];
            if constexpr (LW) {
#pragma unroll
                for (int c = 0; c < CPL; ++c) lw_node_g<C>(w[0][cs][c], w[1][cs][c], w[2][cs][c], a.k.lin, f[c]);
            } else {
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
                        ym2 = yfield(q, sl(-2), c);
                        yp2 = yfield(q, sl(2), c);
                    }
                    d[2 * q] = S::diff(m2, m1, p1, p2);
                    d[2 * q + 1] = S::diff(ym2, yfield(q, sl(-1), c), yfield(q, sl(1), c), yp2);
                }
                fd_node_fstar<C, FORCE>(w[0][cs][c], jxa[c], jya[c], d, a.k, f[c]);
            }
            }
            // populations moving along +x come from the column on the left, along -x from
            // the column on the right
            const C f1l = from_left(f[CPL - 1][1]), f5l = from_left(f[CPL - 1][5]), f8l = from_left(f[CPL - 1][8]);
            const C f3r = from_right(f[0][3]), f6r = from_right(f[0][6]), f7r = from_right(f[0][7]);
            const int os = sl(-DIR);  // window slot of the output row b = r - DIR
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
                // row sums leaving row r upward (to r + 1) and downward (to r - 1), and the
                // same groups of this node's own populations
                const C up = row_sum(f[c][2], u5, u6), upx = u5 - u6;
                const C dn = row_sum(f[c][4], d8, d7), dnx = d8 - d7;
                const C lu = row_sum(f[c][2], f[c][5], f[c][6]), lux = f[c][5] - f[c][6];
                const C ld = row_sum(f[c][4], f[c][8], f[c][7]), ldx = f[c][8] - f[c][7];
                const C fw = DIR > 0 ? up : dn, fwx = DIR > 0 ? upx : dnx;  // forward
                const C bw = DIR > 0 ? dn : up, bwx = DIR > 0 ? dnx : upx;  // backward
                const C lf = DIR > 0 ? lu : ld, lfx = DIR > 0 ? lux : ldx;  // own, forward group
                const C lb = DIR > 0 ? ld : lu, lbx = DIR > 0 ? ldx : lux;  // own, backward group
                C pc, pcx;
                same_row_part<C>(c1 - f[c][1], c3 - f[c][3], pc, pcx);
                const C pF = FW[c] - lf, pFx = FWX[c] - lfx;  // row r, from the row before it
                const C pB = bw - LB[c], pBx = bwx - LBX[c];  // row b, from row r
                if (!start_edge && it == 0) {
                    // f* of the first row: its backward sums complete the first output row
                    // of the neighbour across the start side, which sends its own back
                    lds[wv][START_S][c][lane] = bw;
                    lds[wv][START_SX][c][lane] = bwx;
                    lds[wv][OWN_PC][c][lane] = pc;
                    lds[wv][OWN_PCX][c][lane] = pcx;
                    lds[wv][OWN_L][c][lane] = lf;
                    lds[wv][OWN_LX][c][lane] = lfx;
                    lds[wv][OWN_R][c][lane] = w[0][cs][c];
                    lds[wv][OWN_X][c][lane] = w[1][cs][c];
                    lds[wv][OWN_Y][c][lane] = w[2][cs][c];
                }
                if (!start_edge && it == 1) {
                    lds[wv][OWN_P2][c][lane] = pB;
                    lds[wv][OWN_P2X][c][lane] = pBx;
                }
                // output row b
                C nr, nxv, nyv;
                if constexpr (DIR > 0)
                    fd_finish<C, FORCE>(QP[c], pB, pBx, w[0][os][c], w[1][os][c], w[2][os][c], a.k.dfx, a.k.dfy, nr,
                                        nxv, nyv);
                else
                    fd_finish<C, FORCE>(fd_partial<C>(PC[c], PCX[c], pB, pBx), PF[c], PFX[c], w[0][os][c],
                                        w[1][os][c], w[2][os][c], a.k.dfx, a.k.dfy, nr, nxv, nyv);
                round_out(min(max(first + DIR * (it - 1), 0), ny - 1), c, nr, nxv, nyv, gr.v[c], gx.v[c], gy.v[c]);
                if constexpr (DIR > 0) {
                    QP[c] = fd_partial<C>(pc, pcx, pF, pFx);
                } else {
                    PC[c] = pc;
                    PCX[c] = pcx;
                    PF[c] = pF;
                    PFX[c] = pFx;
                }
                FW[c] = fw;
                FWX[c] = fwx;
                LB[c] = lb;
                LBX[c] = lbx;
            }
            // output row b is complete once f* of the rows on both sides of it are known
            {
                const int orow = min(max(first + DIR * (it - 1), 0), ny - 1);
                row_store<T, CPL, AM>(row_rsrc(a.odr, orow, 3 * nx, nx), lc, it >= 2, gr);
                row_store<T, CPL, AM>(row_rsrc(a.ojx, orow, 3 * nx, nx), lc, it >= 2, gx);
                row_store<T, CPL, AM>(row_rsrc(a.ojy, orow, 3 * nx, nx), lc, it >= 2, gy);
            }
        }
    }
    // stored values of the last output row in sweep order (end side), completed after the
    // barrier: loaded again (it was loaded a row or two ago and is still in cache)
    const int last = first + DIR * (nf - 1);
    Group<T, CPL> o1r, o1x, o1y;
    if (!empty && !end_edge) {
        o1r = row_load<T, CPL, AM>(row_rsrc(a.dr, last, 3 * nx, nx), lc, true);
        o1x = row_load<T, CPL, AM>(row_rsrc(a.jx, last, 3 * nx, nx), lc, true);
        o1y = row_load<T, CPL, AM>(row_rsrc(a.jy, last, 3 * nx, nx), lc, true);
        // the forward sums of the last f* row complete the last output row of the
        // neighbour across the end side
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            lds[wv][END_S][c][lane] = FW[c];
            lds[wv][END_SX][c][lane] = FWX[c];
        }
    }
    __syncthreads();
    if (empty) return;
    if (!start_edge) {
        // first output row: own same-row and next-row parts, and the sums sent across the
        // start side by the neighbour there
        const int nb = wv - DIR;
        Group<T, CPL> gr, gx, gy;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const C pF = lds[nb][START_S][c][lane] - lds[wv][OWN_L][c][lane];
            const C pFx = lds[nb][START_SX][c][lane] - lds[wv][OWN_LX][c][lane];
            const C pc = lds[wv][OWN_PC][c][lane], pcx = lds[wv][OWN_PCX][c][lane];
            const C p2 = lds[wv][OWN_P2][c][lane], p2x = lds[wv][OWN_P2X][c][lane];
            const C odr = lds[wv][OWN_R][c][lane], ojx = lds[wv][OWN_X][c][lane], ojy = lds[wv][OWN_Y][c][lane];
            C nr, nxv, nyv;
            if constexpr (DIR > 0)
                fd_finish<C, FORCE>(fd_partial<C>(pc, pcx, pF, pFx), p2, p2x, odr, ojx, ojy, a.k.dfx, a.k.dfy, nr,
                                    nxv, nyv);
            else
                fd_finish<C, FORCE>(fd_partial<C>(pc, pcx, p2, p2x), pF, pFx, odr, ojx, ojy, a.k.dfx, a.k.dfy, nr,
                                    nxv, nyv);
            round_out(first, c, nr, nxv, nyv, gr.v[c], gx.v[c], gy.v[c]);
        }
        row_store<T, CPL, AM>(row_rsrc(a.odr, first, 3 * nx, nx), lc, true, gr);
        row_store<T, CPL, AM>(row_rsrc(a.ojx, first, 3 * nx, nx), lc, true, gx);
        row_store<T, CPL, AM>(row_rsrc(a.ojy, first, 3 * nx, nx), lc, true, gy);
    }
    if (!end_edge) {
        // last output row: carried parts and the sums sent across the end side
        const int nb = wv + DIR;
        Group<T, CPL> gr, gx, gy;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const C pB = lds[nb][END_S][c][lane] - LB[c];
            const C pBx = lds[nb][END_SX][c][lane] - LBX[c];
            C nr, nxv, nyv;
            if constexpr (DIR > 0)
                fd_finish<C, FORCE>(QP[c], pB, pBx, Storage<T>::load(o1r.v[c]), Storage<T>::load(o1x.v[c]),
                                    Storage<T>::load(o1y.v[c]), a.k.dfx, a.k.dfy, nr, nxv, nyv);
            else
                fd_finish<C, FORCE>(fd_partial<C>(PC[c], PCX[c], pB, pBx), PF[c], PFX[c], Storage<T>::load(o1r.v[c]),
                                    Storage<T>::load(o1x.v[c]), Storage<T>::load(o1y.v[c]), a.k.dfx, a.k.dfy, nr,
                                    nxv, nyv);
            round_out(last, c, nr, nxv, nyv, gr.v[c], gx.v[c], gy.v[c]);
        }
        row_store<T, CPL, AM>(row_rsrc(a.odr, last, 3 * nx, nx), lc, true, gr);
        row_store<T, CPL, AM>(row_rsrc(a.ojx, last, 3 * nx, nx), lc, true, gx);
        row_store<T, CPL, AM>(row_rsrc(a.ojy, last, 3 * nx, nx), lc, true, gy);
    }
}

// One tile: the block's WV wavefronts over row band `band` of the column strip that stores
// columns [x0, x0 + S) of one grid (`last`: the grid's last strip, reaching column nx - 1).
// Called by every wavefront of the block (it contains a block barrier).
template <typename T, int CPL, int ST, bool WALLS, bool FORCE, int AM>
__device__ __forceinline__ void sweep_tile(const TileArgs<T> &a, int band, int x0, bool last)
{
    using C = typename Storage<T>::C;
    using G = Strip<CPL, Stencil<ST>::H>;
    static_assert(CPL >= 2 || ST != 5, "5-point differences need two columns per lane");
    __shared__ C lds[WV][NSLOT][CPL][64];

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nx = a.nx, ny = a.ny;
    // first column of this lane (unwrapped).  With element-aligned accesses the last strip of
    // a grid wider than one strip is shifted left to end at column nx - 1: no lane's columns
    // then cross the periodic edge (it falls between lanes), so no lane needs the per-column
    // path.  The columns it shares with the strip before it are computed by both, from the
    // same inputs in the same order, and both store the same bits there.
    const bool shift_last = AM == AM_UNAL && last && nx > G::S;
    const int xl = (shift_last ? nx - G::S : x0) - G::P + CPL * lane;
    const bool stored = CPL * lane >= G::P && CPL * lane < G::P + G::S;  // the strip's own columns
    static_assert(AM != AM_UNAL || sizeof(T) >= 4, "element-aligned vector accesses need 4- or 8-byte elements");
    const LaneCols<CPL, AM> lc = make_lane_cols<T, CPL, AM>(xl, nx, stored);

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
    if (wv & 1)
        sweep_wave<1, T, CPL, ST, WALLS, FORCE, AM>(a, lds, wv, lane, lc, xl, ybeg, yend, empty, bottom, top);
    else
        sweep_wave<-1, T, CPL, ST, WALLS, FORCE, AM>(a, lds, wv, lane, lc, xl, ybeg, yend, empty, bottom, top);
}


// Host-side strip width of a (dtype, CPL, stencil) combination.
template <int CPL, int H> constexpr int strip_stride() { return Strip<CPL, H>::S; }

template <typename C> inline FdCoef<C> make_coef(int stencil, double s_xx, double s_e, double fx, double fy)
{
    const double scale = stencil == 3 ? Stencil<3>::SCALE : Stencil<5>::SCALE;
    FdCoef<C> k;
    const double ke = 2.0 * scale * (1.0 - 1.0 / s_e);
    k.eax = C(-ke / 36.0);
    k.edg = C(ke / 18.0);
    k.e0 = C(-ke / 9.0);
    k.kxx = C(scale * (1.0 - 1.0 / s_xx));
    k.kxx2 = C(2.0 * scale * (1.0 - 1.0 / s_xx));
    k.hfx = C(0.5 * fx);
    k.hfy = C(0.5 * fy);
    k.qfx = C(0.25 * fx);
    k.qfy = C(0.25 * fy);
    k.dfx = C(fx);
    k.dfy = C(fy);
    k.lin = C(2.0 / s_xx - 1.0);
    return k;
}

}  // namespace sweep
}  // namespace fdlbm
