// Device-side building blocks shared by the FD-LBM kernels: storage types, the per-node
// reconstruction of the post-collision populations (section 2 of Dubois, Lallemand,
// Obrecht, Tekitek) and the update order of the propagation (section 1, eq. 2).
//
// Every kernel that advances an FD-LBM state calls fd_node_fstar() with the same inputs
// in the same order, and forms the new state with row_sum(), same_row_part(), fd_partial()
// and fd_finish()
// in the same order, so the reference and the fused kernels produce bit-identical states.
// The library is compiled with -ffp-contract=off; every fused multiply-add below is
// written out.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdlbm {

// ------------------------------------------------------------------ storage types ----
template <typename T> struct Storage;
// store() rounds to nearest; store_r(v, r) is the rounding a step uses for its new state,
// given 13 random bits r (used only where STOCHASTIC).
template <> struct Storage<double> {
    using C = double;  // arithmetic type
    static constexpr bool STOCHASTIC = false;
    static __device__ __forceinline__ double load(double v) { return v; }
    static __device__ __forceinline__ double store(double v) { return v; }
    static __device__ __forceinline__ double store_r(double v, uint32_t) { return v; }
};
template <> struct Storage<float> {
    using C = float;
    static constexpr bool STOCHASTIC = false;
    static __device__ __forceinline__ float load(float v) { return v; }
    static __device__ __forceinline__ float store(float v) { return v; }
    static __device__ __forceinline__ float store_r(float v, uint32_t) { return v; }
};
template <> struct Storage<__half> {
    using C = float;
    static constexpr bool STOCHASTIC = false;
    static __device__ __forceinline__ float load(__half v) { return __half2float(v); }
    static __device__ __forceinline__ __half store(float v) { return __float2half_rn(v); }
    static __device__ __forceinline__ __half store_r(float v, uint32_t) { return __float2half_rn(v); }
};

// FP16 deviations whose new values are rounded stochastically: up or down to the two
// neighbouring FP16 values with probabilities proportional to the distance to the other one,
// so the rounding is unbiased and an increment smaller than half a unit of the stored value
// is kept on average instead of being lost every step.  For a value in the FP16 normal range
// one FP16 unit spans 2^13 units of its FP32 pattern; adding r - 2^12 (r uniform in
// [0, 2^13)) to that pattern and rounding to nearest gives floor((m + r) / 2^13) for the
// magnitude bits m, which rounds up with probability (m mod 2^13) / 2^13.  Below the FP16
// normal range only the lowest 13 of the dropped bits are randomised.  Loads, set_state and
// the boundary fills round to nearest.
struct HalfSR {
    __half h;
};
template <> struct Storage<HalfSR> {
    using C = float;
    static constexpr bool STOCHASTIC = true;
    static __device__ __forceinline__ float load(HalfSR v) { return __half2float(v.h); }
    static __device__ __forceinline__ HalfSR store(float v) { return HalfSR{__float2half_rn(v)}; }
    static __device__ __forceinline__ HalfSR store_r(float v, uint32_t r)
    {
        uint32_t b = __builtin_bit_cast(uint32_t, v);
        // sign and magnitude: the addition moves |v| (patterns this small are zero in FP16)
        if ((b & 0x7fffffffu) >= 0x1000u) b = b + r - 0x1000u;
        return HalfSR{__float2half_rn(__builtin_bit_cast(float, b))};
    }
};

// The PCG hash of Jarzynski and Olano ("Hash functions for GPU rendering", JCGT 9(3),
// 2020): one round of a PCG generator with an output permutation, as a 32-bit to 32-bit
// map.  The random bits of stochastic rounding are counter-based: node index and step.
__host__ __device__ __forceinline__ uint32_t pcg_hash(uint32_t x)
{
    const uint32_t state = x * 747796405u + 2891336453u;
    const uint32_t word = ((state >> ((state >> 28u) + 4u)) ^ state) * 277803737u;
    return (word >> 22u) ^ word;
}
// 13 random bits for each of drho, jx, jy of node `node` (linear index j*nx + i, modulo
// 2^32) at the step whose seed is `seed` (pcg_hash of the step count).
__device__ __forceinline__ void sr_draw(uint32_t node, uint32_t seed, uint32_t (&r)[3])
{
    const uint32_t h0 = pcg_hash(node ^ seed);
    const uint32_t h1 = pcg_hash(h0);
    r[0] = h0 & 0x1fffu;
    r[1] = (h0 >> 16) & 0x1fffu;
    r[2] = h1 & 0x1fffu;
}

// Layout of a state of NF fields in HBM: row-interleaved, row j of field f starting at
// element (NF j + f) nx, so that the rows a sweep reads (and writes) together are adjacent.
// HBM serves three adjacent rows about 12 % faster than three rows in separate planes (a
// plain copy of 8192^2 FP32 fields: 6.09 against 5.43 TB/s); the FD-LBM step runs 6 % and
// the MRT step 11 % faster than with planes (8192^2, FP32).  Element of node (i, j), field f:
template <int NF> __host__ __device__ __forceinline__ size_t row_elem(size_t i, size_t j, int f, size_t nx)
{
    return (NF * j + f) * nx + i;
}
// the three-word state (drho, Jx, Jy) of FD-LBM and LW-ACM
__host__ __device__ __forceinline__ size_t fd_elem(size_t i, size_t j, int f, size_t nx) { return row_elem<3>(i, j, f, nx); }
// the nine populations f_k - w_k of MRT
__host__ __device__ __forceinline__ size_t pop_elem(size_t i, size_t j, int k, size_t nx) { return row_elem<9>(i, j, k, nx); }

__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/rho.  FP32 uses the hardware reciprocal (1 ulp); FP64 the IEEE division.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Finite differences of section 2 in unscaled form.  With g(+-1), g(+-2) the values at the
// neighbours along one axis:
//   3 points: D = g(+1) - g(-1)                    (derivative = D / 2)
//   5 points: D = 6 (g(+1) - g(-1)) - (g(+2) - g(-2))  (derivative = D / 8,
//             i.e. 3/4 (g(+1) - g(-1)) - 1/8 (g(+2) - g(-2)))
// The theta terms are linear in the derivatives, so the power-of-two scale is folded into
// the relaxation factors, which is exact.
template <int STENCIL> struct Stencil;
// The LW-ACM step (section 1-b) runs on the same kernels as "stencil 1": it takes no
// differences, so a node's populations depend on the node alone (half width 0).
template <> struct Stencil<1> {
    static constexpr int H = 0;
    static constexpr double SCALE = 0.5;
    template <typename C> static __device__ __forceinline__ C diff(C, C, C, C) { return C(0); }
};
template <> struct Stencil<3> {
    static constexpr int H = 1;  // half width
    static constexpr double SCALE = 0.5;
    template <typename C> static __device__ __forceinline__ C diff(C m2, C m1, C p1, C p2) {
        (void)m2; (void)p2;
        return p1 - m1;
    }
};
template <> struct Stencil<5> {
    static constexpr int H = 2;
    static constexpr double SCALE = 0.125;
    template <typename C> static __device__ __forceinline__ C diff(C m2, C m1, C p1, C p2) {
        return fmac(C(6), p1 - m1, -(p2 - m2));
    }
};

// Ghost rows beyond a wall at distance xi past the last fluid row (0 < xi <= 1; sections
// 3-b and 3-c).  The ghost node at distance d beyond the wall takes the value at its mirror
// point, d inside the fluid, with the velocity negated: linear extrapolation with zero
// velocity on the wall.  The mirror value is interpolated between the fluid rows around it,
// or, between the wall and the last fluid row, between zero velocity on the wall and that
// row (the density taken from that row); the case depends on where the wall cuts the link,
// as in Bouzidi et al.  Ghost row g (g = 1, 2, 3 rows beyond the last fluid row) holds
//   drho = car v(sa) + cbr v(sb),   J = caj v(sa) + cbj v(sb)
// with fluid rows sa, sb counted from the wall (0 = the last fluid row); sb < 0: one row.
// At xi = 1/2 ghost row g is fluid row g - 1 with J negated (car = 1, caj = -1).
constexpr int NGHOST = 3;
template <typename C> struct GhostRule {
    int sa, sb;
    C car, caj, cbr, cbj;
};
template <typename C> struct GhostRules {
    GhostRule<C> g[NGHOST];
};
template <typename C> inline GhostRules<C> ghost_rules(double xi)
{
    GhostRules<C> r;
    for (int g = 1; g <= NGHOST; ++g) {
        GhostRule<C> &q = r.g[g - 1];
        const double ym = g - 2.0 * xi;  // mirror point, rows inside the last fluid row
        if (ym >= 0.0) {
            const int s0 = (int)ym;
            const double t = ym - s0;
            q.sa = s0;
            q.car = C(1.0 - t);
            q.caj = C(-(1.0 - t));
            if (t == 0.0) {
                q.sb = -1;
                q.cbr = q.cbj = C(0);
            } else {
                q.sb = s0 + 1;
                q.cbr = C(t);
                q.cbj = C(-t);
            }
        } else {
            q.sa = 0;
            q.sb = -1;
            q.car = C(1);
            q.caj = C(-(ym + xi) / xi);
            q.cbr = q.cbj = C(0);
        }
    }
    return r;
}
// The rule of the ghost row at distance g (clamped to the table; rows past the third
// ghost row are never used), selected without indexing the table dynamically.
template <typename C> __device__ __forceinline__ GhostRule<C> ghost_rule(const GhostRules<C> &r, int g)
{
    return g <= 1 ? r.g[0] : g == 2 ? r.g[1] : r.g[2];
}

// x + f for the force terms: a run without body force drops the additions (its kernels are
// instantiated with FORCE = false; adding a zero changes no value).
template <bool FORCE, typename C> __device__ __forceinline__ C plus_force(C x, C f) { return FORCE ? x + f : x; }

// Per-step constants of the reconstruction.
template <typename C> struct FdCoef {
    // (1 - 1/s_e) theta_E enters the populations with the weights -1/36 (axes), 1/18
    // (diagonals) and -1/9 (rest); with the derivative scale, per unit of theta_E / 2:
    C eax;    // -2 SCALE (1 - 1/s_e) / 36
    C edg;    //  2 SCALE (1 - 1/s_e) / 18
    C e0;     // -2 SCALE (1 - 1/s_e) / 9
    C kxx;    // SCALE * (1 - 1/s_xx)  multiplies theta_XY
    C kxx2;   // 2 kxx                 multiplies theta_XX / 2
    C hfx, hfy;  // F/2: J_a = J + F/2 (Strang splitting, section 1)
    C qfx, qfy;  // F/4: axis populations carry (J_a + F/4)/3
    C dfx, dfy;  // F  : diagonal populations carry (J_a + F)/12
    C lin;       // LW-ACM: 1 - Theta = 6 nu = 2/s_xx - 1 (see lw_node_g)
};

// Inputs of one node: J_a = J + F/2 and the ten unscaled derivatives (of drho, of the
// stored J and of the products of J_a)
//   d[0] = D_x rho, d[1] = D_y rho, d[2] = D_x Jx, d[3] = D_y Jy, d[4] = D_x Jy,
//   d[5] = D_y Jx, d[6] = D_x Jx^2, d[7] = D_y JxJy, d[8] = D_x JxJy, d[9] = D_y Jy^2.
// Output: the nine post-collision populations as deviations f*_k - w_k.
//
// Section 2: theta_E, theta_XX, theta_XY (the defects of conservation at rho close to 1,
// with v read as the stored momentum, the linear part of theta_XY as
// (1/3)(d_x J_y + d_y J_x), and theta_E = (2 - 6|J|^2) div J - 2 J.grad rho, the sign of
// whose cubic term gives the bulk viscosity zeta (1 - 3V^2) in a mean flow that section 2
// states); post-collision moments
//   E = -2 rho + 3|J|^2/rho + (1 - 1/s_e) theta_E,  XX = (Jx^2 - Jy^2)/rho + (1 - 1/s_xx) theta_XX,
//   XY = Jx Jy/rho + (1 - 1/s_xx) theta_XY,  q = -J,  eps = rho - 3|J|^2/rho;
// then f* = M^{-1} m* written out per velocity (M^{-1} = M^T diag(1/9, 1/6, 1/6, 1/36,
// 1/4, 1/4, 1/12, 1/12, 1/36), section 1), as deviations from the rest populations.
template <typename C, bool FORCE>
__device__ __forceinline__ void fd_node_fstar(C dr, C jx, C jy, const C (&d)[10], const FdCoef<C> &k, C (&f)[9])
{
    const C rx = d[0], ry = d[1], a = d[2], b = d[3], c = d[4], dd = d[5];
    const C sA = d[6] + d[7];  // D_x Jx^2 + D_y JxJy
    const C sB = d[8] + d[9];  // D_x JxJy + D_y Jy^2
    const C p0 = jx * jx, q0 = jy * jy, r0 = jx * jy;
    const C j2 = p0 + q0;

    const C w = fmac(jx, rx, jy * ry);                               // J . grad rho
    const C th_e_h = fmac(fmac(C(-3), j2, C(1)), a + b, -w);        // theta_E / 2
    // Jx and Jy enter theta_XX and theta_XY only through rx / 3 + sA and ry / 3 + sB:
    //   theta_XX / 2 = 1/3 (D_x Jx - D_y Jy) - (Jx wx - Jy wy)
    //   theta_XY     = 1/3 (D_x Jy + D_y Jx) - (Jx wy + Jy wx)
    const C wx = fmac(rx, C(1.0 / 3.0), sA), wy = fmac(ry, C(1.0 / 3.0), sB);
    const C th_xx_h = fmac(C(1.0 / 3.0), a - b, -fmac(jx, wx, -(jy * wy)));
    const C th_xy = fmac(C(1.0 / 3.0), c + dd, -fmac(jx, wy, jy * wx));

    const C rinv = recip(C(1) + dr);
    const C K = j2 * rinv;
    const C XX = fmac(p0 - q0, rinv, k.kxx2 * th_xx_h);
    const C XY = fmac(r0, rinv, k.kxx * th_xy);

    // deviation populations (rest moments m0 = (1,0,0,-2,0,0,0,0,1) removed)
    const C k12 = K * C(1.0 / 12.0);
    const C A_ax = fmac(dr, C(1.0 / 9.0), fmac(th_e_h, k.eax, k12));
    const C A_dg = fmac(dr, C(1.0 / 36.0), fmac(th_e_h, k.edg, k12));
    f[0] = fmac(dr, C(4.0 / 9.0), fmac(K, C(-2.0 / 3.0), th_e_h * k.e0));
    // the odd parts (J/3 on the axes, (+-Jx +-Jy)/12 on the diagonals) enter through fused
    // multiply-adds with the constant: one instruction per population
    const C axp = fmac(XX, C(0.25), A_ax), axm = fmac(XX, C(-0.25), A_ax);
    const C ux = plus_force<FORCE>(jx, k.qfx), uy = plus_force<FORCE>(jy, k.qfy);
    f[1] = fmac(ux, C(1.0 / 3.0), axp);
    f[3] = fmac(ux, C(-1.0 / 3.0), axp);
    f[2] = fmac(uy, C(1.0 / 3.0), axm);
    f[4] = fmac(uy, C(-1.0 / 3.0), axm);
    const C dgp = fmac(XY, C(0.25), A_dg), dgm = fmac(XY, C(-0.25), A_dg);
    const C vx = plus_force<FORCE>(jx, k.dfx), vy = plus_force<FORCE>(jy, k.dfy);
    const C s = vx + vy, t = vy - vx;
    f[5] = fmac(s, C(1.0 / 12.0), dgp);
    f[7] = fmac(s, C(-1.0 / 12.0), dgp);
    f[6] = fmac(t, C(1.0 / 12.0), dgm);
    f[8] = fmac(t, C(-1.0 / 12.0), dgm);
}

// LW-ACM (section 1-b): f*_k(x) = f^eq_k(x) + Theta (f^eo_k(x + e_k) - f^eo_k(x)) with
// Theta = 1 - 6 nu, and f* propagates to x + e_k.  Regrouped by the node it depends on, the
// population that arrives at x along k is g_k(x - e_k) + Theta f^eo_k(x) with
// g_k = f^eq_k - Theta f^eo_k.  f^eo (the part of f^eq odd in J) carries no mass and
// momentum J, so the node's own term adds Theta J(x) to J; g carries drho and lin J with
// lin = 1 - Theta.  The update is therefore the FD-LBM one of fd_partial() / fd_finish()
// with g in place of f*: new = old + sum_k [g_k(x - e_k) - g_k(x)] for drho and for J.
// f^eo is linear in J, so g is the equilibrium of the section 1-a table with its linear
// part scaled by lin.  Output: the nine g_k as deviations from the rest populations.
template <typename C> __device__ __forceinline__ void lw_node_g(C dr, C jx, C jy, C lin, C (&f)[9])
{
    const C p0 = jx * jx, q0 = jy * jy, r0 = jx * jy;
    const C rinv = recip(C(1) + dr);
    const C K = (p0 + q0) * rinv;  // |J|^2 / rho
    const C XX = (p0 - q0) * rinv, XY = r0 * rinv;
    const C k12 = K * C(1.0 / 12.0);
    const C A_ax = fmac(dr, C(1.0 / 9.0), k12);
    const C A_dg = fmac(dr, C(1.0 / 36.0), k12);
    f[0] = fmac(dr, C(4.0 / 9.0), K * C(-2.0 / 3.0));
    const C axp = fmac(XX, C(0.25), A_ax), axm = fmac(XX, C(-0.25), A_ax);
    const C ux = lin * jx, uy = lin * jy;
    f[1] = fmac(ux, C(1.0 / 3.0), axp);
    f[3] = fmac(ux, C(-1.0 / 3.0), axp);
    f[2] = fmac(uy, C(1.0 / 3.0), axm);
    f[4] = fmac(uy, C(-1.0 / 3.0), axm);
    const C dgp = fmac(XY, C(0.25), A_dg), dgm = fmac(XY, C(-0.25), A_dg);
    const C s = ux + uy, t = uy - ux;
    f[5] = fmac(s, C(1.0 / 12.0), dgp);
    f[7] = fmac(s, C(-1.0 / 12.0), dgp);
    f[6] = fmac(t, C(1.0 / 12.0), dgm);
    f[8] = fmac(t, C(-1.0 / 12.0), dgm);
}

// Propagation (eq. 2) in increment form.  The new state at x sums f*_k(x - e_k); the
// collision conserves mass and adds F to the momentum, so the node's own populations sum
// to sum_k f*_k(x) = drho(x) and sum_k e_k f*_k(x) = J(x) + F, and
//   drho' = drho + sum_k [f*_k(x - e_k) - f*_k(x)],   J' = J + F + sum_k e_k [f*_k(x - e_k) - f*_k(x)].
// The populations are grouped by the row they come from:
//   same row   f1(x - ex), f3(x + ex)                       (f0 stays: no change)
//   row below  f2(x - ey), f5(x - ex - ey), f6(x + ex - ey)
//   row above  f4(x + ey), f8(x - ex + ey), f7(x + ex + ey)
// In the same row each arriving population is compared with the node's own one; the two
// other rows are summed (middle, from the left, from the right) and the same sum of the
// node's own populations is subtracted.  The three small differences are added to the
// stored value last.  Summing the nine arriving populations directly rounds at the scale
// of the field every step, and because the rounded weights 1/9, 1/36, 1/3, 1/12 do not
// add up to exactly one in FP32, a slowly varying field then drifts by about 3e-8 per step.
template <typename C> __device__ __forceinline__ C row_sum(C mid, C from_l, C from_r) { return (mid + from_l) + from_r; }

// Same-row part from e1 = f1(x - ex) - f1(x) and e3 = f3(x + ex) - f3(x): drho and Jx parts.
template <typename C> __device__ __forceinline__ void same_row_part(C e1, C e3, C &pc, C &pcx)
{
    pc = e1 + e3;
    pcx = e1 - e3;
}

// The update in two halves, so that a kernel which meets the three source rows at
// different times forms exactly the same sums.  pc, pu, pd: (arriving - own) for drho from
// the same row, the row below and the row above; pcx, pux, pdx the same for Jx (Jy takes
// pu - pd).  fd_finish adds the row-above part, the body force (fx, fy) and the stored
// state (odr, ojx, ojy).
template <typename C> struct FdPartial {
    C q, qx, pu;
};
template <typename C> __device__ __forceinline__ FdPartial<C> fd_partial(C pc, C pcx, C pu, C pux)
{
    return FdPartial<C>{pc + pu, pcx + pux, pu};
}
template <typename C, bool FORCE>
__device__ __forceinline__ void fd_finish(const FdPartial<C> &a, C pd, C pdx, C odr, C ojx, C ojy, C fx, C fy, C &dr,
                                          C &jx, C &jy)
{
    dr = odr + (a.q + pd);
    jx = ojx + plus_force<FORCE>(a.qx + pdx, fx);
    jy = ojy + plus_force<FORCE>(a.pu - pd, fy);
}

}  // namespace fdlbm
