// Per-node arithmetic of the FD-LBM step on the D3Q19 lattice: the construction of section 2
// (post-collision moments = equilibrium + (1 - 1/s) theta, theta the defect of conservation
// at rho close to 1, f* = M^{-1} m*, propagation by eq. 2) carried over to the 19 velocities
// of D3Q19 and their polynomial moment basis (d'Humieres et al. 2002).
//
// Both the reference kernels and the sweep kernel call d3_fstar() with the same inputs and
// form the new state with the d3_* update helpers in the same order, so they agree bit for
// bit.  Compiled with -ffp-contract=off: every fused multiply-add is written out.
#pragma once

#include "fdlbm_device.hpp"

namespace fdlbm {
namespace d3 {

// Velocity order: 0 rest; 1..6 = +x, -x, +y, -y, +z, -z; 7..18 the edges
// (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
// (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1).  Population 0 never moves and is not formed.
constexpr int Q = 19;

// Per-step constants.  The differences are unscaled (g(+1) - g(-1), twice the derivative) and
// the factor 1/2 is folded in here, as are the norms of the moment rows and the weights the
// corrections enter the populations with:
//   energy e = 19|c|^2 - 30, |e|^2 = 2394, weight -11 on faces and 8 on edges;
//   3p_xx = 3c_x^2 - |c|^2, |.|^2 = 36; p_ww = c_y^2 - c_z^2, |.|^2 = 12;
//   p_xy, p_yz, p_xz, |.|^2 = 4.
template <typename C> struct Coef3 {
    C kf;   // -11 (1 - 1/s_e) / 252 = -11 (1 - 1/s_e) 19 / (2 * 2394): energy, faces, times 2/3
            // (per unit of te_h = 3/2 te, below)
    C kd;   //   8 (1 - 1/s_e) / 252 times 2/3: energy, edges
    C kp;   // (1 - 1/s_nu) / 36: 3p_xx per unit of the half diagonal defects h_aa = u_aa / 2
    C k2p;  // 2 kp
    C kw;   // (1 - 1/s_nu) / 12: p_ww per unit of h_aa
    C ko;   // (1 - 1/s_nu) / 8 : p_xy, p_yz, p_xz per unit of u_ab
};
template <typename C> inline Coef3<C> coef3(double s_nu, double s_e)
{
    const double a = 1.0 - 1.0 / s_e, b = 1.0 - 1.0 / s_nu;
    return Coef3<C>{C(-11.0 * a / 252.0 * (2.0 / 3.0)), C(8.0 * a / 252.0 * (2.0 / 3.0)), C(b / 36.0), C(b / 18.0),
                    C(b / 12.0), C(b / 8.0)};
}

// a b - c d, the difference of a product between the two neighbours along an axis
template <typename C> __device__ __forceinline__ C d3_pdiff(C a, C b, C c, C d) { return fmac(a, b, -(c * d)); }

// Inputs of one node: the stored deviations and the unscaled differences
//   gr[a] = D_a drho,  dj[a][b] = D_a J_b,  dp[a] = (D_x(J_a J_x) + D_y(J_a J_y)) + D_z(J_a J_z).
// Output f[1..18]: post-collision populations as deviations f*_q - w_q.
//
// Defects (unscaled, u = 2 theta):
//   u_ab = 1/3 [(D_a J_b + D_b J_a) - (J_a D_b rho + J_b D_a rho)] - (J_a dp_b + J_b dp_a)
//   te   = (2/3 - 2|J|^2) div J - 2/3 J.grad rho    (the energy's trace term)
// Corrections of the second-order moments, per population (columns of M^{-1} = M^T / norms),
// with h_aa = u_aa / 2:
//   fe = kf te, ee = kd te, pp = kp (2h_xx - h_yy - h_zz), pw = kw (h_yy - h_zz), p_ab = ko u_ab
// (te is formed as te_h = 3/2 te, with kf and kd scaled to match; kp and kw are applied where
// pp and pw enter the populations)
//   face x: fe + 2pp         face y: fe - pp + pw        face z: fe - pp - pw
//   edge xy: ee + pp + pw +- p_xy    edge xz: ee + pp - pw +- p_xz    edge yz: ee - 2pp +- p_yz
// Equilibrium (deviations), with T = drho - 3/2 |J|^2/rho and Q_ab = J_a J_b / rho:
//   face +-a: T/18 + Q_aa/4 +- J_a/6
//   edge (s_a, s_b): T/36 + (Q_aa + Q_bb)/8 + s_a s_b Q_ab/4 + (s_a J_a + s_b J_b)/12
template <typename C>
__device__ __forceinline__ void d3_fstar(C dr, const C (&j)[3], const C (&gr)[3], const C (&dj)[3][3], const C (&dp)[3],
                                         const Coef3<C> &k, C (&f)[Q])
{
    const C third = C(1.0 / 3.0);
    // J_b multiplies D_b rho / 3 + dp_b wherever it appears in the defects: w_b
    const C w0 = fmac(gr[0], third, dp[0]), w1 = fmac(gr[1], third, dp[1]), w2 = fmac(gr[2], third, dp[2]);
    // half diagonal defects h_aa = u_aa / 2 = 1/3 D_a J_a - J_a w_a
    const C hxx = fmac(third, dj[0][0], -(j[0] * w0));
    const C hyy = fmac(third, dj[1][1], -(j[1] * w1));
    const C hzz = fmac(third, dj[2][2], -(j[2] * w2));
    // off-diagonal defects u_ab = 1/3 (D_a J_b + D_b J_a) - (J_a w_b + J_b w_a)
    const C uxy = fmac(third, dj[0][1] + dj[1][0], -fmac(j[0], w1, j[1] * w0));
    const C uxz = fmac(third, dj[0][2] + dj[2][0], -fmac(j[0], w2, j[2] * w0));
    const C uyz = fmac(third, dj[1][2] + dj[2][1], -fmac(j[1], w2, j[2] * w1));
    const C pxx = j[0] * j[0], pyy = j[1] * j[1], pzz = j[2] * j[2];
    const C j2 = (pxx + pyy) + pzz;
    const C div = (dj[0][0] + dj[1][1]) + dj[2][2];
    const C jg = fmac(j[0], gr[0], fmac(j[1], gr[1], j[2] * gr[2]));
    const C te_h = fmac(fmac(C(-3), j2, C(1)), div, -jg);  // 3/2 te

    const C fe = k.kf * te_h, ee = k.kd * te_h;
    const C pq = fmac(C(2), hxx, -hyy - hzz);  // pp / kp
    const C wq = hyy - hzz;                    // pw / kw
    const C cxy = k.ko * uxy, cxz = k.ko * uxz, cyz = k.ko * uyz;

    const C rinv = recip(C(1) + dr);
    const C qxx = pxx * rinv, qyy = pyy * rinv, qzz = pzz * rinv;
    const C T = fmac(C(-1.5), (qxx + qyy) + qzz, dr);
    const C t18 = T * C(1.0 / 18.0), t36 = T * C(1.0 / 36.0);

    // faces
    const C fmp = fmac(-pq, k.kp, fe);  // fe - pp
    const C Fx = fmac(qxx, C(0.25), t18) + fmac(pq, k.k2p, fe);
    const C Fy = fmac(qyy, C(0.25), t18) + fmac(wq, k.kw, fmp);
    const C Fz = fmac(qzz, C(0.25), t18) + fmac(-wq, k.kw, fmp);
    f[1] = fmac(j[0], C(1.0 / 6.0), Fx);
    f[2] = fmac(j[0], C(-1.0 / 6.0), Fx);
    f[3] = fmac(j[1], C(1.0 / 6.0), Fy);
    f[4] = fmac(j[1], C(-1.0 / 6.0), Fy);
    f[5] = fmac(j[2], C(1.0 / 6.0), Fz);
    f[6] = fmac(j[2], C(-1.0 / 6.0), Fz);

    // edges
    const C hx = j[0] * C(1.0 / 12.0), hy = j[1] * C(1.0 / 12.0), hz = j[2] * C(1.0 / 12.0);
    const C epp = fmac(pq, k.kp, ee);  // ee + pp
    {
        const C B = fmac(qxx + qyy, C(0.125), t36) + fmac(wq, k.kw, epp);
        const C Cc = fmac(j[0] * j[1], C(0.25) * rinv, cxy);
        const C bp = B + Cc, bm = B - Cc, s = hx + hy, t = hx - hy;
        f[7] = bp + s;
        f[8] = bp - s;
        f[9] = bm + t;
        f[10] = bm - t;
    }
    {
        const C B = fmac(qxx + qzz, C(0.125), t36) + fmac(-wq, k.kw, epp);
        const C Cc = fmac(j[0] * j[2], C(0.25) * rinv, cxz);
        const C bp = B + Cc, bm = B - Cc, s = hx + hz, t = hx - hz;
        f[11] = bp + s;
        f[12] = bp - s;
        f[13] = bm + t;
        f[14] = bm - t;
    }
    {
        const C B = fmac(qyy + qzz, C(0.125), t36) + fmac(-pq, k.k2p, ee);
        const C Cc = fmac(j[1] * j[2], C(0.25) * rinv, cyz);
        const C bp = B + Cc, bm = B - Cc, s = hy + hz, t = hy - hz;
        f[15] = bp + s;
        f[16] = bp - s;
        f[17] = bm + t;
        f[18] = bm - t;
    }
    f[0] = C(0);
}

// dp[a] from the unscaled differences of the products along x, y and z.
template <typename C> __device__ __forceinline__ C d3_flux(C dxa, C dya, C dza) { return (dxa + dya) + dza; }

// ------------------------------------------------------------------ propagation ----
// The new state (eq. 2) in increment form, as for D2Q9: the node's own populations sum to
// drho and J, so drho' = drho + sum_q [f*_q(x - c_q) - f*_q(x)] and J' likewise with c_q.
// The populations are grouped by the row and plane they come from, (c_y, c_z):
//   (0,0)   f1 from x-1, f2 from x+1                       (same row and plane)
//   (1,0)   f3, f7 from x-1, f10 from x+1    (-1,0)  f4, f9 from x-1, f8 from x+1
//   (0,1)   f5, f11 from x-1, f14 from x+1   (0,-1)  f6, f13 from x-1, f12 from x+1
//   (1,1) f15   (-1,-1) f16   (1,-1) f17   (-1,1) f18
// A group of three is summed where it starts, with its x-shift: S = (mid + from_left) +
// from_right and X = from_left - from_right; the destination subtracts the same sums of its
// own populations.  The parts from the plane below (lo), the same plane (mid) and the plane
// above (hi) are added in that order, then the stored value.
template <typename C> __device__ __forceinline__ C d3_sum(C mid, C from_l, C from_r) { return (mid + from_l) + from_r; }

template <typename C> struct D3Part {
    C r, x, y, z;
};
// lo: dS, dX of group (0,1); d11, dm11 the differences of f15 and f18
template <typename C> __device__ __forceinline__ D3Part<C> d3_lo(C dS, C dX, C d11, C dm11)
{
    const C r = (dS + d11) + dm11;
    return D3Part<C>{r, dX, d11 - dm11, r};
}
// mid: e1 = f1(x-1) - f1(x), e2 = f2(x+1) - f2(x); dS, dX of groups (1,0) and (-1,0).  The
// sum of lo and mid is what the node keeps until the plane above has arrived.
template <typename C>
__device__ __forceinline__ D3Part<C> d3_lo_mid(const D3Part<C> &lo, C e1, C e2, C dS10, C dX10, C dSm10, C dXm10)
{
    const C r = ((e1 + e2) + dS10) + dSm10;
    const C x = ((e1 - e2) + dX10) + dXm10;
    const C y = dS10 - dSm10;
    return D3Part<C>{lo.r + r, lo.x + x, lo.y + y, lo.z};
}
// hi: dS, dX of group (0,-1); d1m1, dm1m1 the differences of f17 and f16.  Adds the stored
// state (o*) and returns the new one.
template <typename C>
__device__ __forceinline__ void d3_finish(const D3Part<C> &p, C dS, C dX, C d1m1, C dm1m1, C odr, C ojx, C ojy, C ojz,
                                          C &dr, C &jx, C &jy, C &jz)
{
    const C r = (dS + d1m1) + dm1m1;
    dr = odr + (p.r + r);
    jx = ojx + (p.x + dX);
    jy = ojy + (p.y + (d1m1 - dm1m1));
    jz = ojz + (p.z - r);
}

}  // namespace d3
}  // namespace fdlbm
