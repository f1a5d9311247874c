/*
 * FP64 CPU oracle for the FD-LBM step on the three-dimensional D3Q19 lattice: the model of
 * section 2 of Dubois, Lallemand, Obrecht and Tekitek (arXiv 1803.00437) carried over to
 * D3Q19, which the Conclusion says was analysed but whose expressions the paper does not
 * print.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the bench's CPU-baseline
 * leg may load it.  It shares no code, header or constant table with the HIP library.
 *
 * The construction is the one of section 2, applied to D3Q19 (readings D1-D5):
 *   D1  velocities and moments: the 19 velocities (rest, 6 faces, 12 edges) and the
 *       orthogonal polynomial moment basis of d'Humieres et al. (2002), the three-dimensional
 *       reference of the paper: rho, e = 19|c|^2 - 30, eps = (21|c|^4 - 53|c|^2 + 24)/2,
 *       j_a = c_a, q_a = (5|c|^2 - 9) c_a, 3p_xx = 3c_x^2 - |c|^2, 3pi_xx = (3|c|^2 - 5) 3p_xx,
 *       p_ww = c_y^2 - c_z^2, pi_ww = (3|c|^2 - 5) p_ww, p_xy, p_yz, p_xz = c_a c_b,
 *       m_x = c_x (c_y^2 - c_z^2), m_y = c_y (c_z^2 - c_x^2), m_z = c_z (c_x^2 - c_y^2);
 *   D2  equilibria: every non-conserved moment takes the value of the second-order
 *       polynomial equilibrium f^eq_k = w_k [rho + 3 c.J + 9/2 (c.J)^2/rho - 3/2 |J|^2/rho]
 *       (as the D2Q9 table of section 1-a does), w = 1/3, 1/18, 1/36;
 *   D3  the six second-order moments (e, 3p_xx, p_ww, p_xy, p_yz, p_xz) take
 *       m* = m^eq + (1 - 1/s) theta (eq. order2), s = s_e for e and s_nu for the other five;
 *       every other moment is at equilibrium (rate 1), as q and eps are in section 2;
 *   D4  theta of a second-order moment is the same combination of the defects of the stress
 *       components theta_ab, expanded at rho close to 1 with v read as J, exactly as the
 *       D2Q9 terms of section 2 are:
 *         theta_ab = 1/3 (d_a J_b + d_b J_a) - 1/3 (J_a d_b rho + J_b d_a rho)
 *                    - J_a D_b - J_b D_a,          D_a = sum_c d_c (J_a J_c),
 *       for 3p_xx, p_ww, p_xy, p_yz, p_xz; for the energy the trace
 *         tr = 2/3 div J - 2/3 J.grad rho - 2 |J|^2 div J,   theta_e = 19 tr
 *       (e = 19 tr Pi - 30 rho).  On a flow that does not depend on z with J_z = 0 these are
 *       the theta_XX, theta_XY and theta_E / 3 of section 2 (with the velocity-cubic term of
 *       the energy read as for D2Q9: the bulk viscosity in a mean flow V is zeta (1 - 3V^2));
 *   D5  derivatives are the 3-point centred differences of section 2, periodic in x, y, z.
 * The step then propagates f* (eq. 2) and keeps rho, J.
 *
 * What pins this file (tests/test_oracle_d3q19.py): the velocity set and weights against
 * the isotropy they must have; the moment rows against their polynomials and orthogonality;
 * conservation and fixed points; the reduction to textbook D3Q19 BGK with tau = 1 at unit
 * rates; its linear response against the independently written amplification matrix, whose
 * transport coefficients equal those of a brute-force D3Q19 MRT at order k^2 in every
 * direction (shear nu = (1/s_nu - 1/2)/3, sound speed 1/sqrt 3, bulk (2/9)(1/s_e - 1/2)),
 * whose shear viscosity in a mean flow is nu (1 - 3V^2) and whose bulk coefficient is
 * (1 - 3V^2)/2; the density-gradient terms against the defect a BGK step leaves.
 *
 * Conventions (all FP64): fields are nx*ny*nz arrays, x fastest: element (k*ny + j)*nx + i
 * is node (x=i, y=j, z=k).  The stored state is the deviation from rest: drho, jx, jy, jz.
 * Populations are deviations f_q - w_q.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q3 19

/* velocity order: rest; +x, -x, +y, -y, +z, -z; the twelve edges in opposite pairs */
static const int CX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

/* the six second-order rows of the basis (D1) */
enum { M3_E = 1, M3_PXX = 9, M3_PWW = 11, M3_PXY = 13, M3_PYZ = 14, M3_PXZ = 15 };

static double weight3(int q)
{
    const int c2 = CX3[q] * CX3[q] + CY3[q] * CY3[q] + CZ3[q] * CZ3[q];
    return c2 == 0 ? 1.0 / 3.0 : c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
}

/* Row r of the moment matrix at velocity q (D1). */
static double moment_row3(int r, int q)
{
    const double x = CX3[q], y = CY3[q], z = CZ3[q];
    const double c2 = x * x + y * y + z * z;
    switch (r) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return x * (y * y - z * z);
    case 17: return y * (z * z - x * x);
    default: return z * (x * x - y * y);
    }
}

static void moment_matrix3(double m[Q3][Q3])
{
    for (int r = 0; r < Q3; ++r)
        for (int q = 0; q < Q3; ++q) m[r][q] = moment_row3(r, q);
}

/* M^{-1} = M^T diag(1 / |row|^2): the rows are orthogonal (checked by the tests). */
static void inverse_moment_matrix3(double minv[Q3][Q3])
{
    double m[Q3][Q3];
    moment_matrix3(m);
    for (int r = 0; r < Q3; ++r) {
        double n2 = 0.0;
        for (int q = 0; q < Q3; ++q) n2 += m[r][q] * m[r][q];
        for (int q = 0; q < Q3; ++q) minv[q][r] = m[r][q] / n2;
    }
}

void oracle_d3q19_velocities(int32_t *cx, int32_t *cy, int32_t *cz)
{
    for (int q = 0; q < Q3; ++q) {
        cx[q] = CX3[q];
        cy[q] = CY3[q];
        cz[q] = CZ3[q];
    }
}

void oracle_d3q19_moment_matrix(double *out361)
{
    double m[Q3][Q3];
    moment_matrix3(m);
    memcpy(out361, m, sizeof m);
}

static inline int wrap3(int i, int n) { return ((i % n) + n) % n; }

typedef struct {
    int nx, ny, nz;
} grid3;

static inline size_t idx3(const grid3 *g, int i, int j, int k)
{
    return ((size_t)wrap3(k, g->nz) * (size_t)g->ny + (size_t)wrap3(j, g->ny)) * (size_t)g->nx +
           (size_t)wrap3(i, g->nx);
}

/* 3-point centred difference along axis a (0 = x, 1 = y, 2 = z) of f at node (i, j, k). */
static double d3(const grid3 *g, const double *f, int a, int i, int j, int k)
{
    const int di = a == 0, dj = a == 1, dk = a == 2;
    return 0.5 * (f[idx3(g, i + di, j + dj, k + dk)] - f[idx3(g, i - di, j - dj, k - dk)]);
}

/* The six defects (D4) at node (i, j, k): out = theta for e, 3p_xx, p_ww, p_xy, p_yz, p_xz.
 * J[a] are the momentum fields, P[a][c] the product fields J_a J_c. */
static void thetas3(const grid3 *g, const double *r, const double *const J[3], const double *const P[3][3], int i,
                    int j, int k, double th[6])
{
    const size_t p = idx3(g, i, j, k);
    double gr[3], dj[3][3], D[3], v[3];
    for (int a = 0; a < 3; ++a) {
        v[a] = J[a][p];
        gr[a] = d3(g, r, a, i, j, k);
        for (int b = 0; b < 3; ++b) dj[a][b] = d3(g, J[b], a, i, j, k); /* d_a J_b */
    }
    for (int a = 0; a < 3; ++a) {
        D[a] = 0.0;
        for (int c = 0; c < 3; ++c) D[a] += d3(g, P[a][c], c, i, j, k);
    }
    double t[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            t[a][b] = (dj[a][b] + dj[b][a]) / 3.0 - (v[a] * gr[b] + v[b] * gr[a]) / 3.0 - v[a] * D[b] - v[b] * D[a];
    const double div = dj[0][0] + dj[1][1] + dj[2][2];
    const double jg = v[0] * gr[0] + v[1] * gr[1] + v[2] * gr[2];
    const double j2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double tr = 2.0 / 3.0 * div - 2.0 / 3.0 * jg - 2.0 * j2 * div;
    th[0] = 19.0 * tr;
    th[1] = 2.0 * t[0][0] - t[1][1] - t[2][2];
    th[2] = t[1][1] - t[2][2];
    th[3] = t[0][1];
    th[4] = t[1][2];
    th[5] = t[0][2];
}

static int check3(int nx, int ny, int nz) { return nx < 3 || ny < 3 || nz < 3; }

typedef struct {
    double *prod[6]; /* xx, xy, xz, yy, yz, zz */
} products3;

static int products_alloc(products3 *p, size_t n)
{
    for (int a = 0; a < 6; ++a) {
        p->prod[a] = (double *)malloc(n * sizeof(double));
        if (!p->prod[a]) return 0;
    }
    return 1;
}

static void products_free(products3 *p)
{
    for (int a = 0; a < 6; ++a) free(p->prod[a]);
}

static void products_fill(products3 *p, const double *const J[3], size_t n)
{
    for (size_t s = 0; s < n; ++s) {
        p->prod[0][s] = J[0][s] * J[0][s];
        p->prod[1][s] = J[0][s] * J[1][s];
        p->prod[2][s] = J[0][s] * J[2][s];
        p->prod[3][s] = J[1][s] * J[1][s];
        p->prod[4][s] = J[1][s] * J[2][s];
        p->prod[5][s] = J[2][s] * J[2][s];
    }
}

static void products_view(const products3 *p, const double *P[3][3])
{
    P[0][0] = p->prod[0];
    P[0][1] = P[1][0] = p->prod[1];
    P[0][2] = P[2][0] = p->prod[2];
    P[1][1] = p->prod[3];
    P[1][2] = P[2][1] = p->prod[4];
    P[2][2] = p->prod[5];
}

/* The defects (D4) at every node: out6 holds six nx*ny*nz fields (e, 3p_xx, p_ww, p_xy,
 * p_yz, p_xz), periodic. */
int oracle_fd3d_theta(int nx, int ny, int nz, const double *drho, const double *jx, const double *jy,
                      const double *jz, double *out6)
{
    if (check3(nx, ny, nz)) return -1;
    const grid3 g = {nx, ny, nz};
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    const double *J[3] = {jx, jy, jz};
    products3 pr;
    if (!products_alloc(&pr, n)) return -2;
    products_fill(&pr, J, n);
    const double *P[3][3];
    products_view(&pr, P);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double th[6];
                thetas3(&g, drho, J, P, i, j, k, th);
                const size_t p = idx3(&g, i, j, k);
                for (int q = 0; q < 6; ++q) out6[(size_t)q * n + p] = th[q];
            }
    products_free(&pr);
    return 0;
}

/* Advance the D3Q19 FD-LBM state by nsteps (periodic in x, y, z). */
int oracle_fd3d_step(int nx, int ny, int nz, double s_e, double s_nu, double *drho, double *jx, double *jy,
                     double *jz, int64_t nsteps)
{
    if (check3(nx, ny, nz)) return -1;
    const grid3 g = {nx, ny, nz};
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double m[Q3][Q3], minv[Q3][Q3], w[Q3];
    moment_matrix3(m);
    inverse_moment_matrix3(minv);
    for (int q = 0; q < Q3; ++q) w[q] = weight3(q);
    static const int second[6] = {M3_E, M3_PXX, M3_PWW, M3_PXY, M3_PYZ, M3_PXZ};
    const double ce = 1.0 - 1.0 / s_e, cn = 1.0 - 1.0 / s_nu;
    double *fstar = (double *)malloc((size_t)Q3 * n * sizeof(double));
    products3 pr;
    if (!fstar || !products_alloc(&pr, n)) return -2;
    double *J[3] = {jx, jy, jz};
    const double *Jc[3] = {jx, jy, jz};
    const double *P[3][3];
    products_view(&pr, P);

    for (int64_t step = 0; step < nsteps; ++step) {
        products_fill(&pr, Jc, n);
        /* collision: f* = M^{-1} m* at every node (deviations from the rest populations) */
#pragma omp parallel for schedule(static) collapse(2)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t p = idx3(&g, i, j, k);
                    const double dr = drho[p], rho = 1.0 + dr;
                    const double v[3] = {jx[p], jy[p], jz[p]};
                    const double j2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                    double feq[Q3], dm[Q3], th[6];
                    for (int q = 0; q < Q3; ++q) {
                        const double cu = CX3[q] * v[0] + CY3[q] * v[1] + CZ3[q] * v[2];
                        feq[q] = w[q] * (dr + 3.0 * cu + 4.5 * cu * cu / rho - 1.5 * j2 / rho);
                    }
                    for (int r = 0; r < Q3; ++r) {
                        dm[r] = 0.0;
                        for (int q = 0; q < Q3; ++q) dm[r] += m[r][q] * feq[q];
                    }
                    thetas3(&g, drho, Jc, P, i, j, k, th);
                    dm[second[0]] += ce * th[0];
                    for (int t = 1; t < 6; ++t) dm[second[t]] += cn * th[t];
                    for (int q = 0; q < Q3; ++q) {
                        double f = 0.0;
                        for (int r = 0; r < Q3; ++r) f += minv[q][r] * dm[r];
                        fstar[(size_t)q * n + p] = f;
                    }
                }
        /* propagation (eq. 2): the population q arriving at x left x - c_q; f* holds the
         * whole step's post-collision populations, so the state is overwritten in place */
#pragma omp parallel for schedule(static) collapse(2)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t p = idx3(&g, i, j, k);
                    double s[4] = {0.0, 0.0, 0.0, 0.0};
                    for (int q = 0; q < Q3; ++q) {
                        const double f = fstar[(size_t)q * n + idx3(&g, i - CX3[q], j - CY3[q], k - CZ3[q])];
                        s[0] += f;
                        s[1] += CX3[q] * f;
                        s[2] += CY3[q] * f;
                        s[3] += CZ3[q] * f;
                    }
                    drho[p] = s[0];
                    for (int a = 0; a < 3; ++a) J[a][p] = s[a + 1];
                }
    }
    products_free(&pr);
    free(fstar);
    return 0;
}
