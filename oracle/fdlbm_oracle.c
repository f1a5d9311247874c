/*
 * FP64 CPU oracle for the FD-LBM D2Q9 time step, the LW-ACM step of section 1-b and the
 * MRT D2Q9 stream-collide step
 * of Dubois, Lallemand, Obrecht and Tekitek, "Lattice Boltzmann model approximated with
 * finite difference expressions" (Computers & Fluids 155, 2017; arXiv 1803.00437).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the GPU path is
 * checked against.  Only the tests, the smoke check and the bench's CPU-baseline leg may
 * load it.  It shares no code, header or constant table with the HIP library.
 *
 * Conventions (all FP64):
 *   - fields are nx*ny arrays, x fastest: element j*nx + i is node (x=i, y=j);
 *   - the stored state of a node is the deviation from the rest state rho=1, J=0:
 *     drho = rho - 1, jx, jy.  Populations are stored as deviations df_k = f_k - w_k
 *     from the rest populations w = M^{-1} m0, m0 = (1,0,0,-2,0,0,0,0,1).  Because M is
 *     linear, working with deviations is the same algebra as the paper's, with every
 *     rest-state constant cancelled exactly instead of by rounding;
 *   - x is always periodic; y is periodic (walls = 0) or bounded by two walls (walls = 1)
 *     at distance xi beyond the first and last rows, y = -xi and y = ny - 1 + xi (the
 *     channel of section 3-c and Fig. 6; xi = 1/2 puts them half-way to the next rows).
 *
 * Readings of passages that are garbled or silent in the paper:
 *   R1  the printed J_x row has +1 at e_3 and the J_y row +1 at e_4; the other rows fix
 *       e_3 = (-1,0), e_4 = (0,-1), so those two entries are -1 here;
 *   R2  the linear part of theta_XY is (1/3)(d_x v_y + d_y v_x) (printed with a minus);
 *   R3  every "v" inside the theta terms is the stored momentum J (rho close to 1);
 *   R4  derivatives of products (d_x v_x^2 ...) are finite differences of the product field;
 *   R5  the E and eps lines use 3(J_x^2+J_y^2)/rho as in the standard D2Q9 table;
 *   R6  the velocity-cubic term of theta_E is printed as +6|v|^2 div v; section 2 states that
 *       with these expressions the bulk viscosity in a mean flow V is zeta (1 - 3V^2).  A term
 *       c |v|^2 div v gives exactly zeta (1 + c V^2 / 2) in every direction of V and k, so
 *       that statement fixes c = -6: the printed sign is taken as a slip (as in R2);
 *   R8  body force (Strang): J_a = J + F/2 enters equilibria and theta, J* = J + F;
 *   R9  walls at xi = 1/2: ghost nodes hold the linear extrapolation with zero velocity on
 *       the wall (J odd, rho even about the wall); MRT uses halfway bounce-back;
 *   R18 walls at a general distance xi (Fig. 6): ghost nodes hold the mirror-point value
 *       described at fill_ghosts(); MRT uses the linear interpolated bounce-back of Bouzidi
 *       et al. (both reduce to R9 at xi = 1/2);
 *   R16 LW-ACM: the node (i0, j0) in the reconstruction of section 1-b is the one that link
 *       k reaches from (i, j), as in eq. 2; u = J / rho inside f^eq and f^eo.
 *
 * What pins this file (tests/test_oracle_pins.py): the moment matrix against the physical
 * moments it names, the equilibria against the textbook D2Q9 polynomial, the stencils
 * against their exact errors on polynomials, mass/momentum conservation, fixed points, the
 * reduction to textbook BGK at unit rates, its linear response against the amplification
 * matrix (whose hyperviscosities reproduce Table 1), the shear viscosity nu(1 - 3V^2) in
 * mean flow along both axes and both diagonals (every velocity-cubic term of theta_XX and
 * theta_XY), and the Poiseuille parabola.  LW-ACM: the reduction to textbook BGK at
 * Theta = 0, conservation, its linear response (at rest and in a mean flow) against its
 * amplification matrix, which matches the one printed in section 1-b to third order in k,
 * and the transport coefficients printed there (c_s = sqrt(2 nu), Gamma_s = nu/2 + 1/12,
 * nu(v) = nu - v^2/2, instability above c_s).
 * The density-gradient terms of theta_E, theta_XX, theta_XY are pinned against the defect of
 * conservation itself: one textbook-BGK step leaves non-equilibrium moments equal to minus
 * the exact defect, whose first-order expansion for a density wave on a uniform flow is the
 * printed terms plus |J|^2 terms that the paper omits (rho close to 1).
 * The velocity-cubic term of theta_E is pinned by the bulk viscosity of section 2: the
 * acoustic damping of this oracle, linearised about a uniform flow V, has the coefficient
 * (1 - 3V^2)/2 of zeta along axes and diagonals (and its amplification matrix equals the
 * symbol's, which has it at every angle).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Velocity set of section 1: e_0 rest, e_1..e_4 = +x, +y, -x, -y, e_5..e_8 = the diagonals
 * (+x+y), (-x+y), (-x-y), (+x-y). */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Moment matrix of section 1 (rows rho, Jx, Jy, E, XX, XY, qx, qy, eps), reading R1. */
static const double MOM[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {4, -2, -2, -2, -2, 1, 1, 1, 1}};

/* M is orthogonal (section 1): M^{-1} = M^T diag(1/|row_l|^2). */
static void inverse_moment_matrix(double minv[9][9])
{
    for (int l = 0; l < 9; ++l) {
        double n2 = 0.0;
        for (int k = 0; k < 9; ++k) n2 += MOM[l][k] * MOM[l][k];
        for (int k = 0; k < 9; ++k) minv[k][l] = MOM[l][k] / n2;
    }
}

void oracle_moment_matrix(double *out81)
{
    for (int l = 0; l < 9; ++l)
        for (int k = 0; k < 9; ++k) out81[l * 9 + k] = MOM[l][k];
}

void oracle_inverse_moment_matrix(double *out81)
{
    double minv[9][9];
    inverse_moment_matrix(minv);
    for (int k = 0; k < 9; ++k)
        for (int l = 0; l < 9; ++l) out81[k * 9 + l] = minv[k][l];
}

void oracle_velocities(int32_t *ex9, int32_t *ey9)
{
    for (int k = 0; k < 9; ++k) { ex9[k] = EX[k]; ey9[k] = EY[k]; }
}

int oracle_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Fields extended by G ghost rows above and below the fluid rows.                      */
/* ------------------------------------------------------------------------------------ */
#define G 3

typedef struct {
    int nx, ny;
    double *a; /* (ny + 2G) rows of nx */
} xfield;

static int xf_alloc(xfield *f, int nx, int ny)
{
    f->nx = nx;
    f->ny = ny;
    f->a = (double *)calloc((size_t)(ny + 2 * G) * (size_t)nx, sizeof(double));
    return f->a != NULL;
}

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* value at node (i, j); x periodic, j in [-G, ny + G) */
static inline double at(const xfield *f, int i, int j)
{
    return f->a[(size_t)(j + G) * (size_t)f->nx + (size_t)wrap(i, f->nx)];
}

static inline double *row(xfield *f, int j) { return f->a + (size_t)(j + G) * (size_t)f->nx; }

/* Fill ghost rows.  parity = +1 for even fields (density), -1 for odd ones (velocity),
 * 0 for fields that must not be mirrored (periodic case only).
 *
 * Walls (section 3-b, 3-c): the wall lies at distance xi (0 < xi <= 1) beyond the last
 * fluid row, at y = -xi and y = ny - 1 + xi.  Reading R18: the ghost node at distance
 * d = g - xi beyond the wall (ghost row -g, g = 1, 2, ...) holds the value at its mirror
 * point, d inside the fluid (y_m = g - 2 xi), with the velocity negated, so that the
 * velocity varies linearly through zero on the wall.  The value at y_m is interpolated
 * linearly between the fluid rows around it; when y_m lies between the wall and the last
 * fluid row, the velocity is interpolated between zero on the wall and that row, and the
 * density taken from that row (zero normal gradient).  Which expression applies depends on
 * where the wall cuts the link from the last fluid node to the ghost node (xi < or >= 1/2
 * for the first ghost row), as in the scheme of Bouzidi et al.  At xi = 1/2 every ghost
 * row mirrors a fluid row exactly: ghost row -1-m holds parity times fluid row m. */
static void ghost_row(xfield *f, int walls_top, int g, double parity, double xi)
{
    const int nx = f->nx, ny = f->ny;
    /* fluid row k counted from the wall side, and the ghost row written */
    double *dst = walls_top ? row(f, ny - 1 + g) : row(f, -g);
    const double ym = (double)g - 2.0 * xi;
#define FROM(k) (walls_top ? row(f, ny - 1 - (k)) : row(f, (k)))
    if (ym >= 0.0) {
        const int s0 = (int)floor(ym);
        const double t = ym - (double)s0;
        const double *a = FROM(s0);
        if (t == 0.0) {
            for (int i = 0; i < nx; ++i) dst[i] = parity * a[i];
        } else {
            const double *b = FROM(s0 + 1);
            for (int i = 0; i < nx; ++i) dst[i] = parity * ((1.0 - t) * a[i] + t * b[i]);
        }
    } else {
        const double *a = FROM(0);
        const double w = parity < 0.0 ? (ym + xi) / xi : 1.0;
        for (int i = 0; i < nx; ++i) dst[i] = parity * w * a[i];
    }
#undef FROM
}

static void fill_ghosts(xfield *f, int walls, double parity, double xi)
{
    int nx = f->nx, ny = f->ny;
    for (int m = 0; m < G; ++m) {
        double *lo = row(f, -1 - m), *hi = row(f, ny + m);
        if (!walls) {
            const double *slo = row(f, wrap(-1 - m, ny)), *shi = row(f, wrap(ny + m, ny));
            memcpy(lo, slo, (size_t)nx * sizeof(double));
            memcpy(hi, shi, (size_t)nx * sizeof(double));
        } else {
            ghost_row(f, 0, m + 1, parity, xi);
            ghost_row(f, 1, m + 1, parity, xi);
        }
    }
}

/* Section 2: first derivative estimated by finite differences.
 *   3 points:  d_x g ~ (g(i+1) - g(i-1)) / 2
 *   5 points:  d_x g ~ 3/4 (g(i+1) - g(i-1)) - 1/8 (g(i+2) - g(i-2))
 *   9 points (D2Q9 geometry):
 *       d_x g ~ g(i+1,j) - g(i-1,j) - 1/4 [g(i+1,j+1) - g(i-1,j+1) - g(i-1,j-1) + g(i+1,j-1)]
 *       and the same with the roles of x and y exchanged for d_y. */
static inline double ddx(const xfield *g, int stencil, int i, int j)
{
    if (stencil == 3) return 0.5 * (at(g, i + 1, j) - at(g, i - 1, j));
    if (stencil == 5)
        return 0.75 * (at(g, i + 1, j) - at(g, i - 1, j)) - 0.125 * (at(g, i + 2, j) - at(g, i - 2, j));
    return at(g, i + 1, j) - at(g, i - 1, j) -
           0.25 * (at(g, i + 1, j + 1) - at(g, i - 1, j + 1) - at(g, i - 1, j - 1) + at(g, i + 1, j - 1));
}

static inline double ddy(const xfield *g, int stencil, int i, int j)
{
    if (stencil == 3) return 0.5 * (at(g, i, j + 1) - at(g, i, j - 1));
    if (stencil == 5)
        return 0.75 * (at(g, i, j + 1) - at(g, i, j - 1)) - 0.125 * (at(g, i, j + 2) - at(g, i, j - 2));
    return at(g, i, j + 1) - at(g, i, j - 1) -
           0.25 * (at(g, i + 1, j + 1) - at(g, i + 1, j - 1) - at(g, i - 1, j - 1) + at(g, i - 1, j + 1));
}

/* Periodic derivative of one field (stencil checks). axis 0 = x, 1 = y. */
int oracle_fd_derivative(int nx, int ny, int stencil, int axis, const double *in, double *out)
{
    if (nx < 1 || ny < 1 || (stencil != 3 && stencil != 5 && stencil != 9)) return -1;
    xfield g;
    if (!xf_alloc(&g, nx, ny)) return -2;
    for (int j = 0; j < ny; ++j) memcpy(row(&g, j), in + (size_t)j * nx, (size_t)nx * sizeof(double));
    fill_ghosts(&g, 0, 0.0, 0.5);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            out[(size_t)j * nx + i] = axis == 0 ? ddx(&g, stencil, i, j) : ddy(&g, stencil, i, j);
    free(g.a);
    return 0;
}

/*
 * Section 2: the defects of conservation at node (i, j), with v read as the stored momentum
 * J (here J_a, see R3, R8) and the derivatives estimated by finite differences (R4):
 *   theta_E  = (2 - 6|v|^2) div v - 2 v . grad rho
 *   theta_XX = 2/3 (d_x v_x - d_y v_y) - 2/3 (v_x d_x rho - v_y d_y rho)
 *              - 2 [v_x (d_x v_x^2 + d_y v_x v_y) - v_y (d_x v_x v_y + d_y v_y^2)]
 *   theta_XY = 1/3 (d_x v_y + d_y v_x) - 1/3 (v_x d_y rho + v_y d_x rho)
 *              - v_x (d_x v_x v_y + d_y v_y^2) - v_y (d_x v_x^2 + d_y v_x v_y)
 * (R2: + in the linear part of theta_XY; R6: the velocity-cubic term of theta_E with the
 * sign that section 2's bulk viscosity in a mean flow fixes, see the file header.)
 */
static void thetas(const xfield *r, const xfield *vx, const xfield *vy, const xfield *pxx, const xfield *pxy,
                   const xfield *pyy, int stencil, int i, int j, double *te, double *txx, double *txy)
{
    const double ux = at(vx, i, j), uy = at(vy, i, j);
    const double rx = ddx(r, stencil, i, j), ry = ddy(r, stencil, i, j);
    const double uxx = ddx(vx, stencil, i, j), uyy = ddy(vy, stencil, i, j);
    const double uyx = ddx(vy, stencil, i, j), uxy = ddy(vx, stencil, i, j);
    const double dx_xx = ddx(pxx, stencil, i, j), dy_xy = ddy(pxy, stencil, i, j);
    const double dx_xy = ddx(pxy, stencil, i, j), dy_yy = ddy(pyy, stencil, i, j);
    *te = (2.0 - 6.0 * (ux * ux + uy * uy)) * (uxx + uyy) - 2.0 * (ux * rx + uy * ry);
    *txx = (2.0 / 3.0) * (uxx - uyy) - (2.0 / 3.0) * (ux * rx - uy * ry) -
           2.0 * (ux * (dx_xx + dy_xy) - uy * (dx_xy + dy_yy));
    *txy = (1.0 / 3.0) * (uyx + uxy) - (1.0 / 3.0) * (ux * ry + uy * rx) - ux * (dx_xy + dy_yy) -
           uy * (dx_xx + dy_xy);
}

/* The three defects of every node of a periodic state (no force), for the pins. */
int oracle_fd_theta(int nx, int ny, int stencil, const double *drho, const double *jx, const double *jy,
                    double *te, double *txx, double *txy)
{
    if (nx < 1 || ny < 1 || (stencil != 3 && stencil != 5 && stencil != 9)) return -1;
    xfield r, vx, vy, pxx, pxy, pyy;
    int ok = xf_alloc(&r, nx, ny) && xf_alloc(&vx, nx, ny) && xf_alloc(&vy, nx, ny) &&
             xf_alloc(&pxx, nx, ny) && xf_alloc(&pxy, nx, ny) && xf_alloc(&pyy, nx, ny);
    if (!ok) return -2;
    for (int j = 0; j < ny; ++j) {
        memcpy(row(&r, j), drho + (size_t)j * nx, (size_t)nx * sizeof(double));
        memcpy(row(&vx, j), jx + (size_t)j * nx, (size_t)nx * sizeof(double));
        memcpy(row(&vy, j), jy + (size_t)j * nx, (size_t)nx * sizeof(double));
    }
    fill_ghosts(&r, 0, 0.0, 0.5);
    fill_ghosts(&vx, 0, 0.0, 0.5);
    fill_ghosts(&vy, 0, 0.0, 0.5);
    for (int j = -G; j < ny + G; ++j) {
        const double *ax = row(&vx, j), *ay = row(&vy, j);
        double *bxx = row(&pxx, j), *bxy = row(&pxy, j), *byy = row(&pyy, j);
        for (int i = 0; i < nx; ++i) {
            bxx[i] = ax[i] * ax[i];
            bxy[i] = ax[i] * ay[i];
            byy[i] = ay[i] * ay[i];
        }
    }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t p = (size_t)j * nx + (size_t)i;
            thetas(&r, &vx, &vy, &pxx, &pxy, &pyy, stencil, i, j, te + p, txx + p, txy + p);
        }
    free(r.a); free(vx.a); free(vy.a); free(pxx.a); free(pxy.a); free(pyy.a);
    return 0;
}

static int check_grid(int nx, int ny, int walls, double xi)
{
    if (nx < 1 || ny < 1) return -1;
    if (walls && (ny < (xi == 0.5 ? G : G + 1) || !(xi > 0.0 && xi <= 1.0))) return -1;
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* FD-LBM time step (section 2).                                                         */
/* ------------------------------------------------------------------------------------ */
/*
 * One step, node by node, in the order of section 2:
 *   1. primitive variables rho, J at every node (ghost nodes by extrapolation when there
 *      are walls); with a force, J_a = J + F/2 (Strang, section 1);
 *   2. products J_x^2, J_x J_y, J_y^2 and the finite differences of rho, J and the products;
 *   3. the defects of conservation theta_E, theta_XX, theta_XY (section 2);
 *   4. post-collision moments
 *        E   = -2 rho + 3|J|^2/rho + (1 - 1/s_e)  theta_E
 *        XX  = (J_x^2 - J_y^2)/rho + (1 - 1/s_xx) theta_XX
 *        XY  = J_x J_y/rho         + (1 - 1/s_xx) theta_XY
 *        q   = -J,   eps = rho - 3|J|^2/rho,   rho and J conserved (J + F with a force);
 *   5. f* = M^{-1} m*  (section 1);
 *   6. propagation f^{n+1}(x + e_k) = f*_k(x) (eq. 2), then the new rho, J = rows 0..2 of M f.
 */
int oracle_fd_step(int nx, int ny, int stencil, int walls, double xi, double s_e, double s_xx, double fx,
                   double fy, double *drho, double *jx, double *jy, int64_t nsteps)
{
    if (check_grid(nx, ny, walls, xi) || (stencil != 3 && stencil != 5 && stencil != 9)) return -1;
    double minv[9][9];
    inverse_moment_matrix(minv);
    const double ce = 1.0 - 1.0 / s_e, cxx = 1.0 - 1.0 / s_xx;
    const size_t n = (size_t)nx * (size_t)ny;

    xfield r, vx, vy, pxx, pxy, pyy;
    int ok = xf_alloc(&r, nx, ny) && xf_alloc(&vx, nx, ny) && xf_alloc(&vy, nx, ny) &&
             xf_alloc(&pxx, nx, ny) && xf_alloc(&pxy, nx, ny) && xf_alloc(&pyy, nx, ny);
    /* f* on the fluid rows plus one row on each side: rows -1 .. ny */
    const int r0 = walls ? -1 : 0, r1 = walls ? ny + 1 : ny;
    const size_t nstar = (size_t)(r1 - r0) * (size_t)nx;
    double *fstar = (double *)malloc(9 * nstar * sizeof(double));
    double *fnew = (double *)malloc(9 * n * sizeof(double));
    if (!ok || !fstar || !fnew) return -2;

    for (int64_t step = 0; step < nsteps; ++step) {
        /* 1. primitive variables, ghost rows, force half-step */
        for (int j = 0; j < ny; ++j) {
            memcpy(row(&r, j), drho + (size_t)j * nx, (size_t)nx * sizeof(double));
            memcpy(row(&vx, j), jx + (size_t)j * nx, (size_t)nx * sizeof(double));
            memcpy(row(&vy, j), jy + (size_t)j * nx, (size_t)nx * sizeof(double));
        }
        fill_ghosts(&r, walls, +1.0, xi);
        fill_ghosts(&vx, walls, -1.0, xi);
        fill_ghosts(&vy, walls, -1.0, xi);
        for (int j = -G; j < ny + G; ++j) {
            double *ax = row(&vx, j), *ay = row(&vy, j);
            for (int i = 0; i < nx; ++i) { ax[i] += 0.5 * fx; ay[i] += 0.5 * fy; }
        }
        /* 2. product fields */
        for (int j = -G; j < ny + G; ++j) {
            const double *ax = row(&vx, j), *ay = row(&vy, j);
            double *bxx = row(&pxx, j), *bxy = row(&pxy, j), *byy = row(&pyy, j);
            for (int i = 0; i < nx; ++i) {
                bxx[i] = ax[i] * ax[i];
                bxy[i] = ax[i] * ay[i];
                byy[i] = ay[i] * ay[i];
            }
        }
        /* 2-5. derivatives, theta, m*, f* */
#pragma omp parallel for schedule(static)
        for (int j = r0; j < r1; ++j) {
            for (int i = 0; i < nx; ++i) {
                const double dr = at(&r, i, j), rho = 1.0 + dr;
                const double ux = at(&vx, i, j), uy = at(&vy, i, j);
                double theta_e, theta_xx, theta_xy;
                thetas(&r, &vx, &vy, &pxx, &pxy, &pyy, stencil, i, j, &theta_e, &theta_xx, &theta_xy);

                const double j2 = ux * ux + uy * uy;
                double dm[9];
                dm[0] = dr;
                dm[1] = ux + 0.5 * fx;
                dm[2] = uy + 0.5 * fy;
                dm[3] = -2.0 * dr + 3.0 * j2 / rho + ce * theta_e; /* E + 2 */
                dm[4] = (ux * ux - uy * uy) / rho + cxx * theta_xx;
                dm[5] = ux * uy / rho + cxx * theta_xy;
                dm[6] = -ux;
                dm[7] = -uy;
                dm[8] = dr - 3.0 * j2 / rho; /* eps - 1 */

                const size_t s = (size_t)(j - r0) * (size_t)nx + (size_t)i;
                for (int k = 0; k < 9; ++k) {
                    double f = 0.0;
                    for (int l = 0; l < 9; ++l) f += minv[k][l] * dm[l];
                    fstar[(size_t)k * nstar + s] = f;
                }
            }
        }
        /* 6. propagation */
        for (int j = r0; j < r1; ++j) {
            for (int i = 0; i < nx; ++i) {
                const size_t s = (size_t)(j - r0) * (size_t)nx + (size_t)i;
                for (int k = 0; k < 9; ++k) {
                    int jd = j + EY[k], id = wrap(i + EX[k], nx);
                    if (walls) {
                        if (jd < 0 || jd >= ny) continue; /* lands on a ghost node */
                    } else {
                        jd = wrap(jd, ny);
                    }
                    fnew[(size_t)k * n + (size_t)jd * nx + (size_t)id] = fstar[(size_t)k * nstar + s];
                }
            }
        }
        for (size_t p = 0; p < n; ++p) {
            double m0 = 0.0, m1 = 0.0, m2 = 0.0;
            for (int k = 0; k < 9; ++k) {
                const double f = fnew[(size_t)k * n + p];
                m0 += MOM[0][k] * f;
                m1 += MOM[1][k] * f;
                m2 += MOM[2][k] * f;
            }
            drho[p] = m0;
            jx[p] = m1;
            jy[p] = m2;
        }
    }
    free(r.a); free(vx.a); free(vy.a); free(pxx.a); free(pxy.a); free(pyy.a);
    free(fstar);
    free(fnew);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* MRT D2Q9 (section 1, eq. 1 and 2; equilibria and rates of the table in section 1-a). */
/* ------------------------------------------------------------------------------------ */

/* Equilibrium moments of the standard D2Q9 table, as deviations from the rest moments. */
static void equilibrium_moments(double dr, double ux, double uy, double meq[9])
{
    const double rho = 1.0 + dr, j2 = ux * ux + uy * uy;
    meq[0] = dr;
    meq[1] = ux;
    meq[2] = uy;
    meq[3] = -2.0 * dr + 3.0 * j2 / rho;
    meq[4] = (ux * ux - uy * uy) / rho;
    meq[5] = ux * uy / rho;
    meq[6] = -ux;
    meq[7] = -uy;
    meq[8] = dr - 3.0 * j2 / rho;
}

/* f = f^eq(rho, J) = M^{-1} m^eq (the initial populations of an MRT run). */
int oracle_mrt_init(int nx, int ny, const double *drho, const double *jx, const double *jy, double *df)
{
    if (nx < 1 || ny < 1) return -1;
    double minv[9][9];
    inverse_moment_matrix(minv);
    const size_t n = (size_t)nx * (size_t)ny;
    for (size_t p = 0; p < n; ++p) {
        double meq[9];
        equilibrium_moments(drho[p], jx[p], jy[p], meq);
        for (int k = 0; k < 9; ++k) {
            double f = 0.0;
            for (int l = 0; l < 9; ++l) f += minv[k][l] * meq[l];
            df[(size_t)k * n + p] = f;
        }
    }
    return 0;
}

/* rho - 1 and J of a population field (rows 0..2 of M). */
int oracle_mrt_moments(int nx, int ny, const double *df, double *drho, double *jx, double *jy)
{
    if (nx < 1 || ny < 1) return -1;
    const size_t n = (size_t)nx * (size_t)ny;
    for (size_t p = 0; p < n; ++p) {
        double m0 = 0.0, m1 = 0.0, m2 = 0.0;
        for (int k = 0; k < 9; ++k) {
            const double f = df[(size_t)k * n + p];
            m0 += MOM[0][k] * f;
            m1 += MOM[1][k] * f;
            m2 += MOM[2][k] * f;
        }
        drho[p] = m0;
        jx[p] = m1;
        jy[p] = m2;
    }
    return 0;
}

/*
 * MRT step: m = M f; J_a = J + F/2; m*_k = m_k + s_k (m_k^eq(rho, J_a) - m_k) for the
 * non-conserved moments (eq. 1), J* = J + F; f* = M^{-1} m*; f^{n+1}(x + e_k) = f*_k(x)
 * (eq. 2).  With walls, a population whose destination lies beyond a wall returns to its
 * source node x with the opposite velocity.  The wall cuts that link at the fraction q = xi
 * of its length (walls at y = -xi and ny - 1 + xi); the returning population is the
 * linear interpolation of Bouzidi, Firdaouss and Lallemand (reading R18):
 *   q <  1/2:  f_kbar(x) = 2q f*_k(x) + (1 - 2q) f*_k(x - e_k),
 *   q >= 1/2:  f_kbar(x) = f*_k(x) / (2q) + (2q - 1)/(2q) f*_kbar(x),
 * which is halfway bounce-back, f_kbar(x) = f*_k(x), at q = 1/2.
 * Rates: s = (-, -, -, s_e, s_xx, s_xx, s_q, s_q, s_eps).
 */
int oracle_mrt_step(int nx, int ny, int walls, double xi, double s_e, double s_xx, double s_q, double s_eps,
                    double fx, double fy, double *df, int64_t nsteps)
{
    if (check_grid(nx, ny, walls, xi)) return -1;
    double minv[9][9];
    inverse_moment_matrix(minv);
    const double s[9] = {0.0, 0.0, 0.0, s_e, s_xx, s_xx, s_q, s_q, s_eps};
    const size_t n = (size_t)nx * (size_t)ny;
    double *fstar = (double *)malloc(9 * n * sizeof(double));
    double *fnew = (double *)malloc(9 * n * sizeof(double));
    if (!fstar || !fnew) {
        free(fstar);
        free(fnew);
        return -2;
    }
    for (int64_t step = 0; step < nsteps; ++step) {
        /* collision at every node */
#pragma omp parallel for schedule(static)
        for (size_t p = 0; p < n; ++p) {
            double m[9], meq[9], ms[9];
            for (int l = 0; l < 9; ++l) {
                double acc = 0.0;
                for (int k = 0; k < 9; ++k) acc += MOM[l][k] * df[(size_t)k * n + p];
                m[l] = acc;
            }
            const double ux = m[1] + 0.5 * fx, uy = m[2] + 0.5 * fy;
            equilibrium_moments(m[0], ux, uy, meq);
            ms[0] = m[0];
            ms[1] = m[1] + fx;
            ms[2] = m[2] + fy;
            for (int l = 3; l < 9; ++l) ms[l] = m[l] + s[l] * (meq[l] - m[l]);
            for (int k = 0; k < 9; ++k) {
                double f = 0.0;
                for (int l = 0; l < 9; ++l) f += minv[k][l] * ms[l];
                fstar[(size_t)k * n + p] = f;
            }
        }
        /* propagation (eq. 2), interpolated bounce-back at the walls */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                const size_t p = (size_t)j * nx + (size_t)i;
                for (int k = 0; k < 9; ++k) {
                    const double fk = fstar[(size_t)k * n + p];
                    int jd = j + EY[k];
                    const int id = wrap(i + EX[k], nx);
                    if (walls && (jd < 0 || jd >= ny)) {
                        const int kb = OPP[k];
                        double v;
                        if (xi == 0.5) {
                            v = fk;
                        } else if (xi < 0.5) {
                            const size_t pb = (size_t)(j - EY[k]) * nx + (size_t)wrap(i - EX[k], nx);
                            v = 2.0 * xi * fk + (1.0 - 2.0 * xi) * fstar[(size_t)k * n + pb];
                        } else {
                            v = fk / (2.0 * xi) + (2.0 * xi - 1.0) / (2.0 * xi) * fstar[(size_t)kb * n + p];
                        }
                        fnew[(size_t)kb * n + p] = v;
                        continue;
                    }
                    jd = wrap(jd, ny);
                    fnew[(size_t)k * n + (size_t)jd * nx + (size_t)id] = fk;
                }
            }
        }
        memcpy(df, fnew, 9 * n * sizeof(double));
    }
    free(fstar);
    free(fnew);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* LW-ACM (section 1-b), the link-wise artificial-compressibility step the paper takes    */
/* as its starting point.  Periodic grid.                                                 */
/* ------------------------------------------------------------------------------------ */

/*
 * One step, written as section 1-b defines it:
 *   f^eq(rho, u)  the D2Q9 equilibrium of the table in section 1-a (M^{-1} m^eq),
 *   f^eo(rho, u) = (f^eq(rho, u) - f^eq(rho, -u)) / 2,
 *   f*_k(x)      = f^eq_k(x) + Theta (f^eo_k(x + e_k) - f^eo_k(x)),  Theta = 1 - 6 nu,
 * where x + e_k is the node that link k reaches from x (the "(i0, j0)" of eq. 2), and
 *   f^{n+1}_k(x + e_k) = f*_k(x)   (eq. 2);   rho^{n+1}, J^{n+1} = moments of f^{n+1}.
 * The velocity enters through J = rho u (u -> -u is J -> -J at fixed rho > 0).
 * Populations are deviations from w (see the conventions at the top of this file).
 */
int oracle_lwacm_step(int nx, int ny, double nu, double *drho, double *jx, double *jy, int64_t nsteps)
{
    if (nx < 1 || ny < 1 || nsteps < 0) return -1;
    double minv[9][9];
    inverse_moment_matrix(minv);
    const double theta = 1.0 - 6.0 * nu;
    const size_t n = (size_t)nx * (size_t)ny;
    double *feq = (double *)malloc(9 * n * sizeof(double));
    double *feo = (double *)malloc(9 * n * sizeof(double));
    if (!feq || !feo) {
        free(feq);
        free(feo);
        return -2;
    }
    for (int64_t step = 0; step < nsteps; ++step) {
        /* f^eq and f^eo of every node */
#pragma omp parallel for schedule(static)
        for (size_t p = 0; p < n; ++p) {
            double mp[9], mm[9];
            equilibrium_moments(drho[p], jx[p], jy[p], mp);
            equilibrium_moments(drho[p], -jx[p], -jy[p], mm);
            for (int k = 0; k < 9; ++k) {
                double fp = 0.0, fm = 0.0;
                for (int l = 0; l < 9; ++l) {
                    fp += minv[k][l] * mp[l];
                    fm += minv[k][l] * mm[l];
                }
                feq[(size_t)k * n + p] = fp;
                feo[(size_t)k * n + p] = 0.5 * (fp - fm);
            }
        }
        /* the new state at x gathers f*_k from x - e_k, whose link k ends at x */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                const size_t p = (size_t)j * nx + (size_t)i;
                double r = 0.0, x = 0.0, y = 0.0;
                for (int k = 0; k < 9; ++k) {
                    const size_t s = (size_t)wrap(j - EY[k], ny) * nx + (size_t)wrap(i - EX[k], nx);
                    const double fs = feq[(size_t)k * n + s] + theta * (feo[(size_t)k * n + p] - feo[(size_t)k * n + s]);
                    r += fs;
                    x += EX[k] * fs;
                    y += EY[k] * fs;
                }
                /* only feq and feo are read in this pass, so the state is overwritten in place */
                drho[p] = r;
                jx[p] = x;
                jy[p] = y;
            }
        }
    }
    free(feq);
    free(feo);
    return 0;
}
