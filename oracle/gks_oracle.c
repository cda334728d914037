/*
 * gks_oracle.c -- test infrastructure, not part of the product.
 *
 * Plain, slow, FP64 reference of the third-order compact gas-kinetic scheme
 * (GKS) on tetrahedra of Ji, Zhao, Shyy & Xu.  Every function follows the
 * paper's steps in its order and notation; it is deliberately unoptimised:
 *
 *   - geometry by the paper's own quadratures (Sec. 2.1 three-point face rule,
 *     Sec. 4.1 five-point volume rule, weight of the centre point read as
 *     -2/15 so that the rule integrates cubics exactly); with quadratic
 *     elements (or_create_quadratic) both rules run on the isoparametric
 *     maps, each face Gauss point with its own normal and weight;
 *   - reconstruction solves the least-squares (step 1) and constrained
 *     least-squares (step 2) systems cell by cell, every stage, by Gaussian
 *     elimination with partial pivoting (Secs. 4.1-4.3);
 *   - the gas-kinetic solver expands every integrand into monomials in
 *     (u, v, w, xi^2) and takes Maxwellian moments term by term, and solves
 *     the 5x5 moment systems for the microscopic slopes numerically
 *     (Sec. 2.2, eqs. 2nd-flux, co, new-equ-part);
 *   - two-stage fourth-order time stepping and Gauss-theorem gradient update
 *     (Secs. 2.3 and 3).
 *
 * The flux may also take the smooth-flow form of the distribution (eq.
 * 2nd-smooth-flux): the equilibrium g^c, with the kinetically weighted W^c
 * and slopes of eq. new-equ-part, and no kinetic part.
 *
 * Walls (face_cell[2f+1] = -1) carry a tag (Sec. 4.4).  Next to any wall,
 * cells use one-sided reconstructions (the own averaged gradient, and a
 * linear least-squares fit in step 2, where fewer than three neighbours
 * remain).  Slip walls (tag 2): the flux sees the mirror image of the
 * interior state as ghost.  No-slip adiabatic (3) and isothermal (4) walls:
 * the momentum (and at isothermal walls the energy) of the adjacent cells'
 * reconstructions is constrained to the wall values in both steps, and the
 * ghost is the reflected state.  Far field (5): the locally one-dimensional
 * Riemann-invariant state against the free stream, with zero gradients.
 *
 * Pins (the tests/test_oracle_*.py suites, no GPU): quadrature exactness,
 * the quadratic elements' closed forms and fourth-order wall convergence,
 * reconstruction exactness on polynomials and the paper's convergence orders,
 * Maxwellian moments against closed forms, the flux against the Euler and
 * Navier-Stokes fluxes of smooth states, conservation, free-stream
 * preservation, the walls' constraints and ghost symmetries.  Parity
 * unpinned: the Prandtl correction beyond continuous linear data (pinned
 * there against the Chapman-Enskog heat flux), and the magnitudes of the
 * nonlinear-weight errors (their orders and the exactness are pinned; the
 * paper's tabulated magnitudes are not reproduced).
 *
 * Loops over cells and faces may run under OpenMP; every output element is
 * written by exactly one iteration, and all sums run in a fixed serial
 * order, so results do not depend on the thread count.
 *
 * Readings of silent or ambiguous passages (both this file and the library
 * follow them): polynomials are fitted in coordinates centred at the target
 * centroid and scaled by h = |Omega|^(1/3); least-squares rows are the
 * averaged (divided by |Omega_m|) equations with unit weights; the smoothness
 * factor |Delta_0| of the two-step indicator is |Omega_0|^(2/3); each
 * multi-index enters the smoothness indicator once; the positivity fallback
 * acts per cell on all five components; p_l, p_r of the collision time are
 * the reconstructed point pressures; tau = mu / p^c; the stage-2 flux uses
 * the same dt with the time origin reset; the Prandtl number enters through
 * a correction of the time-integrated energy flux by (1/Pr - 1) times the
 * time-integrated heat flux of the interface distribution about U^c.
 */
/* The arithmetic type of everything that depends on the state: double, or
 * in the tangent build (compiled as C++ with OR_TANGENT) a forward-mode dual
 * number that also carries directional derivatives.  Geometry stays double. */
#ifdef OR_TANGENT
#include "or_dual.hpp"
typedef or_dual real;
#define OR_REAL or_dual
#define OR_VALUE(x) ((x).v)
/* Non-differentiable points of the scheme: the collision-time jump (site 0)
 * and the absolute values in the WENO indicators (site 1).  The tangent
 * build counts, per direction k, the evaluations whose argument x lies
 * within the kink distance of zero, |x| < eps |dx/dv_k|: a central
 * difference of step eps along v_k straddles such a kink. */
static double or_kink_eps = 0.0;
static long or_kinks[2][OR_NDIR];
static or_dual or_kink_abs(const or_dual &x, int site)
{
    for (int k = 0; k < OR_NDIR; ++k)
        if (std::fabs(x.v) < or_kink_eps * std::fabs(x.d[k])) {
#pragma omp atomic
            or_kinks[site][k] += 1;
        }
    return fabs(x);
}
#define OR_KINK_ABS(x, site) or_kink_abs((x), (site))
#else
typedef double real;
#define OR_VALUE(x) (x)
#define OR_KINK_ABS(x, site) fabs(x)
#endif
#include "gks_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NC 5 /* conservative components */
/* wall face tags (a wall face has no neighbour) */
#define TAG_SLIP 2
#define TAG_NOSLIP_ADIABATIC 3
#define TAG_NOSLIP_ISOTHERMAL 4
#define TAG_FARFIELD 5

/* ======================================================================== */
/* small dense linear algebra                                               */
/* ======================================================================== */

/* Solve A X = B by Gaussian elimination with partial pivoting.  A is n x n
 * (row-major, destroyed), B is n x m (row-major, overwritten by X).
 * Returns 0, or -1 if a pivot is exactly zero. */
static int gepp(int n, int m, real *A, real *B)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        real best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            real v = fabs(A[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) { real t = A[k*n+j]; A[k*n+j] = A[p*n+j]; A[p*n+j] = t; }
            for (int j = 0; j < m; ++j) { real t = B[k*m+j]; B[k*m+j] = B[p*m+j]; B[p*m+j] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            real f = A[i * n + k] / A[k * n + k];
            if (f == 0.0) continue;
            for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            for (int j = 0; j < m; ++j) B[i * m + j] -= f * B[k * m + j];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        for (int j = 0; j < m; ++j) {
            real s = B[k * m + j];
            for (int i = k + 1; i < n; ++i) s -= A[k * n + i] * B[i * m + j];
            B[k * m + j] = s / A[k * n + k];
        }
    }
    return 0;
}

/* ======================================================================== */
/* quadrature rules of the paper                                            */
/* ======================================================================== */

/* Sec. 4.1 (eq. base-int-change and the rule after it): five points on the
 * reference tetrahedron; centre weight -2/15, the other four 3/40. */
static const double VQ_PTS[5][3] = {
    {0.25, 0.25, 0.25},
    {0.5, 1.0 / 6.0, 1.0 / 6.0},
    {1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0},
    {1.0 / 6.0, 1.0 / 6.0, 0.5},
    {1.0 / 6.0, 0.5, 1.0 / 6.0},
};
static const double VQ_W[5] = {-2.0 / 15.0, 3.0 / 40.0, 3.0 / 40.0, 3.0 / 40.0, 3.0 / 40.0};

/* Sec. 2.1: three Gauss points on the reference triangle, weights 1/3
 * (the factor 1/2 of the reference area is applied separately). */
static const double FQ_PTS[3][2] = {
    {1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
static const double FQ_W[3] = {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0};

void or_volume_rule(double pts[15], double w[5])
{
    for (int q = 0; q < 5; ++q) {
        for (int d = 0; d < 3; ++d) pts[3 * q + d] = VQ_PTS[q][d];
        w[q] = VQ_W[q];
    }
}

void or_face_rule(double pts[6], double w[3])
{
    for (int q = 0; q < 3; ++q) {
        pts[2 * q] = FQ_PTS[q][0];
        pts[2 * q + 1] = FQ_PTS[q][1];
        w[q] = FQ_W[q];
    }
}

/* Linear (straight-edged) isoparametric tetrahedron: X = v0 + xi (v1-v0) +
 * eta (v2-v0) + zeta (v3-v0), the quadratic map of Sec. 4.1 when every edge
 * is straight. */
static void tet_map(const double v[4][3], const double xi[3], double X[3])
{
    for (int d = 0; d < 3; ++d)
        X[d] = v[0][d] + xi[0] * (v[1][d] - v[0][d]) + xi[1] * (v[2][d] - v[0][d]) +
               xi[2] * (v[3][d] - v[0][d]);
}

static double tet_jac(const double v[4][3])
{
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) {
        a[d] = v[1][d] - v[0][d];
        b[d] = v[2][d] - v[0][d];
        c[d] = v[3][d] - v[0][d];
    }
    return a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
           a[2] * (b[0] * c[1] - b[1] * c[0]);
}

/* Average over a tetrahedron of y^k, y = (x - origin) / h, for |k| <= 2:
 * out[0] = 1, out[1..3] = y_j, out[4..9] = (yy_xx, yy_yy, yy_zz, yy_xy,
 * yy_xz, yy_yz), by the five-point rule. */
static void tet_avg_monomials(const double v[4][3], const double origin[3], double h,
                              double out[10])
{
    double s[10] = {0};
    double wsum = 0.0;
    for (int q = 0; q < 5; ++q) {
        double X[3], y[3];
        tet_map(v, VQ_PTS[q], X);
        for (int d = 0; d < 3; ++d) y[d] = (X[d] - origin[d]) / h;
        double w = VQ_W[q];
        s[0] += w;
        s[1] += w * y[0]; s[2] += w * y[1]; s[3] += w * y[2];
        s[4] += w * y[0] * y[0]; s[5] += w * y[1] * y[1]; s[6] += w * y[2] * y[2];
        s[7] += w * y[0] * y[1]; s[8] += w * y[0] * y[2]; s[9] += w * y[1] * y[2];
        wsum += w;
    }
    for (int i = 0; i < 10; ++i) out[i] = s[i] / wsum;
}

/* Sec. 4.1: the ten shape functions of the quadratic tetrahedron at
 * xi = (xi, eta, zeta) and their derivatives; control points in the order of
 * the shape functions: the four vertices, then the points on the edges
 * (0,1), (1,2), (0,2), (0,3), (1,3), (2,3). */
static void qtet_shape(const double xi[3], double N[10], double dN[10][3])
{
    double a = xi[0], b = xi[1], g = xi[2], L = 1.0 - a - b - g;
    N[0] = L * (2.0 * L - 1.0);
    N[1] = a * (2.0 * a - 1.0);
    N[2] = b * (2.0 * b - 1.0);
    N[3] = g * (2.0 * g - 1.0);
    N[4] = 4.0 * a * L;
    N[5] = 4.0 * a * b;
    N[6] = 4.0 * b * L;
    N[7] = 4.0 * g * L;
    N[8] = 4.0 * g * a;
    N[9] = 4.0 * g * b;
    const double d[10][3] = {
        {1.0 - 4.0 * L, 1.0 - 4.0 * L, 1.0 - 4.0 * L},
        {4.0 * a - 1.0, 0.0, 0.0},
        {0.0, 4.0 * b - 1.0, 0.0},
        {0.0, 0.0, 4.0 * g - 1.0},
        {4.0 * (L - a), -4.0 * a, -4.0 * a},
        {4.0 * b, 4.0 * a, 0.0},
        {-4.0 * b, 4.0 * (L - b), -4.0 * b},
        {-4.0 * g, -4.0 * g, 4.0 * (L - g)},
        {4.0 * g, 0.0, 4.0 * a},
        {0.0, 4.0 * g, 4.0 * b},
    };
    memcpy(dN, d, sizeof(d));
}

/* The isoparametric map of a quadratic tetrahedron with control points x:
 * X(xi), and det dX/dxi there (eq. base-int-change). */
static double qtet_point(const double x[10][3], const double xi[3], double X[3])
{
    double N[10], dN[10][3], J[3][3] = {{0}};
    qtet_shape(xi, N, dN);
    for (int d = 0; d < 3; ++d) {
        X[d] = 0.0;
        for (int l = 0; l < 10; ++l) {
            X[d] += N[l] * x[l][d];
            for (int j = 0; j < 3; ++j) J[d][j] += dN[l][j] * x[l][d];
        }
    }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Sec. 2.1: the six shape functions of the quadratic triangle at (xi, eta)
 * and their derivatives; control points: the three vertices, then the
 * points on the edges (0,1), (1,2), (0,2). */
static void qtri_shape(double xi, double eta, double N[6], double dN[6][2])
{
    double L = 1.0 - xi - eta;
    N[0] = L * (2.0 * L - 1.0);
    N[1] = xi * (2.0 * xi - 1.0);
    N[2] = eta * (2.0 * eta - 1.0);
    N[3] = 4.0 * xi * L;
    N[4] = 4.0 * xi * eta;
    N[5] = 4.0 * eta * L;
    const double d[6][2] = {{1.0 - 4.0 * L, 1.0 - 4.0 * L}, {4.0 * xi - 1.0, 0.0}, {0.0, 4.0 * eta - 1.0},
                            {4.0 * (L - xi), -4.0 * xi}, {4.0 * eta, 4.0 * xi}, {-4.0 * eta, 4.0 * (L - eta)}};
    memcpy(dN, d, sizeof(d));
}

/* control-point index of the edge between local vertices a and b */
static const int QEDGE[4][4] = {{-1, 4, 6, 7}, {4, -1, 5, 8}, {6, 5, -1, 9}, {7, 8, 9, -1}};

/* ======================================================================== */
/* mesh and geometry                                                        */
/* ======================================================================== */

struct or_ctx {
    or_config cfg;
    int64_t nc, nf;
    double (*cv)[4][3];   /* cell vertex coordinates */
    double *vol;          /* |Omega| */
    double (*cen)[3];     /* centroid */
    double (*m2)[6];      /* centroid second moments / |Omega| */
    double *dr;           /* inscribed-sphere estimate 3|Omega| / sum |Gamma| */
    int64_t (*nbr)[4];    /* von Neumann neighbours (-1: none) */
    int64_t (*cface)[4];  /* the face shared with each neighbour slot */
    double (*noff)[4][3]; /* translation that brings the neighbour next to the cell */
    int64_t (*fcell)[2];
    int32_t *ftag;
    double (*fwu)[3];     /* velocity of a no-slip wall face (global frame) */
    double (*fshift)[3];
    double *farea;
    double (*fnorm)[3];
    double (*fgp)[3][3];  /* Gauss points, owner frame */
    double (*fpn)[3][3];  /* unit normal at each Gauss point (outward from the owner) */
    double (*fpw)[3];     /* weight of each Gauss point: omega_m of Sec. 2.1, the area included */
    int curved;           /* quadratic elements (control points given) */
    double (*cx)[10][3];  /* control points of each cell (curved meshes) */
    /* stage storage */
    real *Wn, *Ln, *Ltn;  /* W^n [5][nc], L(W^n), dL/dt(W^n) */
    char *fflat;          /* the face's Gauss points share one normal (bitwise) */
    real *FG0;            /* stage 1: sum_k w_k W_k(0) n_k per face [15][nf]; on a flat face
                             rows 0..4 hold sum_k w_k W_k(0) */
    real *fgrad;          /* last face terms: sum_k w_k W_k(0) n_k and sum_k w_k W_k(dt) n_k [30][nf] */
    real *slopes, *coef, *fterm;
    int32_t *flag;
    int have_stage1;
};

int or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

void or_destroy(or_ctx *c)
{
    if (!c) return;
    free(c->cv); free(c->vol); free(c->cen); free(c->m2); free(c->dr);
    free(c->nbr); free(c->cface); free(c->noff); free(c->fcell); free(c->ftag); free(c->fwu);
    free(c->fshift); free(c->farea); free(c->fnorm); free(c->fgp); free(c->fpn); free(c->fpw); free(c->cx);
    free(c->Wn); free(c->Ln); free(c->Ltn); free(c->FG0); free(c->fgrad); free(c->fflat);
    free(c->slopes); free(c->coef); free(c->fterm); free(c->flag);
    free(c);
}

or_ctx *or_create(const or_config *cfg, int64_t n_vert, const double *xyz,
                  int64_t n_cell, const int64_t *tet, int64_t n_face,
                  const int64_t *face_vert, const int64_t *face_cell,
                  const int32_t *face_tag, const double *face_shift, const double *face_wall_u)
{
    return or_create_quadratic(cfg, n_vert, xyz, n_cell, tet, n_face, face_vert, face_cell, face_tag,
                               face_shift, face_wall_u, NULL);
}

or_ctx *or_create_quadratic(const or_config *cfg, int64_t n_vert, const double *xyz,
                            int64_t n_cell, const int64_t *tet, int64_t n_face,
                            const int64_t *face_vert, const int64_t *face_cell,
                            const int32_t *face_tag, const double *face_shift, const double *face_wall_u,
                            const double *tet_mid)
{
    if (!cfg || n_cell <= 0 || n_face <= 0 || n_vert <= 0) return NULL;
    or_ctx *c = (or_ctx *)xcalloc(1, sizeof(or_ctx));
    c->cfg = *cfg;
    c->nc = n_cell;
    c->nf = n_face;
    int64_t nc = n_cell, nf = n_face;
    c->cv = (__typeof__(c->cv))xcalloc(nc, sizeof(*c->cv));
    c->vol = (__typeof__(c->vol))xcalloc(nc, sizeof(double));
    c->cen = (__typeof__(c->cen))xcalloc(nc, sizeof(*c->cen));
    c->m2 = (__typeof__(c->m2))xcalloc(nc, sizeof(*c->m2));
    c->dr = (__typeof__(c->dr))xcalloc(nc, sizeof(double));
    c->nbr = (__typeof__(c->nbr))xcalloc(nc, sizeof(*c->nbr));
    c->cface = (__typeof__(c->cface))xcalloc(nc, sizeof(*c->cface));
    c->noff = (__typeof__(c->noff))xcalloc(nc, sizeof(*c->noff));
    c->fcell = (__typeof__(c->fcell))xcalloc(nf, sizeof(*c->fcell));
    c->ftag = (__typeof__(c->ftag))xcalloc(nf, sizeof(int32_t));
    c->fwu = (__typeof__(c->fwu))xcalloc(nf, sizeof(*c->fwu));
    c->fshift = (__typeof__(c->fshift))xcalloc(nf, sizeof(*c->fshift));
    c->farea = (__typeof__(c->farea))xcalloc(nf, sizeof(double));
    c->fnorm = (__typeof__(c->fnorm))xcalloc(nf, sizeof(*c->fnorm));
    c->fgp = (__typeof__(c->fgp))xcalloc(nf, sizeof(*c->fgp));
    c->fpn = (__typeof__(c->fpn))xcalloc(nf, sizeof(*c->fpn));
    c->fpw = (__typeof__(c->fpw))xcalloc(nf, sizeof(*c->fpw));
    c->Wn = (real *)xcalloc(5 * nc, sizeof(real));
    c->Ln = (real *)xcalloc(5 * nc, sizeof(real));
    c->Ltn = (real *)xcalloc(5 * nc, sizeof(real));
    c->FG0 = (real *)xcalloc(15 * nf, sizeof(real));
    c->fflat = (char *)xcalloc(nf, 1);
    c->fgrad = (real *)xcalloc(30 * nf, sizeof(real));
    c->slopes = (real *)xcalloc(15 * nc, sizeof(real));
    c->coef = (real *)xcalloc(50 * nc, sizeof(real));
    c->fterm = (real *)xcalloc(20 * nf, sizeof(real));
    c->flag = (__typeof__(c->flag))xcalloc(nc, sizeof(int32_t));
    c->curved = tet_mid != NULL;
    if (c->curved) c->cx = (__typeof__(c->cx))xcalloc(nc, sizeof(*c->cx));

    /* cells: |Omega| = |J| / 6, centroid and second moments by the 5-point rule */
    for (int64_t i = 0; i < nc; ++i) {
        for (int a = 0; a < 4; ++a) {
            int64_t vv = tet[4 * i + a];
            if (vv < 0 || vv >= n_vert) { or_destroy(c); return NULL; }
            for (int d = 0; d < 3; ++d) c->cv[i][a][d] = xyz[3 * vv + d];
        }
        double J = fabs(tet_jac(c->cv[i]));
        if (!(J > 0.0)) { or_destroy(c); return NULL; }
        for (int a = 0; a < 4; ++a) { c->nbr[i][a] = -1; c->cface[i][a] = -1; }
        if (c->curved) {
            /* eq. base-int-change: |Omega|, the centroid and the second moments
             * by the five-point rule on the isoparametric map */
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d) c->cx[i][a][d] = c->cv[i][a][d];
            for (int e = 0; e < 6; ++e)
                for (int d = 0; d < 3; ++d) c->cx[i][4 + e][d] = tet_mid[(6 * i + e) * 3 + d];
            double X[5][3], w[5], V = 0.0, cen[3] = {0, 0, 0}, m2[6] = {0, 0, 0, 0, 0, 0};
            /* a valid element keeps the straight one's orientation at every point */
            double orient = tet_jac(c->cv[i]) > 0.0 ? 1.0 : -1.0;
            for (int q = 0; q < 5; ++q) {
                double dj = orient * qtet_point(c->cx[i], VQ_PTS[q], X[q]);
                if (!(dj > 0.0)) { or_destroy(c); return NULL; }
                w[q] = VQ_W[q] * dj;
                V += w[q];
            }
            if (!(V > 0.0)) { or_destroy(c); return NULL; }
            for (int q = 0; q < 5; ++q)
                for (int d = 0; d < 3; ++d) cen[d] += w[q] * X[q][d];
            for (int d = 0; d < 3; ++d) cen[d] /= V;
            for (int q = 0; q < 5; ++q) {
                double r[3] = {X[q][0] - cen[0], X[q][1] - cen[1], X[q][2] - cen[2]};
                m2[0] += w[q] * r[0] * r[0]; m2[1] += w[q] * r[1] * r[1]; m2[2] += w[q] * r[2] * r[2];
                m2[3] += w[q] * r[0] * r[1]; m2[4] += w[q] * r[0] * r[2]; m2[5] += w[q] * r[1] * r[2];
            }
            c->vol[i] = V;
            for (int d = 0; d < 3; ++d) c->cen[i][d] = cen[d];
            for (int k = 0; k < 6; ++k) c->m2[i][k] = m2[k] / V;
            continue;
        }
        c->vol[i] = J / 6.0;
        double zero[3] = {0, 0, 0}, mono[10];
        tet_avg_monomials(c->cv[i], zero, 1.0, mono);
        for (int d = 0; d < 3; ++d) c->cen[i][d] = mono[1 + d];
        tet_avg_monomials(c->cv[i], c->cen[i], 1.0, mono);
        for (int k = 0; k < 6; ++k) c->m2[i][k] = mono[4 + k];
    }

    /* faces: area, owner-outward unit normal and the three Gauss points */
    double *sumarea = (double *)xcalloc(nc, sizeof(double));
    for (int64_t f = 0; f < nf; ++f) {
        int64_t L = face_cell[2 * f], R = face_cell[2 * f + 1];
        if (L < 0 || L >= nc || R >= nc) { free(sumarea); or_destroy(c); return NULL; }
        c->fcell[f][0] = L;
        c->fcell[f][1] = R;
        c->ftag[f] = face_tag[f];
        if (R < 0 && face_tag[f] != TAG_SLIP && face_tag[f] != TAG_NOSLIP_ADIABATIC &&
            face_tag[f] != TAG_NOSLIP_ISOTHERMAL && face_tag[f] != TAG_FARFIELD) {
            free(sumarea); or_destroy(c); return NULL;
        }
        for (int d = 0; d < 3; ++d) c->fwu[f][d] = face_wall_u ? face_wall_u[3 * f + d] : 0.0;
        for (int d = 0; d < 3; ++d) c->fshift[f][d] = face_shift[3 * f + d];
        double x[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) x[a][d] = xyz[3 * face_vert[3 * f + a] + d];
        double Xxi[3], Xeta[3], cr[3];
        for (int d = 0; d < 3; ++d) { Xxi[d] = x[1][d] - x[0][d]; Xeta[d] = x[2][d] - x[0][d]; }
        cr[0] = Xxi[1] * Xeta[2] - Xxi[2] * Xeta[1];
        cr[1] = Xxi[2] * Xeta[0] - Xxi[0] * Xeta[2];
        cr[2] = Xxi[0] * Xeta[1] - Xxi[1] * Xeta[0];
        double nrm = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(nrm > 0.0)) { free(sumarea); or_destroy(c); return NULL; }
        c->farea[f] = 0.5 * nrm;
        for (int q = 0; q < 3; ++q) {
            double xi = FQ_PTS[q][0], eta = FQ_PTS[q][1];
            for (int d = 0; d < 3; ++d)
                c->fgp[f][q][d] = x[0][d] * (1.0 - xi - eta) + x[1][d] * xi + x[2][d] * eta;
        }
        double out = 0.0;
        for (int d = 0; d < 3; ++d) out += cr[d] * (c->fgp[f][0][d] - c->cen[L][d]);
        double sgn = out > 0 ? 1.0 : -1.0;
        for (int d = 0; d < 3; ++d) c->fnorm[f][d] = sgn * cr[d] / nrm;
        for (int q = 0; q < 3; ++q) {
            c->fpw[f][q] = FQ_W[q] * c->farea[f];
            for (int d = 0; d < 3; ++d) c->fpn[f][q][d] = c->fnorm[f][d];
        }
        if (c->curved) {
            /* Sec. 2.1, eq. flux-para-coord-gauss: the quadratic triangle through
             * the vertices and the owner's edge points; at each Gauss point the
             * normal X_xi x X_eta / |X_xi x X_eta| and the weight
             * (1/2) w_m |X_xi x X_eta| */
            double tx[6][3];
            int loc[3];
            for (int a = 0; a < 3; ++a) {
                loc[a] = -1;
                for (int k = 0; k < 4; ++k)
                    if (tet[4 * L + k] == face_vert[3 * f + a]) loc[a] = k;
                if (loc[a] < 0) { free(sumarea); or_destroy(c); return NULL; }
                for (int d = 0; d < 3; ++d) tx[a][d] = x[a][d];
            }
            const int ep[3][2] = {{0, 1}, {1, 2}, {0, 2}};
            for (int e = 0; e < 3; ++e)
                for (int d = 0; d < 3; ++d) tx[3 + e][d] = c->cx[L][QEDGE[loc[ep[e][0]]][loc[ep[e][1]]]][d];
            double area = 0.0;
            for (int q = 0; q < 3; ++q) {
                double N[6], dN[6][2], Xa[3] = {0, 0, 0}, Xb[3] = {0, 0, 0}, X[3] = {0, 0, 0}, cq[3];
                qtri_shape(FQ_PTS[q][0], FQ_PTS[q][1], N, dN);
                for (int l = 0; l < 6; ++l)
                    for (int d = 0; d < 3; ++d) {
                        X[d] += N[l] * tx[l][d];
                        Xa[d] += dN[l][0] * tx[l][d];
                        Xb[d] += dN[l][1] * tx[l][d];
                    }
                cq[0] = Xa[1] * Xb[2] - Xa[2] * Xb[1];
                cq[1] = Xa[2] * Xb[0] - Xa[0] * Xb[2];
                cq[2] = Xa[0] * Xb[1] - Xa[1] * Xb[0];
                double jq = sqrt(cq[0] * cq[0] + cq[1] * cq[1] + cq[2] * cq[2]);
                if (!(jq > 0.0)) { free(sumarea); or_destroy(c); return NULL; }
                c->fpw[f][q] = 0.5 * FQ_W[q] * jq;
                area += c->fpw[f][q];
                for (int d = 0; d < 3; ++d) {
                    c->fgp[f][q][d] = X[d];
                    c->fpn[f][q][d] = sgn * cq[d] / jq;
                }
            }
            c->farea[f] = area;
        }
        c->fflat[f] = 1;
        for (int q = 1; q < 3; ++q)
            for (int d = 0; d < 3; ++d)
                if (c->fpn[f][q][d] != c->fpn[f][0][d]) c->fflat[f] = 0;
        sumarea[L] += c->farea[f];
        if (R >= 0) sumarea[R] += c->farea[f];
        /* neighbour slots */
        int ok = 0;
        for (int a = 0; a < 4 && R >= 0; ++a)
            if (c->cface[L][a] < 0) {
                c->cface[L][a] = f; c->nbr[L][a] = R;
                for (int d = 0; d < 3; ++d) c->noff[L][a][d] = c->fshift[f][d];
                ok = 1; break;
            }
        if (R < 0) {
            for (int a = 0; a < 4; ++a)
                if (c->cface[L][a] < 0) { c->cface[L][a] = f; ok = 1; break; }
        }
        if (!ok) { free(sumarea); or_destroy(c); return NULL; }
        if (R >= 0) {
            ok = 0;
            for (int a = 0; a < 4; ++a)
                if (c->cface[R][a] < 0) {
                    c->cface[R][a] = f; c->nbr[R][a] = L;
                    for (int d = 0; d < 3; ++d) c->noff[R][a][d] = -c->fshift[f][d];
                    ok = 1; break;
                }
            if (!ok) { free(sumarea); or_destroy(c); return NULL; }
        }
    }
    /* Sec. 5, eq. time-step: inscribed-sphere estimate */
    for (int64_t i = 0; i < nc; ++i) c->dr[i] = 3.0 * c->vol[i] / sumarea[i];
    free(sumarea);
    for (int64_t i = 0; i < nc; ++i)
        for (int a = 0; a < 4; ++a)
            if (c->cface[i][a] < 0) { or_destroy(c); return NULL; }
    return c;
}

int or_geometry(const or_ctx *c, double *vol, double *cen, double *mom2, double *dr)
{
    int64_t n = c->nc;
    for (int64_t i = 0; i < n; ++i) {
        if (vol) vol[i] = c->vol[i];
        if (dr) dr[i] = c->dr[i];
        for (int d = 0; d < 3 && cen; ++d) cen[d * n + i] = c->cen[i][d];
        for (int k = 0; k < 6 && mom2; ++k) mom2[k * n + i] = c->m2[i][k];
    }
    return 0;
}

int or_face_points(const or_ctx *c, double *normal, double *weight)
{
    int64_t n = c->nf;
    for (int64_t f = 0; f < n; ++f)
        for (int q = 0; q < 3; ++q) {
            if (weight) weight[q * n + f] = c->fpw[f][q];
            for (int d = 0; d < 3 && normal; ++d) normal[(3 * q + d) * n + f] = c->fpn[f][q][d];
        }
    return 0;
}

int or_face_geometry(const or_ctx *c, double *area, double *normal, double *gp)
{
    int64_t n = c->nf;
    for (int64_t f = 0; f < n; ++f) {
        if (area) area[f] = c->farea[f];
        for (int d = 0; d < 3 && normal; ++d) normal[d * n + f] = c->fnorm[f][d];
        for (int q = 0; q < 3 && gp; ++q)
            for (int d = 0; d < 3; ++d) gp[(3 * q + d) * n + f] = c->fgp[f][q][d];
    }
    return 0;
}

/* The averages of tet_avg_monomials over cell m translated by shift; a
 * quadratic cell by the five-point rule on its isoparametric map (eq.
 * base-int-change), the weights times |det J|. */
static void cell_avg_monomials(const or_ctx *c, int64_t m, const double shift[3], const double origin[3],
                               double h, double out[10])
{
    if (!c->curved) {
        double v[4][3];
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) v[k][d] = c->cv[m][k][d] + shift[d];
        tet_avg_monomials(v, origin, h, out);
        return;
    }
    double x[10][3], s[10] = {0}, wsum = 0.0;
    for (int k = 0; k < 10; ++k)
        for (int d = 0; d < 3; ++d) x[k][d] = c->cx[m][k][d] + shift[d];
    for (int q = 0; q < 5; ++q) {
        double X[3], y[3];
        double w = VQ_W[q] * fabs(qtet_point(x, VQ_PTS[q], X));
        for (int d = 0; d < 3; ++d) y[d] = (X[d] - origin[d]) / h;
        s[0] += w;
        s[1] += w * y[0]; s[2] += w * y[1]; s[3] += w * y[2];
        s[4] += w * y[0] * y[0]; s[5] += w * y[1] * y[1]; s[6] += w * y[2] * y[2];
        s[7] += w * y[0] * y[1]; s[8] += w * y[0] * y[2]; s[9] += w * y[1] * y[2];
        wsum += w;
    }
    for (int k = 0; k < 10; ++k) out[k] = s[k] / wsum;
}

/* the same for neighbour slot a of cell i, translated next to cell i */
static void neighbour_monomials(const or_ctx *c, int64_t i, int a, double h, double out[10])
{
    cell_avg_monomials(c, c->nbr[i][a], c->noff[i][a], c->cen[i], h, out);
}

static const double NO_SHIFT[3] = {0.0, 0.0, 0.0};

/* ======================================================================== */
/* reconstruction, step 1 (Sec. 4.3): P^1 by least squares on the cell     */
/* averages of the von Neumann neighbours                                   */
/* ======================================================================== */

/* No-slip walls (Sec. 4.4): the velocity is prescribed on both kinds, the
 * temperature too on isothermal walls, so momentum is constrained at every
 * no-slip face and the energy at the isothermal ones; the density never. */
static int face_constrains(const or_ctx *c, int64_t f, int q)
{
    if (c->fcell[f][1] >= 0) return 0;
    int t = c->ftag[f];
    if (t != TAG_NOSLIP_ADIABATIC && t != TAG_NOSLIP_ISOTHERMAL) return 0;
    if (q >= 1 && q <= 3) return 1;
    return q == 4 && t == TAG_NOSLIP_ISOTHERMAL;
}

/* the prescribed value of component q at a point of wall face f, from the
 * density reconstructed there: rho U_wall, or rho (|U_wall|^2 / 2 +
 * T_wall / (gamma - 1)) with T = p / rho */
static real wall_value(const or_ctx *c, int64_t f, int q, real rho)
{
    const double *u = c->fwu[f];
    if (q <= 3) return rho * u[q - 1];
    return rho * (0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) + c->cfg.wall_T / (c->cfg.gamma - 1.0));
}

/* Boundary cells (Sec. 4.4, reconstruction for the boundary cells): with
 * fewer than three neighbours the cell's own averaged gradient serves as the
 * slopes; a singular least-squares matrix gives P^1 = P^0 (zero slopes).
 * Components constrained at no-slip faces (density first, then momentum and
 * energy from the reconstructed density) are fitted by constrained least
 * squares with one equality row at each constrained face's centre, if the
 * neighbours and constraints number at least three and the constraints at
 * most three. */
static void slopes_cell(const or_ctx *c, int64_t i, const real *W, const real *gW, real b[NC][3])
{
    int64_t n = c->nc;
    double h = cbrt(c->vol[i]);
    real D[4][3];
    int nn = 0;
    int64_t mm[4];
    for (int a = 0; a < 4; ++a) {
        if (c->nbr[i][a] < 0) continue;
        double mono[10];
        neighbour_monomials(c, i, a, h, mono);
        /* row m: average over Omega_m of the linear basis y_j (zero mean on Omega_0) */
        for (int d = 0; d < 3; ++d) D[nn][d] = mono[1 + d];
        mm[nn++] = c->nbr[i][a];
    }
    /* normal equations (D^T D) b' = D^T (Q_m - Q_0) for all components */
    real A[9], B[3 * NC];
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            real t = 0;
            for (int k = 0; k < nn; ++k) t += D[k][r] * D[k][s];
            A[3 * r + s] = t;
        }
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < NC; ++q) {
            real t = 0;
            for (int k = 0; k < nn; ++k) t += D[k][r] * (W[q * n + mm[k]] - W[q * n + i]);
            B[r * NC + q] = t;
        }
    real A0[9];
    memcpy(A0, A, sizeof(A));
    if (nn < 3) {
        for (int q = 0; q < NC; ++q)
            for (int d = 0; d < 3; ++d) b[q][d] = gW ? gW[(3 * q + d) * n + i] : 0.0;
    } else if (gepp(3, NC, A, B) != 0) {
        for (int q = 0; q < NC; ++q)
            for (int d = 0; d < 3; ++d) b[q][d] = 0.0;
    } else {
        for (int q = 0; q < NC; ++q)
            for (int d = 0; d < 3; ++d) b[q][d] = B[d * NC + q] / h; /* back to physical units */
    }
    /* no-slip walls: the constrained components, after the density */
    for (int q = 1; q < NC; ++q) {
        int64_t fl[4];
        int ncon = 0;
        for (int a = 0; a < 4; ++a)
            if (face_constrains(c, c->cface[i][a], q)) fl[ncon++] = c->cface[i][a];
        if (ncon == 0 || ncon > 3) continue; /* more than three: the plain fit above */
        if (nn + ncon < 3) {
            for (int d = 0; d < 3; ++d) b[q][d] = gW ? gW[(3 * q + d) * n + i] : 0.0;
            continue;
        }
        /* KKT system [D^T D  C^T; C  0] [b'; lambda] = [D^T (Q_m - Q_0); e] */
        int N = 3 + ncon;
        real K[36], R[6];
        memset(K, 0, sizeof(K));
        for (int r = 0; r < 3; ++r) {
            for (int s2 = 0; s2 < 3; ++s2) K[r * N + s2] = A0[3 * r + s2];
            real t = 0;
            for (int k = 0; k < nn; ++k) t += D[k][r] * (W[q * n + mm[k]] - W[q * n + i]);
            R[r] = t;
        }
        for (int j = 0; j < ncon; ++j) {
            int64_t f = fl[j];
            real x[3], rho = W[i];
            for (int d = 0; d < 3; ++d) {
                x[d] = (c->fgp[f][0][d] + c->fgp[f][1][d] + c->fgp[f][2][d]) / 3.0 - c->cen[i][d];
                rho += b[0][d] * x[d];
            }
            for (int r = 0; r < 3; ++r) K[r * N + 3 + j] = K[(3 + j) * N + r] = x[r] / h;
            R[3 + j] = wall_value(c, f, q, rho) - W[q * n + i];
        }
        if (gepp(N, 1, K, R) != 0) {
            for (int d = 0; d < 3; ++d) b[q][d] = 0.0;
        } else {
            for (int d = 0; d < 3; ++d) b[q][d] = R[d] / h;
        }
    }
}

int or_slopes(or_ctx *c, const real *W, const real *gW, real *b)
{
    int64_t n = c->nc;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        real s[NC][3];
        slopes_cell(c, i, W, gW, s);
        for (int q = 0; q < NC; ++q)
            for (int d = 0; d < 3; ++d) b[(3 * q + d) * n + i] = s[q][d];
    }
    return 0;
}

/* ======================================================================== */
/* reconstruction, step 2 (Secs. 4.1-4.3)                                   */
/* ======================================================================== */

/* polynomial about the centroid: value c0, gradient G, Hessian H
 * (xx,yy,zz,xy,xz,yz) -- P(r) = c0 + G.r + 1/2 r^T H r */
typedef struct { real c0, G[3], H[6]; } qpoly_t;

static real quad_eval(const qpoly_t *p, const double r[3])
{
    return p->c0 + p->G[0] * r[0] + p->G[1] * r[1] + p->G[2] * r[2] +
           0.5 * (p->H[0] * r[0] * r[0] + p->H[1] * r[1] * r[1] + p->H[2] * r[2] * r[2]) +
           p->H[3] * r[0] * r[1] + p->H[4] * r[0] * r[2] + p->H[5] * r[1] * r[2];
}

static void quad_grad(const qpoly_t *p, const double r[3], real g[3])
{
    g[0] = p->G[0] + p->H[0] * r[0] + p->H[3] * r[1] + p->H[4] * r[2];
    g[1] = p->G[1] + p->H[3] * r[0] + p->H[1] * r[1] + p->H[5] * r[2];
    g[2] = p->G[2] + p->H[4] * r[0] + p->H[5] * r[1] + p->H[2] * r[2];
}

static qpoly_t quad_lin(real a, const qpoly_t *p, real b, const qpoly_t *q)
{
    qpoly_t r;
    r.c0 = a * p->c0 + b * q->c0;
    for (int d = 0; d < 3; ++d) r.G[d] = a * p->G[d] + b * q->G[d];
    for (int k = 0; k < 6; ++k) r.H[k] = a * p->H[k] + b * q->H[k];
    return r;
}

/* exponent vectors of the 9 basis monomials y^k, 1 <= |k| <= 2 (eq. base) */
static const int KEXP[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0}, {0, 2, 0},
                               {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};

/* average of y^e for |e| <= 2 from the monomial table of tet_avg_monomials */
static double mono_lookup(const double mono[10], int ex, int ey, int ez)
{
    int s = ex + ey + ez;
    if (s == 0) return mono[0];
    if (s == 1) return ex ? mono[1] : (ey ? mono[2] : mono[3]);
    if (ex == 2) return mono[4];
    if (ey == 2) return mono[5];
    if (ez == 2) return mono[6];
    if (ex && ey) return mono[7];
    if (ex && ez) return mono[8];
    return mono[9];
}

/* Rows of the step-2 fit of cell i (eqs. large-stenci-condition-1/2), in
 * y = (x - c_0) / h for the basis y^k - <y^k>_0: E and e, the neighbour
 * averages (E[.][k] = <y^k>_m - <y^k>_0, e = Q_m - Q_0 per component); A and
 * bb, the neighbour averaged derivatives (bb = h dQ_m/dx_j). */
static void p2_rows(const or_ctx *c, int64_t i, const real *W, const real *gW, double mono0[10],
                    double E[4][9], real e[4][NC], double A[12][9], real bb[12][NC], int *ne_, int *na_)
{
    int64_t n = c->nc;
    double h = cbrt(c->vol[i]);
    cell_avg_monomials(c, i, NO_SHIFT, c->cen[i], h, mono0);
    int ne = 0, na = 0;
    for (int a = 0; a < 4; ++a) {
        int64_t m = c->nbr[i][a];
        if (m < 0) continue;
        double mono[10];
        neighbour_monomials(c, i, a, h, mono);
        for (int k = 0; k < 9; ++k)
            E[ne][k] = mono_lookup(mono, KEXP[k][0], KEXP[k][1], KEXP[k][2]) -
                       mono_lookup(mono0, KEXP[k][0], KEXP[k][1], KEXP[k][2]);
        for (int q = 0; q < NC; ++q) e[ne][q] = W[q * n + m] - W[q * n + i];
        ++ne;
        for (int j = 0; j < 3; ++j) {
            for (int k = 0; k < 9; ++k) {
                int ex[3] = {KEXP[k][0], KEXP[k][1], KEXP[k][2]};
                int kj = ex[j];
                if (kj == 0) { A[na][k] = 0.0; continue; }
                ex[j] -= 1;
                A[na][k] = kj * mono_lookup(mono, ex[0], ex[1], ex[2]);
            }
            for (int q = 0; q < NC; ++q) bb[na][q] = h * gW[(3 * q + j) * n + m];
            ++na;
        }
    }
    *ne_ = ne;
    *na_ = na;
}

/* The first-order polynomial fitted to the step-2 data (neighbour averages
 * and averaged derivatives) by least squares, normal equations on the three
 * linear coefficients: the fallback of Sec. 4.4 for component q. */
static void p2_linear(double E[4][9], real e[4][NC], double A[12][9], real bb[12][NC], int ne, int na,
                      double h, real Q0, int q, qpoly_t *p)
{
    real A3[9], B3[3];
    for (int r = 0; r < 3; ++r) {
        for (int s2 = 0; s2 < 3; ++s2) {
            real t = 0.0;
            for (int k = 0; k < ne; ++k) t += E[k][r] * E[k][s2];
            for (int k = 0; k < na; ++k) t += A[k][r] * A[k][s2];
            A3[3 * r + s2] = t;
        }
        real t = 0.0;
        for (int k = 0; k < ne; ++k) t += E[k][r] * e[k][q];
        for (int k = 0; k < na; ++k) t += A[k][r] * bb[k][q];
        B3[r] = t;
    }
    int rc3 = (ne + na) >= 3 ? gepp(3, 1, A3, B3) : -1;
    memset(p, 0, sizeof(*p));
    p->c0 = Q0;
    if (rc3 == 0)
        for (int d = 0; d < 3; ++d) p->G[d] = B3[d] / h;
}

/* P^2(y) = Q0 + sum_k a_k (y^k - <y^k>_0), back to physical r = h y */
static void p2_from_basis(const real ak[9], const double mono0[10], double h, real Q0, qpoly_t *p)
{
    p->c0 = Q0;
    for (int k = 3; k < 9; ++k) p->c0 -= ak[k] * mono_lookup(mono0, KEXP[k][0], KEXP[k][1], KEXP[k][2]);
    for (int d = 0; d < 3; ++d) p->G[d] = ak[d] / h;
    p->H[0] = 2.0 * ak[3] / (h * h);
    p->H[1] = 2.0 * ak[4] / (h * h);
    p->H[2] = 2.0 * ak[5] / (h * h);
    p->H[3] = ak[6] / (h * h);
    p->H[4] = ak[7] / (h * h);
    p->H[5] = ak[8] / (h * h);
}

/* Constrained least squares for P^2 (eqs. large-stenci-condition-1/2):
 * equality rows reproduce the neighbour averages, least-squares rows the
 * neighbour averaged derivatives; the cell's own averaged derivative is not
 * used.  Solved through the KKT system.  Returns per component the
 * polynomial about the centroid. */
static void p2_cell(const or_ctx *c, int64_t i, const real *W, const real *gW,
                    qpoly_t P2[NC])
{
    int64_t n = c->nc;
    double h = cbrt(c->vol[i]);
    double mono0[10], E[4][9], A[12][9];
    real e[4][NC], bb[12][NC];
    int ne, na;
    p2_rows(c, i, W, gW, mono0, E, e, A, bb, &ne, &na);
    /* KKT: [A^T A  E^T; E  0] [a; lambda] = [A^T b; e] */
    int N = 9 + ne;
    real K[13 * 13], B[13 * NC];
    memset(K, 0, sizeof(K));
    memset(B, 0, sizeof(B));
    for (int r = 0; r < 9; ++r) {
        for (int s = 0; s < 9; ++s) {
            real t = 0;
            for (int k = 0; k < na; ++k) t += A[k][r] * A[k][s];
            K[r * N + s] = t;
        }
        for (int s = 0; s < ne; ++s) K[r * N + 9 + s] = E[s][r];
        for (int q = 0; q < NC; ++q) {
            real t = 0;
            for (int k = 0; k < na; ++k) t += A[k][r] * bb[k][q];
            B[r * NC + q] = t;
        }
    }
    for (int s = 0; s < ne; ++s) {
        for (int r = 0; r < 9; ++r) K[(9 + s) * N + r] = E[s][r];
        for (int q = 0; q < NC; ++q) B[(9 + s) * NC + q] = e[s][q];
    }
    int rc = ne >= 3 ? gepp(N, NC, K, B) : -1;
    for (int q = 0; q < NC; ++q) {
        if (rc != 0) {
            /* boundary cells with fewer than three neighbours, or a singular
             * system (Sec. 4.4): the linear least-squares fallback */
            p2_linear(E, e, A, bb, ne, na, h, W[q * n + i], q, &P2[q]);
            continue;
        }
        real ak[9];
        for (int k = 0; k < 9; ++k) ak[k] = B[k * NC + q];
        memset(&P2[q], 0, sizeof(qpoly_t));
        p2_from_basis(ak, mono0, h, W[q * n + i], &P2[q]);
    }
}

/* Sec. 4.4, step 2, component q of a cell with no-slip faces that constrain
 * it: weighted constrained least squares whose equality rows are the wall
 * values at the Gauss points of those faces (three per face), from the
 * cell's reconstructed density Rrho there, and whose least-squares rows are
 * all the neighbour data (averages and averaged derivatives).  With more
 * than nine constraints, fewer than nine data and constraints together, or a
 * singular system: the linear least-squares fallback.  P is left unchanged
 * when no face constrains q. */
static void p2_wall(const or_ctx *c, int64_t i, const real *W, const real *gW, int q,
                    const qpoly_t *Rrho, qpoly_t *P)
{
    int64_t n = c->nc;
    int64_t fl[4];
    int nfc = 0;
    for (int a = 0; a < 4; ++a)
        if (face_constrains(c, c->cface[i][a], q)) fl[nfc++] = c->cface[i][a];
    if (nfc == 0) return;
    double h = cbrt(c->vol[i]);
    real Q0 = W[q * n + i];
    double mono0[10], E[4][9], A[12][9];
    real e[4][NC], bb[12][NC];
    int ne, na;
    p2_rows(c, i, W, gW, mono0, E, e, A, bb, &ne, &na);
    int ng = 3 * nfc;
    if (ng > 9 || 4 * ne + ng < 9) {
        p2_linear(E, e, A, bb, ne, na, h, Q0, q, P);
        return;
    }
    int N = 9 + ng;
    real K[18 * 18], B[18];
    memset(K, 0, sizeof(K));
    for (int r = 0; r < 9; ++r) {
        for (int s2 = 0; s2 < 9; ++s2) {
            real t = 0.0;
            for (int k = 0; k < ne; ++k) t += E[k][r] * E[k][s2];
            for (int k = 0; k < na; ++k) t += A[k][r] * A[k][s2];
            K[r * N + s2] = t;
        }
        real t = 0.0;
        for (int k = 0; k < ne; ++k) t += E[k][r] * e[k][q];
        for (int k = 0; k < na; ++k) t += A[k][r] * bb[k][q];
        B[r] = t;
    }
    for (int j = 0; j < nfc; ++j) {
        int64_t f = fl[j];
        for (int g = 0; g < 3; ++g) {
            int row = 9 + 3 * j + g;
            double x[3], y[3];
            for (int d = 0; d < 3; ++d) {
                x[d] = c->fgp[f][g][d] - c->cen[i][d];
                y[d] = x[d] / h;
            }
            for (int k = 0; k < 9; ++k) {
                real v = 1.0;
                for (int d = 0; d < 3; ++d)
                    for (int t = 0; t < KEXP[k][d]; ++t) v *= y[d];
                v -= mono_lookup(mono0, KEXP[k][0], KEXP[k][1], KEXP[k][2]);
                K[k * N + row] = K[row * N + k] = v;
            }
            B[row] = wall_value(c, f, q, quad_eval(Rrho, x)) - Q0;
        }
    }
    if (gepp(N, 1, K, B) != 0) {
        p2_linear(E, e, A, bb, ne, na, h, Q0, q, P);
        return;
    }
    memset(P, 0, sizeof(*P));
    p2_from_basis(B, mono0, h, Q0, P);
}

/* eq. smooth-indicator for a polynomial about the centroid of cell i, with
 * derivatives up to order r; the integrals use the five-point rule (exact
 * for the quadratic integrands that occur here on a straight cell; on a
 * quadratic cell the rule of eq. base-int-change). */
static real smoothness(const or_ctx *c, int64_t i, const qpoly_t *p, int r)
{
    real vol = c->vol[i];
    real s1 = 0.0, wsum = 0.0;
    for (int q = 0; q < 5; ++q) {
        double X[3], rr[3], w = VQ_W[q];
        real g[3];
        if (c->curved)
            w *= fabs(qtet_point(c->cx[i], VQ_PTS[q], X));
        else
            tet_map(c->cv[i], VQ_PTS[q], X);
        for (int d = 0; d < 3; ++d) rr[d] = X[d] - c->cen[i][d];
        quad_grad(p, rr, g);
        s1 += w * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        wsum += w;
    }
    /* integral over Omega = |Omega| * average */
    real beta = pow(vol, 2.0 / 3.0 - 1.0) * vol * (s1 / wsum);
    if (r >= 2) {
        real s2 = 0.0;
        for (int k = 0; k < 6; ++k) s2 += p->H[k] * p->H[k];
        if (c->cfg.weno_reading & OR_READ_MIXED2)
            for (int k = 3; k < 6; ++k) s2 += p->H[k] * p->H[k];
        beta += pow(vol, 4.0 / 3.0 - 1.0) * vol * s2;
    }
    return beta;
}

/* Gauss points of the four faces of cell i, relative to its centroid */
static int cell_face_points(const or_ctx *c, int64_t i, double r[12][3])
{
    int k = 0;
    for (int a = 0; a < 4; ++a) {
        int64_t f = c->cface[i][a];
        double sh[3] = {0, 0, 0};
        if (c->fcell[f][1] == i)
            for (int d = 0; d < 3; ++d) sh[d] = c->fshift[f][d];
        for (int q = 0; q < 3; ++q, ++k)
            for (int d = 0; d < 3; ++d) r[k][d] = c->fgp[f][q][d] - sh[d] - c->cen[i][d];
    }
    return k;
}

/* eq. p0-non-linear-weight: the two-step indicator of P^0 for component q,
 * from the neighbours' step-1 slopes */
static real beta0_two_step(const or_ctx *c, int64_t i, const real *slopes, int q)
{
    const or_config *cf = &c->cfg;
    int64_t n = c->nc;
    real vol23 = pow(c->vol[i], 2.0 / 3.0), eps = cf->eps_weno;
    real b0[4];
    int nb = 0;
    for (int a = 0; a < 4; ++a) {
        int64_t m = c->nbr[i][a];
        if (m < 0) continue;
        real s = 0;
        for (int d = 0; d < 3; ++d) {
            real v = slopes[(3 * q + d) * n + m];
            s += v * v;
        }
        b0[nb++] = ((cf->weno_reading & OR_READ_B0VOL) ? c->vol[i] : vol23) * s;
    }
    real beta0 = 0.0;
    if (nb > 0) {
        real sum = 0.0;
        int npair = 0;
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < j; ++k) { sum += OR_KINK_ABS(b0[j] - b0[k], 1); ++npair; }
        real sigma1 = npair ? pow(sum / npair, 4.0 / 3.0) : 0.0;
        real w[4], ws = 0.0;
        for (int j = 0; j < nb; ++j) {
            real r = sigma1 / (eps + b0[j]);
            w[j] = 1.0 + ((cf->weno_reading & OR_READ_POW1ST2) ? r * r : r);
            ws += w[j];
        }
        for (int j = 0; j < nb; ++j) beta0 += (w[j] / ws) * b0[j];
    }
    return beta0;
}

static int positivity_fallback(const or_ctx *c, int64_t i, const real *W, qpoly_t R[NC]);

/* (sigma / (eps + beta))^2 of eq. non-linear-weight (the first power under
 * the alternative reading OR_READ_POW1) */
static real wpow(real r, int reading) { return (reading & OR_READ_POW1) ? r : r * r; }

/* Second-order scheme (eq. final_weno_expression-2nd): R = w11 p1 + w01 p0
 * with p1 = (P^1 - g01 P^0) / g11, p0 = P^0, sigma = |beta1 - beta0|^(4/3) */
static int reconstruct_cell_2nd(const or_ctx *c, int64_t i, const real *W, const real *slopes,
                                qpoly_t R[NC])
{
    const or_config *cf = &c->cfg;
    int64_t n = c->nc;
    const double g11 = cf->lw1[0], g01 = cf->lw1[1], eps = cf->eps_weno;
    const int rd = cf->weno_reading;
    for (int q = 0; q < NC; ++q) {
        qpoly_t P0;
        memset(&P0, 0, sizeof(P0));
        P0.c0 = W[q * n + i];
        qpoly_t P1 = P0;
        for (int d = 0; d < 3; ++d) P1.G[d] = slopes[(3 * q + d) * n + i];
        if (!cf->nonlinear) { R[q] = P1; continue; }
        qpoly_t p1 = quad_lin(1.0 / g11, &P1, -g01 / g11, &P0);
        real beta1 = smoothness(c, i, (rd & OR_READ_BETA_LOWER) ? &p1 : &P1, 1);
        real beta0 = beta0_two_step(c, i, slopes, q);
        real sigma = pow(OR_KINK_ABS(beta1 - beta0, 1), (rd & OR_READ_SIGMA1) ? 1.0 : 4.0 / 3.0);
        real w1 = g11 * (1.0 + wpow(sigma / (eps + beta1), rd));
        real w0 = g01 * (1.0 + wpow(sigma / (eps + beta0), rd));
        real ws = w0 + w1;
        w0 /= ws; w1 /= ws;
        R[q] = quad_lin(w1, &p1, w0, &P0);
    }
    return positivity_fallback(c, i, W, R);
}

/* Secs. 4.2-4.3: multi-resolution WENO with the two-step indicator for P^0 */
static int reconstruct_cell(const or_ctx *c, int64_t i, const real *W, const real *gW,
                            const real *slopes, qpoly_t R[NC], qpoly_t *p2out)
{
    const or_config *cf = &c->cfg;
    int64_t n = c->nc;
    if (cf->order == 2) return reconstruct_cell_2nd(c, i, W, slopes, R);
    qpoly_t P2[NC];
    p2_cell(c, i, W, gW, P2);
    const double g22 = cf->lw2[0], g12 = cf->lw2[1], g02 = cf->lw2[2];
    const double g11 = cf->lw1[0], g01 = cf->lw1[1];
    const double eps = cf->eps_weno;
    const int rd = cf->weno_reading;
    for (int q = 0; q < NC; ++q) {
        real Q0 = W[q * n + i];
        qpoly_t P0;
        memset(&P0, 0, sizeof(P0));
        P0.c0 = Q0;
        qpoly_t P1 = P0;
        for (int d = 0; d < 3; ++d) P1.G[d] = slopes[(3 * q + d) * n + i];
        /* no-slip walls: momentum and energy from the reconstructed density */
        if (q > 0) p2_wall(c, i, W, gW, q, &R[0], &P2[q]);
        if (p2out) p2out[q] = P2[q];
        if (!cf->nonlinear) { R[q] = P2[q]; continue; }
        /* the three hierarchical polynomials */
        qpoly_t p0 = P0;
        qpoly_t p1 = quad_lin(1.0 / g11, &P1, -g01 / g11, &P0);
        qpoly_t t = quad_lin(1.0 / g22, &P2[q], -g12 / g22, &p1);
        qpoly_t p2 = quad_lin(1.0, &t, -g02 / g22, &p0);
        /* indicators of P^1 and P^2 */
        int lower = rd & OR_READ_BETA_LOWER;
        real beta1 = smoothness(c, i, lower ? &p1 : &P1, 1);
        real beta2 = smoothness(c, i, lower ? &p2 : &P2[q], 2);
        /* eq. p0-non-linear-weight: indicator of P^0 from the neighbours' slopes */
        real beta0 = beta0_two_step(c, i, slopes, q);
        /* global indicator and nonlinear weights (eq. non-linear-weight) */
        real sigma = pow(0.5 * (OR_KINK_ABS(beta2 - beta1, 1) + OR_KINK_ABS(beta2 - beta0, 1)),
                           (rd & OR_READ_SIGMA1) ? 1.0 : 4.0 / 3.0);
        real w2 = g22 * (1.0 + wpow(sigma / (eps + beta2), rd));
        real w1 = g12 * (1.0 + wpow(sigma / (eps + beta1), rd));
        real w0 = g02 * (1.0 + wpow(sigma / (eps + beta0), rd));
        real ws = w0 + w1 + w2;
        w0 /= ws; w1 /= ws; w2 /= ws;
        /* their weighted sum */
        qpoly_t s = quad_lin(w2, &p2, w1, &p1);
        R[q] = quad_lin(1.0, &s, w0, &p0);
    }
    return positivity_fallback(c, i, W, R);
}

/* positivity of density and pressure at the cell's face Gauss points;
 * otherwise the first-order (constant) reconstruction */
static int positivity_fallback(const or_ctx *c, int64_t i, const real *W, qpoly_t R[NC])
{
    const or_config *cf = &c->cfg;
    int64_t n = c->nc;
    double r[12][3];
    int np = cell_face_points(c, i, r);
    int bad = 0;
    for (int k = 0; k < np && !bad; ++k) {
        real v[NC];
        for (int q = 0; q < NC; ++q) v[q] = quad_eval(&R[q], r[k]);
        real rho = v[0];
        real pr = (cf->gamma - 1.0) * (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho);
        if (!(rho > 0.0) || !(pr > 0.0)) bad = 1;
    }
    if (bad) {
        for (int q = 0; q < NC; ++q) {
            memset(&R[q], 0, sizeof(qpoly_t));
            R[q].c0 = W[q * n + i];
        }
    }
    return bad;
}

static void pack_quad(const qpoly_t *p, real *out, int64_t n, int64_t i, int q)
{
    real *o = out + (size_t)(10 * q) * n + i;
    o[0] = p->c0;
    for (int d = 0; d < 3; ++d) o[(1 + d) * n] = p->G[d];
    for (int k = 0; k < 6; ++k) o[(4 + k) * n] = p->H[k];
}

int or_reconstruct(or_ctx *c, const real *W, const real *gW, real *coef, int32_t *flag,
                   real *p2coef)
{
    int64_t n = c->nc;
    or_slopes(c, W, gW, c->slopes);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        qpoly_t R[NC], P2[NC];
        memset(P2, 0, sizeof(P2)); /* the second-order scheme has no P^2 */
        int bad = reconstruct_cell(c, i, W, gW, c->slopes, R, P2);
        for (int q = 0; q < NC; ++q) {
            pack_quad(&R[q], coef, n, i, q);
            if (p2coef) pack_quad(&P2[q], p2coef, n, i, q);
        }
        if (flag) flag[i] = bad;
    }
    return 0;
}

/* ======================================================================== */
/* gas-kinetic solver (Sec. 2.2)                                            */
/* ======================================================================== */

/* A polynomial in the particle velocity (u, v, w) and xi^2, kept as an
 * unsimplified list of monomials c u^e0 v^e1 w^e2 (xi^2)^e3. */
#define MAXMONO 1024
#define NMOM 12
typedef struct { real c; int e[4]; } mono_t;
typedef struct { int n; mono_t m[MAXMONO]; } poly_t;

static void poly_zero(poly_t *p) { p->n = 0; }
static void poly_term(poly_t *p, real c, int eu, int ev, int ew, int ex)
{
    if (p->n >= MAXMONO) abort();
    mono_t *t = &p->m[p->n++];
    t->c = c; t->e[0] = eu; t->e[1] = ev; t->e[2] = ew; t->e[3] = ex;
}
static void poly_mul(const poly_t *a, const poly_t *b, poly_t *out)
{
    poly_zero(out);
    for (int i = 0; i < a->n; ++i)
        for (int j = 0; j < b->n; ++j)
            poly_term(out, a->m[i].c * b->m[j].c, a->m[i].e[0] + b->m[j].e[0],
                      a->m[i].e[1] + b->m[j].e[1], a->m[i].e[2] + b->m[j].e[2],
                      a->m[i].e[3] + b->m[j].e[3]);
}
static void poly_add_to(poly_t *acc, const poly_t *p, real s)
{
    for (int i = 0; i < p->n; ++i)
        poly_term(acc, s * p->m[i].c, p->m[i].e[0], p->m[i].e[1], p->m[i].e[2], p->m[i].e[3]);
}

/* psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2) / 2) */
static void poly_psi(int j, poly_t *p)
{
    poly_zero(p);
    switch (j) {
    case 0: poly_term(p, 1.0, 0, 0, 0, 0); break;
    case 1: poly_term(p, 1.0, 1, 0, 0, 0); break;
    case 2: poly_term(p, 1.0, 0, 1, 0, 0); break;
    case 3: poly_term(p, 1.0, 0, 0, 1, 0); break;
    default:
        poly_term(p, 0.5, 2, 0, 0, 0); poly_term(p, 0.5, 0, 2, 0, 0);
        poly_term(p, 0.5, 0, 0, 2, 0); poly_term(p, 0.5, 0, 0, 0, 1);
    }
}
/* s = s_j psi_j */
static void poly_slope(const real s[5], poly_t *p)
{
    poly_zero(p);
    for (int j = 0; j < 5; ++j) {
        poly_t t;
        poly_psi(j, &t);
        poly_add_to(p, &t, s[j]);
    }
}
static void poly_velocity(int d, poly_t *p) /* u_d */
{
    poly_zero(p);
    poly_term(p, 1.0, d == 0, d == 1, d == 2, 0);
}

/* Maxwellian g = rho (lam/pi)^((K+3)/2) exp(-lam((u-U)^2+(v-V)^2+(w-W)^2+xi^2)),
 * determined from W by eq. get-glr: rho E = rho (|U|^2/2 + (K+3)/(4 lam)).
 * Moments are normalised by rho. */
typedef struct {
    real rho, U, V, Wv, lam;
    real mu[NMOM], mup[NMOM], mun[NMOM], mv[NMOM], mw[NMOM], mx[4];
} maxw_t;

enum { FULL = 0, POS = 1, NEG = 2 };

static void full_moments(real U, real lam, real *m)
{
    m[0] = 1.0;
    m[1] = U;
    for (int k = 0; k + 2 < NMOM; ++k) m[k + 2] = U * m[k + 1] + (k + 1) / (2.0 * lam) * m[k];
}

static int maxwellian(const or_config *cf, const real W[5], maxw_t *g)
{
    real K = cf->K;
    g->rho = W[0];
    if (!(g->rho > 0.0)) return -1;
    g->U = W[1] / W[0];
    g->V = W[2] / W[0];
    g->Wv = W[3] / W[0];
    real ein = W[4] / W[0] - 0.5 * (g->U * g->U + g->V * g->V + g->Wv * g->Wv);
    if (!(ein > 0.0)) return -1;
    g->lam = (K + 3.0) / (4.0 * ein);
    real lam = g->lam;
    full_moments(g->U, lam, g->mu);
    full_moments(g->V, lam, g->mv);
    full_moments(g->Wv, lam, g->mw);
    /* half spaces: <u^0>_{u>0} = erfc(-sqrt(lam) U)/2,
     * <u^1>_{u>0} = U <u^0>_{u>0} + exp(-lam U^2) / (2 sqrt(pi lam)); the
     * same three-term recursion as the full moments holds above order 1 */
    real sl = sqrt(lam), ex = exp(-lam * g->U * g->U) / (2.0 * sqrt(M_PI * lam));
    g->mup[0] = 0.5 * erfc(-sl * g->U);
    g->mup[1] = g->U * g->mup[0] + ex;
    g->mun[0] = 0.5 * erfc(sl * g->U);
    g->mun[1] = g->U * g->mun[0] - ex;
    for (int k = 0; k + 2 < NMOM; ++k) {
        g->mup[k + 2] = g->U * g->mup[k + 1] + (k + 1) / (2.0 * lam) * g->mup[k];
        g->mun[k + 2] = g->U * g->mun[k + 1] + (k + 1) / (2.0 * lam) * g->mun[k];
    }
    /* internal variables: K Gaussian degrees of freedom of variance 1/(2 lam) */
    g->mx[0] = 1.0;
    g->mx[1] = K / (2.0 * lam);
    g->mx[2] = K * (K + 2.0) / (4.0 * lam * lam);
    g->mx[3] = K * (K + 2.0) * (K + 4.0) / (8.0 * lam * lam * lam);
    return 0;
}

/* normalised moment of a polynomial: integral of p g over the chosen half of
 * u, divided by rho */
static real moment(const poly_t *p, const maxw_t *g, int half)
{
    const real *mu = half == POS ? g->mup : (half == NEG ? g->mun : g->mu);
    real s = 0.0;
    for (int i = 0; i < p->n; ++i) {
        const mono_t *t = &p->m[i];
        if (t->e[0] >= NMOM || t->e[1] >= NMOM || t->e[2] >= NMOM || t->e[3] > 3) abort();
        s += t->c * mu[t->e[0]] * g->mv[t->e[1]] * g->mw[t->e[2]] * g->mx[t->e[3]];
    }
    return s;
}

/* vector of moments <X psi_j>, j = 0..4 */
static void moment_psi(const poly_t *X, const maxw_t *g, int half, real out[5])
{
    for (int j = 0; j < 5; ++j) {
        poly_t psi, t;
        poly_psi(j, &psi);
        poly_mul(X, &psi, &t);
        out[j] = moment(&t, g, half);
    }
}

/* eq. co: solve <psi psi^T> s = rhs (normalised by rho) for the slope s */
static int solve_slope(const maxw_t *g, const real rhs[5], real s[5])
{
    real M[25], B[5];
    for (int j = 0; j < 5; ++j)
        for (int k = 0; k < 5; ++k) {
            poly_t a, b, t;
            poly_psi(j, &a);
            poly_psi(k, &b);
            poly_mul(&a, &b, &t);
            M[5 * j + k] = moment(&t, g, FULL);
        }
    for (int j = 0; j < 5; ++j) B[j] = rhs[j];
    if (gepp(5, 1, M, B) != 0) return -1;
    for (int j = 0; j < 5; ++j) s[j] = B[j];
    return 0;
}

/* A from the compatibility condition <A + a_x u + a_y v + a_z w> = 0 */
static int solve_time_slope(const maxw_t *g, real a[3][5], real A[5])
{
    real rhs[5] = {0, 0, 0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        poly_t sp, ud, t;
        poly_slope(a[d], &sp);
        poly_velocity(d, &ud);
        poly_mul(&ud, &sp, &t);
        real m[5];
        moment_psi(&t, g, FULL, m);
        for (int j = 0; j < 5; ++j) rhs[j] -= m[j];
    }
    return solve_slope(g, rhs, A);
}

/* rotation of eq. rotate-matrix-3d (Lambda when n1 = -1) */
static void rotation(const double n[3], double T[3][3])
{
    if (n[0] == -1.0) {
        T[0][0] = -1; T[0][1] = 0; T[0][2] = 0;
        T[1][0] = 0; T[1][1] = -1; T[1][2] = 0;
        T[2][0] = 0; T[2][1] = 0; T[2][2] = 1;
        return;
    }
    double n1 = n[0], n2 = n[1], n3 = n[2];
    T[0][0] = n1; T[0][1] = n2; T[0][2] = n3;
    T[1][0] = -n2; T[1][1] = n1 + n3 * n3 / (1.0 + n1); T[1][2] = -n2 * n3 / (1.0 + n1);
    T[2][0] = -n3; T[2][1] = -n2 * n3 / (1.0 + n1); T[2][2] = 1.0 - n3 * n3 / (1.0 + n1);
}

/* state and gradient into the local frame: W~ = T W; derivative along local
 * axis j is sum_i T_ji d/dx_i, then T on the components */
static void to_local(const double T[3][3], const real W[5], const real gW[15],
                     real Wl[5], real gl[3][5])
{
    Wl[0] = W[0];
    Wl[4] = W[4];
    for (int r = 0; r < 3; ++r) Wl[1 + r] = T[r][0] * W[1] + T[r][1] * W[2] + T[r][2] * W[3];
    for (int j = 0; j < 3; ++j) {
        real dW[5];
        for (int q = 0; q < 5; ++q)
            dW[q] = T[j][0] * gW[3 * q + 0] + T[j][1] * gW[3 * q + 1] + T[j][2] * gW[3 * q + 2];
        gl[j][0] = dW[0];
        gl[j][4] = dW[4];
        for (int r = 0; r < 3; ++r) gl[j][1 + r] = T[r][0] * dW[1] + T[r][1] * dW[2] + T[r][2] * dW[3];
    }
}

/* back to the global frame with T^{-1} = T^T */
static void to_global(const double T[3][3], const real Fl[5], real F[5])
{
    F[0] = Fl[0];
    F[4] = Fl[4];
    for (int r = 0; r < 3; ++r) F[1 + r] = T[0][r] * Fl[1] + T[1][r] * Fl[2] + T[2][r] * Fl[3];
}

/* Moment vectors of the three parts of eq. 2nd-flux for one Maxwellian:
 *   F0 = <u psi>, F1 = sum_d <u u_d (a_d.psi) psi>, F2 = <u (A.psi) psi>,
 *   V0 = <psi>,   V1 = sum_d <u_d (a_d.psi) psi>,   V2 = <(A.psi) psi>,
 *   Q0..Q2 = the same with the heat-flux weight in place of u psi. */
typedef struct { real F[3][5], V[3][5], Q[3]; } parts_t;

static void part_moments(const maxw_t *g, int half, real a[3][5], const real A[5],
                         const poly_t *qw, parts_t *P)
{
    poly_t one, u, sumF, sumV, As, t, tt;
    poly_zero(&one);
    poly_term(&one, 1.0, 0, 0, 0, 0);
    poly_velocity(0, &u);
    poly_zero(&sumV);
    for (int d = 0; d < 3; ++d) {
        poly_t sp, ud;
        poly_slope(a[d], &sp);
        poly_velocity(d, &ud);
        poly_mul(&ud, &sp, &t);
        poly_add_to(&sumV, &t, 1.0);
    }
    poly_mul(&u, &sumV, &sumF);
    poly_slope(A, &As);
    moment_psi(&u, g, half, P->F[0]);
    moment_psi(&sumF, g, half, P->F[1]);
    poly_mul(&u, &As, &t);
    moment_psi(&t, g, half, P->F[2]);
    moment_psi(&one, g, half, P->V[0]);
    moment_psi(&sumV, g, half, P->V[1]);
    moment_psi(&As, g, half, P->V[2]);
    P->Q[0] = moment(qw, g, half);
    poly_mul(qw, &sumV, &tt);
    P->Q[1] = moment(&tt, g, half);
    poly_mul(qw, &As, &tt);
    P->Q[2] = moment(&tt, g, half);
}

/* Everything the time-dependent distribution of eq. 2nd-flux needs at one
 * point, in the local frame. */
typedef struct {
    real rhoc, rhol, rhor, tau, taun;
    int smooth; /* eq. 2nd-smooth-flux: the equilibrium part alone */
    parts_t c, l, r;
} interface_t;

static int build_interface(const or_config *cf, const real Wl[5], real gl[3][5],
                           const real Wr[5], real gr[3][5], double dt, interface_t *I)
{
    maxw_t ml, mr, mc;
    if (maxwellian(cf, Wl, &ml) || maxwellian(cf, Wr, &mr)) return -1;
    /* microscopic slopes of both sides, eq. co */
    real al[3][5], ar[3][5];
    for (int d = 0; d < 3; ++d) {
        real bl[5], br[5];
        for (int q = 0; q < 5; ++q) { bl[q] = gl[d][q] / ml.rho; br[q] = gr[d][q] / mr.rho; }
        if (solve_slope(&ml, bl, al[d]) || solve_slope(&mr, br, ar[d])) return -1;
    }
    /* eq. new-equ-part: kinetic weighting of the equilibrium and its slopes */
    real Wc[5], gc[3][5];
    {
        poly_t one;
        poly_zero(&one);
        poly_term(&one, 1.0, 0, 0, 0, 0);
        real mp[5], mn[5];
        moment_psi(&one, &ml, POS, mp);
        moment_psi(&one, &mr, NEG, mn);
        for (int q = 0; q < 5; ++q) Wc[q] = ml.rho * mp[q] + mr.rho * mn[q];
        for (int d = 0; d < 3; ++d) {
            poly_t sl, sr;
            poly_slope(al[d], &sl);
            poly_slope(ar[d], &sr);
            moment_psi(&sl, &ml, POS, mp);
            moment_psi(&sr, &mr, NEG, mn);
            for (int q = 0; q < 5; ++q) gc[d][q] = ml.rho * mp[q] + mr.rho * mn[q];
        }
    }
    if (maxwellian(cf, Wc, &mc)) return -1;
    real ac[3][5], Ac[5], Al[5] = {0, 0, 0, 0, 0}, Ar[5] = {0, 0, 0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        real b[5];
        for (int q = 0; q < 5; ++q) b[q] = gc[d][q] / mc.rho;
        if (solve_slope(&mc, b, ac[d])) return -1;
    }
    if (solve_time_slope(&mc, ac, Ac)) return -1;
    /* collision times (Sec. 2.2) */
    real pl = ml.rho / (2.0 * ml.lam), pr = mr.rho / (2.0 * mr.lam), pc = mc.rho / (2.0 * mc.lam);
    real jump = cf->c_tau * OR_KINK_ABS((pl - pr) / (pl + pr), 0) * dt;
    if (cf->viscous) {
        I->tau = cf->mu / pc;
        I->taun = cf->mu / pc + jump;
    } else {
        I->tau = 0.0;
        I->taun = cf->eps_tau * dt + jump;
    }
    /* eq. 2nd-smooth-flux keeps tau = mu / p (0 for Euler) and drops tau_n
     * with the kinetic part */
    I->smooth = cf->flux == 1;
    if (I->tau > 0.0 && !I->smooth) {
        if (solve_time_slope(&ml, al, Al) || solve_time_slope(&mr, ar, Ar)) return -1;
    }
    /* heat-flux weight (u-U^c)(|u-U^c|^2 + xi^2)/2 about the interface velocity */
    poly_t du, dv, dw, c2, t, qw;
    poly_zero(&du); poly_term(&du, 1.0, 1, 0, 0, 0); poly_term(&du, -mc.U, 0, 0, 0, 0);
    poly_zero(&dv); poly_term(&dv, 1.0, 0, 1, 0, 0); poly_term(&dv, -mc.V, 0, 0, 0, 0);
    poly_zero(&dw); poly_term(&dw, 1.0, 0, 0, 1, 0); poly_term(&dw, -mc.Wv, 0, 0, 0, 0);
    poly_zero(&c2);
    poly_mul(&du, &du, &t); poly_add_to(&c2, &t, 1.0);
    poly_mul(&dv, &dv, &t); poly_add_to(&c2, &t, 1.0);
    poly_mul(&dw, &dw, &t); poly_add_to(&c2, &t, 1.0);
    poly_term(&c2, 1.0, 0, 0, 0, 1);
    poly_mul(&du, &c2, &qw);
    for (int i = 0; i < qw.n; ++i) qw.m[i].c *= 0.5;

    I->rhoc = mc.rho;
    I->rhol = ml.rho;
    I->rhor = mr.rho;
    part_moments(&mc, FULL, ac, Ac, &qw, &I->c);
    if (I->smooth) {
        memset(&I->l, 0, sizeof(parts_t));
        memset(&I->r, 0, sizeof(parts_t));
    } else {
        part_moments(&ml, POS, al, Al, &qw, &I->l);
        part_moments(&mr, NEG, ar, Ar, &qw, &I->r);
    }
    return 0;
}

/* time integral over [0, delta] of eq. 2nd-flux taken against u psi */
static void integrated_flux(const or_config *cf, const interface_t *I, double delta, real F[5])
{
    real tau = I->tau, tn = I->taun;
    real c1, c2, c3, c4, c5, c6;
    if (I->smooth) {
        /* eq. 2nd-smooth-flux: g^c - tau (a^c.u + A^c) g^c + t A^c g^c,
         * integrated over [0, delta] */
        c1 = delta;
        c2 = -tau * delta;
        c3 = 0.5 * delta * delta - tau * delta;
        c4 = c5 = c6 = 0.0;
    } else {
        real e = exp(-delta / tn);
        real E1 = tn * (1.0 - e);
        real E2 = tn * tn * (1.0 - e) - tn * delta * e;
        c1 = delta - E1;
        c2 = E2 + tau * E1 - tau * delta;
        c3 = 0.5 * delta * delta - tau * delta + tau * E1;
        c4 = E1;
        c5 = -(tau * E1 + E2);
        c6 = -tau * E1;
    }
    for (int q = 0; q < 5; ++q)
        F[q] = I->rhoc * (c1 * I->c.F[0][q] + c2 * I->c.F[1][q] + c3 * I->c.F[2][q]) +
               I->rhol * (c4 * I->l.F[0][q] + c5 * I->l.F[1][q] + c6 * I->l.F[2][q]) +
               I->rhor * (c4 * I->r.F[0][q] + c5 * I->r.F[1][q] + c6 * I->r.F[2][q]);
    if (cf->prandtl != 1.0) {
        real qh = I->rhoc * (c1 * I->c.Q[0] + c2 * I->c.Q[1] + c3 * I->c.Q[2]) +
                    I->rhol * (c4 * I->l.Q[0] + c5 * I->l.Q[1] + c6 * I->l.Q[2]) +
                    I->rhor * (c4 * I->r.Q[0] + c5 * I->r.Q[1] + c6 * I->r.Q[2]);
        F[4] += (1.0 / cf->prandtl - 1.0) * qh;
    }
}

/* the coefficients of eq. 2nd-flux at time t (un-integrated) */
static void point_coeffs(const interface_t *I, double t, real d[6])
{
    real tau = I->tau;
    if (I->smooth) { /* eq. 2nd-smooth-flux */
        d[0] = 1.0;
        d[1] = -tau;
        d[2] = t - tau;
        d[3] = d[4] = d[5] = 0.0;
        return;
    }
    real e = exp(-t / I->taun);
    d[0] = 1.0 - e;
    d[1] = (t + tau) * e - tau;
    d[2] = t - tau + tau * e;
    d[3] = e;
    d[4] = -(tau + t) * e;
    d[5] = -tau * e;
}

/* eq. point-interface: conservative variables of the distribution at time t */
static void point_state(const interface_t *I, double t, real Wt[5])
{
    real d[6];
    point_coeffs(I, t, d);
    for (int q = 0; q < 5; ++q)
        Wt[q] = I->rhoc * (d[0] * I->c.V[0][q] + d[1] * I->c.V[1][q] + d[2] * I->c.V[2][q]) +
                I->rhol * (d[3] * I->l.V[0][q] + d[4] * I->l.V[1][q] + d[5] * I->l.V[2][q]) +
                I->rhor * (d[3] * I->r.V[0][q] + d[4] * I->r.V[1][q] + d[5] * I->r.V[2][q]);
}

static void point_flux_density(const or_config *cf, const interface_t *I, double t, real F[5])
{
    real d[6];
    point_coeffs(I, t, d);
    for (int q = 0; q < 5; ++q)
        F[q] = I->rhoc * (d[0] * I->c.F[0][q] + d[1] * I->c.F[1][q] + d[2] * I->c.F[2][q]) +
               I->rhol * (d[3] * I->l.F[0][q] + d[4] * I->l.F[1][q] + d[5] * I->l.F[2][q]) +
               I->rhor * (d[3] * I->r.F[0][q] + d[4] * I->r.F[1][q] + d[5] * I->r.F[2][q]);
    if (cf->prandtl != 1.0) {
        real qh = I->rhoc * (d[0] * I->c.Q[0] + d[1] * I->c.Q[1] + d[2] * I->c.Q[2]) +
                    I->rhol * (d[3] * I->l.Q[0] + d[4] * I->l.Q[1] + d[5] * I->l.Q[2]) +
                    I->rhor * (d[3] * I->r.Q[0] + d[4] * I->r.Q[1] + d[5] * I->r.Q[2]);
        F[4] += (1.0 / cf->prandtl - 1.0) * qh;
    }
}

/* gas-kinetic solver at one point in the global frame; out[20] =
 * F(dt), F(dt/2), W(0), W(dt) */
static int gks_point(const or_config *cf, const double n[3], const real Wl[5],
                     const real gWl[15], const real Wr[5], const real gWr[15],
                     double dt, real out[20])
{
    double T[3][3];
    real wl[5], wr[5], gl[3][5], gr[3][5];
    rotation(n, T);
    to_local(T, Wl, gWl, wl, gl);
    to_local(T, Wr, gWr, wr, gr);
    interface_t I;
    if (build_interface(cf, wl, gl, wr, gr, dt, &I)) return -1;
    real loc[4][5];
    integrated_flux(cf, &I, dt, loc[0]);
    integrated_flux(cf, &I, 0.5 * dt, loc[1]);
    point_state(&I, 0.0, loc[2]);
    point_state(&I, dt, loc[3]);
    for (int k = 0; k < 4; ++k) to_global(T, loc[k], out + 5 * k);
    return 0;
}

int or_point_flux(const or_config *cf, const double n[3], const real Wl[5],
                  const real gWl[15], const real Wr[5], const real gWr[15], double dt,
                  real out[20])
{
    return gks_point(cf, n, Wl, gWl, Wr, gWr, dt, out);
}

int or_point_flux_density(const or_config *cf, const double n[3], const real Wl[5],
                          const real gWl[15], const real Wr[5], const real gWr[15],
                          double dt, double t, real out[5])
{
    double T[3][3];
    real wl[5], wr[5], gl[3][5], gr[3][5], loc[5];
    rotation(n, T);
    to_local(T, Wl, gWl, wl, gl);
    to_local(T, Wr, gWr, wr, gr);
    interface_t I;
    if (build_interface(cf, wl, gl, wr, gr, dt, &I)) return -1;
    point_flux_density(cf, &I, t, loc);
    to_global(T, loc, out);
    return 0;
}

int or_maxwell_moments(const or_config *cf, const real W[5], real out[54])
{
    maxw_t g;
    if (maxwellian(cf, W, &g)) return -1;
    for (int k = 0; k < 10; ++k) {
        out[k] = g.mu[k];
        out[10 + k] = g.mup[k];
        out[20 + k] = g.mun[k];
        out[30 + k] = g.mv[k];
        out[40 + k] = g.mw[k];
    }
    for (int k = 0; k < 4; ++k) out[50 + k] = g.mx[k];
    return 0;
}

/* ======================================================================== */
/* face terms and the two-stage update (Secs. 2.1, 2.3, 3)                  */
/* ======================================================================== */

static void quad_from_coef(const real *coef, int64_t n, int64_t i, int q, qpoly_t *p)
{
    const real *o = coef + (size_t)(10 * q) * n + i;
    p->c0 = o[0];
    for (int d = 0; d < 3; ++d) p->G[d] = o[(1 + d) * n];
    for (int k = 0; k < 6; ++k) p->H[k] = o[(4 + k) * n];
}

/* Slip wall (Sec. 4.4, ghost states): the ghost is the mirror image of the
 * interior solution in the wall plane.  With the reflection P = I - 2 n n^T
 * (P = P^T = P^-1): density and energy W_g(x) = W(P x), momentum
 * m_g(x) = P m(P x); at a point of the wall (P x = x) this gives the ghost
 * value, and by the chain rule grad s_g = P grad s for the scalars and
 * J_g = P J P for the momentum Jacobian J_ab = dm_a/dx_b. */
static void mirror_ghost(const double n[3], const real W[5], const real gW[15], real Wg[5],
                         real gWg[15])
{
    real P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * n[a] * n[b];
    Wg[0] = W[0];
    Wg[4] = W[4];
    for (int a = 0; a < 3; ++a) {
        Wg[1 + a] = 0.0;
        for (int b = 0; b < 3; ++b) Wg[1 + a] += P[a][b] * W[1 + b];
    }
    for (int q = 0; q < 5; q += 4)
        for (int a = 0; a < 3; ++a) {
            gWg[3 * q + a] = 0.0;
            for (int b = 0; b < 3; ++b) gWg[3 * q + a] += P[a][b] * gW[3 * q + b];
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            real t = 0.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) t += P[a][k] * gW[3 * (1 + k) + l] * P[l][b];
            gWg[3 * (1 + a) + b] = t;
        }
}

/* No-slip wall ghost (Sec. 4.4).  The interior point state is mapped to
 * primitive variables with the paper's chain rule (T = p / rho); the ghost
 * reflects it through the wall point: velocity 2 U_wall - U with unchanged
 * derivatives, the same pressure with reversed derivatives, and the same
 * temperature with reversed derivatives (adiabatic) or 2 T_wall - T with
 * unchanged derivatives (isothermal); then back to conservative variables by
 * the same chain rule.  At rest on an adiabatic wall this is the paper's
 * (rho, -rho U, rho E) with unchanged momentum derivatives and reversed
 * density and energy derivatives. */
static void noslip_ghost(const or_config *cf, int iso, const double uw[3], const real W[5],
                         const real gW[15], real Wg[5], real gWg[15])
{
    real g1 = cf->gamma - 1.0;
    real rho = W[0], U[3], Q = 0.0;
    for (int d = 0; d < 3; ++d) { U[d] = W[1 + d] / rho; Q += 0.5 * U[d] * U[d]; }
    real p = g1 * (W[4] - rho * Q), T = p / rho;
    real Ug[3], Qg = 0.0;
    for (int d = 0; d < 3; ++d) { Ug[d] = 2.0 * uw[d] - U[d]; Qg += 0.5 * Ug[d] * Ug[d]; }
    real Tg = iso ? 2.0 * cf->wall_T - T : T, pg = p, rhog = pg / Tg;
    Wg[0] = rhog;
    for (int d = 0; d < 3; ++d) Wg[1 + d] = rhog * Ug[d];
    Wg[4] = rhog * Qg + pg / g1;
    for (int j = 0; j < 3; ++j) { /* derivatives along axis j */
        real drho = gW[j], dU[3], dQ = 0.0;
        for (int d = 0; d < 3; ++d) { dU[d] = (gW[3 * (1 + d) + j] - drho * U[d]) / rho; dQ += U[d] * dU[d]; }
        real dp = g1 * (gW[12 + j] - drho * Q - rho * dQ);
        real dT = (dp - drho * T) / rho;
        real dTg = iso ? dT : -dT, dpg = -dp, dQg = 0.0;
        real drhog = (dpg - dTg * rhog) / Tg;
        gWg[j] = drhog;
        for (int d = 0; d < 3; ++d) { gWg[3 * (1 + d) + j] = drhog * Ug[d] + rhog * dU[d]; dQg += Ug[d] * dU[d]; }
        gWg[12 + j] = drhog * Qg + rhog * dQg + dpg / g1;
    }
}

/* Far field (the Riemann invariants of the paper's external-flow cases): the
 * locally one-dimensional characteristic state along the outward normal n.
 * Supersonic outflow takes the interior state, supersonic inflow the free
 * stream; otherwise the outgoing invariant u_n + 2a/(gamma-1) comes from the
 * interior and the incoming u_n - 2a/(gamma-1) from the free stream, and the
 * entropy p/rho^gamma and tangential velocity from the side the flow comes
 * from.  The ghost is uniform (zero gradients). */
static void farfield_ghost(const or_config *cf, const double n[3], const real W[5], real Wg[5],
                           real gWg[15])
{
    double g = cf->gamma, g1 = g - 1.0;
    const double *Wf = cf->farfield;
    real ri = W[0], rf = Wf[0], Ui[3], Uf[3], ki = 0.0, kf = 0.0, uni = 0.0, unf = 0.0;
    for (int d = 0; d < 3; ++d) {
        Ui[d] = W[1 + d] / ri;
        Uf[d] = Wf[1 + d] / rf;
        ki += 0.5 * Ui[d] * Ui[d];
        kf += 0.5 * Uf[d] * Uf[d];
        uni += Ui[d] * n[d];
        unf += Uf[d] * n[d];
    }
    real pi = g1 * (W[4] - ri * ki), pf = g1 * (Wf[4] - rf * kf);
    real ai = sqrt(g * pi / ri), af = sqrt(g * pf / rf);
    for (int k = 0; k < 15; ++k) gWg[k] = 0.0;
    if (uni >= ai) { /* supersonic outflow */
        for (int q = 0; q < 5; ++q) Wg[q] = W[q];
        return;
    }
    if (uni <= -ai) { /* supersonic inflow */
        for (int q = 0; q < 5; ++q) Wg[q] = Wf[q];
        return;
    }
    real Rp = uni + 2.0 * ai / g1, Rm = unf - 2.0 * af / g1;
    real ub = 0.5 * (Rp + Rm), ab = 0.25 * g1 * (Rp - Rm);
    real s, Ut[3];
    if (ub > 0.0) {
        s = pi / pow(ri, g);
        for (int d = 0; d < 3; ++d) Ut[d] = Ui[d] - uni * n[d];
    } else {
        s = pf / pow(rf, g);
        for (int d = 0; d < 3; ++d) Ut[d] = Uf[d] - unf * n[d];
    }
    real rb = pow(ab * ab / (g * s), 1.0 / g1), pb = rb * ab * ab / g, kb = 0.0;
    Wg[0] = rb;
    for (int d = 0; d < 3; ++d) {
        real u = Ut[d] + ub * n[d];
        Wg[1 + d] = rb * u;
        kb += 0.5 * u * u;
    }
    Wg[4] = pb / g1 + rb * kb;
}

int or_wall_ghost(const or_config *cf, int32_t tag, const double n[3], const double uw[3], const real W[5],
                  const real gW[15], real Wg[5], real gWg[15])
{
    if (tag == TAG_SLIP) mirror_ghost(n, W, gW, Wg, gWg);
    else if (tag == TAG_FARFIELD) farfield_ghost(cf, n, W, Wg, gWg);
    else if (tag == TAG_NOSLIP_ADIABATIC || tag == TAG_NOSLIP_ISOTHERMAL)
        noslip_ghost(cf, tag == TAG_NOSLIP_ISOTHERMAL, uw, W, gW, Wg, gWg);
    else return -1;
    return 0;
}

static int face_terms(or_ctx *c, const real *coef, double dt, real *out, int raw)
{
    int64_t n = c->nc, nf = c->nf;
    int err = 0;
#pragma omp parallel for schedule(static) reduction(| : err)
    for (int64_t f = 0; f < nf; ++f) {
        int64_t L = c->fcell[f][0], R = c->fcell[f][1];
        real acc[20], gacc[30];
        for (int k = 0; k < 20; ++k) acc[k] = 0.0;
        for (int k = 0; k < 30; ++k) gacc[k] = 0.0;
        for (int q = 0; q < 3; ++q) {
            double rl[3], rr[3];
            for (int d = 0; d < 3; ++d) {
                rl[d] = c->fgp[f][q][d] - c->cen[L][d];
                rr[d] = c->fgp[f][q][d] - c->fshift[f][d] - (R >= 0 ? c->cen[R][d] : 0.0);
            }
            real Wl[5], gWl[15], Wr[5], gWr[15];
            for (int k = 0; k < 5; ++k) {
                qpoly_t p;
                quad_from_coef(coef, n, L, k, &p);
                Wl[k] = quad_eval(&p, rl);
                quad_grad(&p, rl, gWl + 3 * k);
                if (R >= 0) {
                    quad_from_coef(coef, n, R, k, &p);
                    Wr[k] = quad_eval(&p, rr);
                    quad_grad(&p, rr, gWr + 3 * k);
                }
            }
            const double *nq = c->fpn[f][q];
            if (R < 0)
                or_wall_ghost(&c->cfg, c->ftag[f], nq, c->fwu[f], Wl, gWl, Wr, gWr);
            real o[20];
            if (gks_point(&c->cfg, nq, Wl, gWl, Wr, gWr, dt, o)) { err |= 1; continue; }
            /* eq. linear-system: F = (4 F(dt/2) - F(dt)) / dt,
             * dF/dt = 4 (F(dt) - 2 F(dt/2)) / dt^2 */
            real w = c->fpw[f][q];
            for (int k = 0; k < 5; ++k) {
                if (raw) { /* the time integrals themselves */
                    acc[k] += w * o[k];
                    acc[5 + k] += w * o[5 + k];
                } else {
                    acc[k] += w * (4.0 * o[5 + k] - o[k]) / dt;
                    acc[5 + k] += w * 4.0 * (o[k] - 2.0 * o[5 + k]) / (dt * dt);
                }
                acc[10 + k] += w * o[10 + k];
                acc[15 + k] += w * o[15 + k];
                /* eq. gauss-formula: the point's share of the surface integral
                 * of W n, at t = 0 and t = dt */
                for (int d = 0; d < 3; ++d) {
                    gacc[3 * k + d] += w * o[10 + k] * nq[d];
                    gacc[15 + 3 * k + d] += w * o[15 + k] * nq[d];
                }
            }
        }
        for (int k = 0; k < 20; ++k) out[(size_t)k * nf + f] = acc[k];
        for (int k = 0; k < 30; ++k) c->fgrad[(size_t)k * nf + f] = gacc[k];
    }
    return err ? -1 : 0;
}

int or_face_terms(or_ctx *c, const real *W, const real *gW, double dt, real *out)
{
    or_reconstruct(c, W, gW, c->coef, c->flag, NULL);
    return face_terms(c, c->coef, dt, out, 0);
}

int or_face_integrals(or_ctx *c, const real *W, const real *gW, double dt, real *out)
{
    or_reconstruct(c, W, gW, c->coef, c->flag, NULL);
    return face_terms(c, c->coef, dt, out, 1);
}

/* eq. flux-operator for every cell, gathered in serial face order:
 * L = -(1/|Omega|) sum (+-) |Gamma| sum_k w_k F_k, same for dL/dt, and the
 * Gauss-theorem gradient (eq. gauss-formula) from the faces' surface
 * integrals of W n, Gf[15][nf] (component q, direction d at 3q+d) */
static void gather(const or_ctx *c, const real *ft, const real *Gf, real *L, real *Lt,
                   real *grad)
{
    int64_t n = c->nc, nf = c->nf;
    if (L) memset(L, 0, sizeof(real) * 5 * n);
    if (Lt) memset(Lt, 0, sizeof(real) * 5 * n);
    if (grad) memset(grad, 0, sizeof(real) * 15 * n);
    for (int64_t f = 0; f < nf; ++f) {
        int64_t side[2] = {c->fcell[f][0], c->fcell[f][1]};
        for (int s = 0; s < 2; ++s) {
            int64_t i = side[s];
            if (i < 0) continue;
            real sg = s == 0 ? 1.0 : -1.0;
            for (int q = 0; q < 5; ++q) {
                if (L) L[q * n + i] -= sg * ft[(size_t)q * nf + f];
                if (Lt) Lt[q * n + i] -= sg * ft[(size_t)(5 + q) * nf + f];
                if (grad)
                    for (int d = 0; d < 3; ++d)
                        grad[(3 * q + d) * n + i] += sg * Gf[(size_t)(3 * q + d) * nf + f];
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        real iv = 1.0 / c->vol[i];
        for (int q = 0; q < 5; ++q) {
            if (L) L[q * n + i] *= iv;
            if (Lt) Lt[q * n + i] *= iv;
        }
        for (int k = 0; k < 15 && grad; ++k) grad[k * n + i] *= iv;
    }
}

int or_stage(or_ctx *c, int stage, double dt, real *W, real *gW)
{
    int64_t n = c->nc, nf = c->nf;
    if (stage != 1 && stage != 2) return -1;
    if (stage == 2 && !c->have_stage1) return -1;
    or_reconstruct(c, W, gW, c->coef, c->flag, NULL);
    if (face_terms(c, c->coef, dt, c->fterm, 0)) return -2;
    real *Gf = (real *)malloc(sizeof(real) * 15 * nf);
    real *L = (real *)malloc(sizeof(real) * 5 * n);
    real *Lt = (real *)malloc(sizeof(real) * 5 * n);
    if (stage == 1) {
        /* eq. step-du with a linear-in-time f: f* = (f(0) + f(dt)) / 2; on a
         * flat face sum_k w_k W_k n_k = (sum_k w_k W_k) n */
        for (int64_t f = 0; f < nf; ++f) {
            if (c->fflat[f]) {
                for (int q = 0; q < 5; ++q) {
                    real w0 = c->fterm[(size_t)(10 + q) * nf + f];
                    real w1 = c->fterm[(size_t)(15 + q) * nf + f];
                    real wf = 0.5 * (w0 + w1);
                    c->FG0[(size_t)q * nf + f] = w0;
                    for (int d = 0; d < 3; ++d) Gf[(size_t)(3 * q + d) * nf + f] = wf * c->fpn[f][0][d];
                }
                continue;
            }
            for (int k = 0; k < 15; ++k) {
                real g0 = c->fgrad[(size_t)k * nf + f];
                real g1 = c->fgrad[(size_t)(15 + k) * nf + f];
                c->FG0[(size_t)k * nf + f] = g0;
                Gf[(size_t)k * nf + f] = 0.5 * (g0 + g1);
            }
        }
        gather(c, c->fterm, Gf, L, Lt, gW);
        /* eq. s2o4, first stage */
        for (int64_t k = 0; k < 5 * n; ++k) {
            c->Wn[k] = W[k];
            c->Ln[k] = L[k];
            c->Ltn[k] = Lt[k];
            W[k] = W[k] + 0.5 * dt * L[k] + 0.125 * dt * dt * Lt[k];
        }
        c->have_stage1 = 1;
    } else {
        /* f^{n+1} = f^n + dt f_t*, f_t* = (f*(dt) - f*(0)) / dt */
        for (int64_t f = 0; f < nf; ++f) {
            if (c->fflat[f]) {
                for (int q = 0; q < 5; ++q) {
                    real wf = c->FG0[(size_t)q * nf + f] + c->fterm[(size_t)(15 + q) * nf + f] -
                              c->fterm[(size_t)(10 + q) * nf + f];
                    for (int d = 0; d < 3; ++d) Gf[(size_t)(3 * q + d) * nf + f] = wf * c->fpn[f][0][d];
                }
                continue;
            }
            for (int k = 0; k < 15; ++k)
                Gf[(size_t)k * nf + f] = c->FG0[(size_t)k * nf + f] + c->fgrad[(size_t)(15 + k) * nf + f] -
                                         c->fgrad[(size_t)k * nf + f];
        }
        gather(c, c->fterm, Gf, L, Lt, gW);
        /* eq. s2o4, second stage: only dL/dt(W*) enters */
        for (int64_t k = 0; k < 5 * n; ++k)
            W[k] = c->Wn[k] + dt * c->Ln[k] + dt * dt / 6.0 * (c->Ltn[k] + 2.0 * Lt[k]);
        c->have_stage1 = 0;
    }
    free(Gf); free(L); free(Lt);
    return 0;
}

int or_last_face_terms(const or_ctx *c, real *out)
{
    memcpy(out, c->fterm, sizeof(real) * 20 * (size_t)c->nf);
    return 0;
}

int or_step(or_ctx *c, double dt, real *W, real *gW)
{
    int rc = or_stage(c, 1, dt, W, gW);
    if (rc) return rc;
    return or_stage(c, 2, dt, W, gW);
}

/* eq. time-step */
double or_compute_dt(const or_ctx *c, const real *W, double cfl)
{
    int64_t n = c->nc;
    const or_config *cf = &c->cfg;
    real best = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        real rho = W[i], u = W[n + i] / rho, v = W[2 * n + i] / rho, w = W[3 * n + i] / rho;
        real p = (cf->gamma - 1.0) * (W[4 * n + i] - 0.5 * rho * (u * u + v * v + w * w));
        real a = sqrt(cf->gamma * p / rho);
        real s = c->dr[i] / (sqrt(u * u + v * v + w * w) + a);
        if (s < best) best = s;
        if (cf->viscous && cf->mu > 0.0) {
            real nu = cf->mu / rho;
            real sv = c->dr[i] * c->dr[i] / (3.0 * nu);
            if (sv < best) best = sv;
        }
    }
    return cfl * OR_VALUE(best);
}

void or_conservation_sums(const or_ctx *c, const real *W, real out[5])
{
    int64_t n = c->nc;
    for (int q = 0; q < 5; ++q) {
        real s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += c->vol[i] * W[q * n + i];
        out[q] = s;
    }
}

#ifdef OR_TANGENT
/* tangent build only: the kink distance eps, and the counts per site and
 * direction since the last reset (out[2][OR_NDIR]) */
extern "C" int or_tangent_ndir(void) { return OR_NDIR; }
extern "C" void or_tangent_set_kink_eps(double eps) { or_kink_eps = eps; }
extern "C" void or_tangent_kinks(long *out, int reset)
{
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < OR_NDIR; ++k) {
            out[s * OR_NDIR + k] = or_kinks[s][k];
            if (reset) or_kinks[s][k] = 0;
        }
}
#endif
