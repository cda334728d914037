/*
 * gks_oracle.h -- test infrastructure, not part of the product.
 *
 * A plain, slow FP64 CPU implementation of one time step of the third-order
 * compact gas-kinetic scheme on tetrahedral meshes (Ji, Zhao, Shyy & Xu,
 * "Two-step multi-resolution reconstruction-based compact gas-kinetic scheme
 * on tetrahedral mesh").  The HIP library is checked against it.  It shares
 * no code with that library.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * Array layouts match the library's public interface: cell fields are
 * component-major, W[5][n_cell] = (rho, rho u, rho v, rho w, rho E) and
 * gW[15][n_cell] with component c, direction d at row 3c+d.
 */
#ifndef GKS_ORACLE_H
#define GKS_ORACLE_H

#include <stdint.h>

/* arithmetic type of state arrays: double (the tangent build of the oracle
 * defines it as its dual type) */
#ifndef OR_REAL
#define OR_REAL double
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double gamma;     /* ratio of specific heats */
    double K;         /* internal degrees of freedom, (5 - 3 gamma) / (gamma - 1) */
    double mu;        /* dynamic viscosity (used when viscous != 0) */
    double prandtl;   /* Prandtl number; 1 leaves the BGK heat flux unchanged */
    double eps_tau;   /* epsilon of the numerical collision time (0.01) */
    double c_tau;     /* C of the pressure-jump term (1) */
    double eps_weno;  /* epsilon of the nonlinear weights (1e-8) */
    double lw2[3];    /* linear weights gamma_{2,2}, gamma_{1,2}, gamma_{0,2} (sum 1) */
    double lw1[2];    /* linear weights gamma_{1,1}, gamma_{0,1} (sum 1) */
    int32_t viscous;  /* 0: Euler (tau = 0); 1: Navier-Stokes (tau = mu / p) */
    int32_t nonlinear;/* 1: multi-resolution WENO weights; 0: R = P^2 (linear) */
    int32_t order;    /* 3: third-order (P^2, eq. final_weno_expression-3rd); 2: second-order
                         (P^1 and P^0 only, eq. final_weno_expression-2nd) */
    int32_t flux;     /* 0: the full distribution of eq. 2nd-flux; 1: its smooth-flow form,
                         eq. 2nd-smooth-flux */
    double wall_T;    /* temperature p / rho of isothermal no-slip walls */
    double farfield[5]; /* free-stream state (conservative) of far-field faces */
    int32_t weno_reading; /* 0: the readings the library follows.  Other bits select alternative
                             readings of Secs. 4.2-4.3, used only to compare against the paper's
                             Tables 2-3: OR_READ_* below */
} or_config;

/* alternative readings of the nonlinear weights (bits of or_config.weno_reading) */
#define OR_READ_POW1 1      /* power 1 instead of 2 in omega_{m,n} (eq. non-linear-weight) */
#define OR_READ_POW1ST2 2   /* power 2 instead of 1 in omega^{1st}_j (eq. p0-non-linear-weight) */
#define OR_READ_B0VOL 4     /* |Delta_0| in beta_{0,j} read as the volume |Omega_0| instead of |Omega_0|^(2/3) */
#define OR_READ_MIXED2 8    /* mixed second derivatives counted twice in beta_2 (eq. smooth-indicator) */
#define OR_READ_BETA_LOWER 16 /* beta_1, beta_2 of the hierarchical p_1, p_2 instead of P^1, P^2 */
#define OR_READ_SIGMA1 32   /* sigma without the power 4/3 */

typedef struct or_ctx or_ctx;

/* Build the oracle's mesh and geometry.  Wall faces (face_cell[2f+1] = -1)
 * carry tag 2 (slip), 3 (no-slip adiabatic), 4 (no-slip isothermal) or 5
 * (far field);
 * face_wall_u[3f..3f+2] is a no-slip face's wall velocity (NULL: walls at
 * rest).  Returns NULL on a malformed mesh. */
or_ctx *or_create(const or_config *cfg, int64_t n_vert, const double *xyz,
                  int64_t n_cell, const int64_t *tet, int64_t n_face,
                  const int64_t *face_vert, const int64_t *face_cell,
                  const int32_t *face_tag, const double *face_shift, const double *face_wall_u);
/* The same mesh with quadratic elements (Sec. 2.1 quadratic triangles,
 * Sec. 4.1 quadratic tetrahedra): tet_mid[(6 i + e) * 3 + d] is the control
 * point on edge e of cell i, edges in the order (0,1), (1,2), (0,2), (0,3),
 * (1,3), (2,3) of its tet[] vertices.  Volumes, centroids and moments come
 * from the five-point rule on the isoparametric map, faces from the
 * quadratic triangle through the owner's edge points, with a normal and a
 * weight per Gauss point. */
or_ctx *or_create_quadratic(const or_config *cfg, int64_t n_vert, const double *xyz,
                            int64_t n_cell, const int64_t *tet, int64_t n_face,
                            const int64_t *face_vert, const int64_t *face_cell,
                            const int32_t *face_tag, const double *face_shift, const double *face_wall_u,
                            const double *tet_mid);
void or_destroy(or_ctx *ctx);
int or_set_threads(int n);

/* Geometry: volume[n], centroid[3][n], second moment about the centroid
 * [6][n] (xx,yy,zz,xy,xz,yz, divided by the volume), inscribed radius dr[n]. */
int or_geometry(const or_ctx *ctx, double *vol, double *cen, double *mom2, double *dr);
/* Per-face area[nf], unit normal[3][nf] (outward from the owner),
 * Gauss points [3 points][3][nf].  On a quadratic face the area is the sum
 * of the point weights and the normal that of the triangle of its vertices. */
int or_face_geometry(const or_ctx *ctx, double *area, double *normal, double *gp);
/* Per Gauss point: unit normal [3 points][3][nf] and weight [3][nf] (omega_m
 * of eq. flux-para-coord-gauss, the face area included). */
int or_face_points(const or_ctx *ctx, double *normal, double *weight);

/* The ghost state of a wall point (tag 2, 3, 4 or 5; n the outward unit
 * normal, uw the wall velocity), global frame. */
int or_wall_ghost(const or_config *cfg, int32_t tag, const double n[3], const double uw[3], const OR_REAL W[5],
                  const OR_REAL gW[15], OR_REAL Wg[5], OR_REAL gWg[15]);

/* Reconstruction step 1: slopes b[15][n] (component c, direction d at 3c+d).
 * A cell with fewer than three neighbours (at walls) takes its own averaged
 * gradient gW (zero if gW is NULL); components constrained at no-slip faces
 * take the constrained fit. */
int or_slopes(or_ctx *ctx, const OR_REAL *W, const OR_REAL *gW, OR_REAL *b);
/* Reconstruction step 2: final polynomial R(x) = c0 + G.r + 1/2 r^T H r about
 * the centroid, coef[50][n] = per component (c0, Gx, Gy, Gz, Hxx, Hyy, Hzz,
 * Hxy, Hxz, Hyz); flag[n] = 1 where the positivity fallback fired.
 * p2coef (optional, same layout) receives the linear P^2 fit. */
int or_reconstruct(or_ctx *ctx, const OR_REAL *W, const OR_REAL *gW, OR_REAL *coef,
                   int32_t *flag, OR_REAL *p2coef);
/* Face terms for a state (W, gW) and step dt: out[20][nf] =
 * |Gamma| sum_k w_k of (F_k (5), dF_k/dt (5), W_k(0) (5), W_k(dt) (5)),
 * in the global frame, normal outward from the owner. */
int or_face_terms(or_ctx *ctx, const OR_REAL *W, const OR_REAL *gW, double dt, OR_REAL *out);
/* The same with the time integrals before the fit of eq. linear-system:
 * out[20][nf] = |Gamma| sum_k w_k of (F_k(dt), F_k(dt/2), W_k(0), W_k(dt)). */
int or_face_integrals(or_ctx *ctx, const OR_REAL *W, const OR_REAL *gW, double dt, OR_REAL *out);

/* One stage of the two-stage fourth-order step, in place on (W, gW).
 * Stage 1 expects W^n and leaves W*; stage 2 expects W* and leaves W^{n+1}. */
int or_stage(or_ctx *ctx, int stage, double dt, OR_REAL *W, OR_REAL *gW);
int or_step(or_ctx *ctx, double dt, OR_REAL *W, OR_REAL *gW);
/* The face terms (layout of or_face_terms) of the last or_stage call. */
int or_last_face_terms(const or_ctx *ctx, OR_REAL *out);
double or_compute_dt(const or_ctx *ctx, const OR_REAL *W, double cfl);
void or_conservation_sums(const or_ctx *ctx, const OR_REAL *W, OR_REAL out[5]);

/* Gas-kinetic solver at one interface point, global frame.  n: unit normal,
 * Wl/Wr: states, gWl/gWr[15] gradients (3c+d).  out[20] = F(dt), F(dt/2)
 * (time integrals of the flux density), W(0), W(dt). */
int or_point_flux(const or_config *cfg, const double n[3], const OR_REAL Wl[5],
                  const OR_REAL gWl[15], const OR_REAL Wr[5], const OR_REAL gWr[15],
                  double dt, OR_REAL out[20]);
/* Flux density F(t) (not integrated) at the same point, out[5]. */
int or_point_flux_density(const or_config *cfg, const double n[3], const OR_REAL Wl[5],
                          const OR_REAL gWl[15], const OR_REAL Wr[5], const OR_REAL gWr[15],
                          double dt, double t, OR_REAL out[5]);
/* Normalised velocity moments of the Maxwellian of W (local frame as given):
 * out[0..9] <u^k>, out[10..19] <u^k>_{u>0}, out[20..29] <u^k>_{u<0},
 * out[30..39] <v^k>, out[40..49] <w^k>, out[50..53] <xi^{2k}>. */
int or_maxwell_moments(const or_config *cfg, const OR_REAL W[5], OR_REAL out[54]);
/* Five-point volume rule and three-point face rule, as used (reference
 * elements): points[5][3] weights[5]; points[3][2] weights[3]. */
void or_volume_rule(double pts[15], double w[5]);
void or_face_rule(double pts[6], double w[3]);

#ifdef __cplusplus
}
#endif
#endif
