/*
 * gks.h -- C interface of libgks, the MI355X (gfx950) implementation of the
 * third-order compact gas-kinetic scheme (GKS) on tetrahedral meshes of
 * Ji, Zhao, Shyy & Xu ("Two-step multi-resolution reconstruction-based
 * compact gas-kinetic scheme on tetrahedral mesh").
 *
 * One time step is the two-stage fourth-order method of Sec. 3 (eq. s2o4).
 * Each stage runs, on one HIP stream:
 *   A1  per cell: P^1 slopes by least squares on neighbour averages (Sec. 4.3,
 *       reconstruction step 1);
 *   A2  per cell: P^2 by constrained least squares (Sec. 4.1), multi-resolution
 *       WENO with the two-step P^0 indicator (Secs. 4.2-4.3, eqs.
 *       smooth-indicator, non-linear-weight, p0-non-linear-weight), and the
 *       positivity fallback to P^0;
 *   B   per face: the time-dependent BGK distribution at three Gauss points
 *       (Sec. 2.2, eqs. 2nd-flux, new-equ-part), its time-integrated fluxes
 *       fitted linearly in time (eq. linear-system) and its interface states
 *       (eqs. point-interface, step-du);
 *   C   per cell: finite-volume update of the averages (eqs. flux-operator,
 *       s2o4) and Gauss-theorem update of the averaged gradients (eq.
 *       gauss-formula), gathering its four faces in a fixed order (no atomics).
 *
 * Conventions for every entry point:
 *   - Return 0 (GKS_OK) on success, a negative gks_status otherwise; no
 *     exception or abort crosses this interface.  gks_last_error() gives a
 *     message for the last failure on a context.
 *   - Cell fields are component-major doubles: W[5][n_cell] holds
 *     (rho, rho u, rho v, rho w, rho E); gW[15][n_cell] holds the
 *     cell-averaged gradient with component c, direction d at row 3c+d.
 *   - Cells and faces are always addressed in the caller's order; the
 *     library may renumber internally.
 *   - Pointers marked "device" must be device memory of the current HIP
 *     device (e.g. from torch.empty(..., device='cuda')); "host" pointers
 *     are ordinary host memory.  Device work runs on the stream set by
 *     gks_set_stream (default: the null stream).
 *   - A context is not thread-safe; use one per thread.
 */
#ifndef GKS_H
#define GKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gks_status;
#define GKS_OK 0
#define GKS_E_INVAL (-1)       /* bad argument or configuration */
#define GKS_E_MESH (-2)        /* mesh rejected (degenerate cell, open surface, bad adjacency) */
#define GKS_E_NONPHYSICAL (-3) /* a cell average with rho <= 0 or p <= 0 */
#define GKS_E_ORDER (-4)       /* stage 2 without a preceding stage 1 */
#define GKS_E_DEVICE (-5)      /* a HIP call failed; sticky until gks_destroy */
#define GKS_E_STATE (-6)       /* call out of sequence (no mesh / workspace / state) */
#define GKS_E_NOMEM (-7)       /* workspace smaller than gks_workspace_bytes */

/* face tags */
#define GKS_FACE_INTERIOR 0
#define GKS_FACE_PERIODIC 1 /* neighbour lies across a periodic seam (face_shift != 0) */
#define GKS_FACE_SLIP 2     /* inviscid wall: mirror ghost state (Sec. 4.4) */
#define GKS_FACE_NOSLIP_ADIABATIC 3  /* no-slip wall at the face's wall velocity, no heat flux (Sec. 4.4) */
#define GKS_FACE_NOSLIP_ISOTHERMAL 4 /* no-slip wall at the wall velocity and temperature wall_T (Sec. 4.4) */
#define GKS_FACE_FARFIELD 5 /* far field: characteristic (Riemann-invariant) state against the free stream farfield */

/* distributions of the gas-kinetic flux */
#define GKS_FLUX_FULL 0   /* eq. 2nd-flux: equilibrium and kinetic parts, collision times tau, tau_n */
#define GKS_FLUX_SMOOTH 1 /* eq. 2nd-smooth-flux: the equilibrium part alone, g^c - tau (a^c.u + A^c) g^c
                             + t A^c g^c, with W^c and its slopes of eq. new-equ-part; for smooth flows */

/* precision forms */
#define GKS_FP64 0
#define GKS_FP32_BULK 1 /* reconstruction and flux arithmetic in FP32, state in FP64 */

typedef struct {
    double gamma;     /* ratio of specific heats, > 1 */
    double mu;        /* dynamic viscosity, >= 0 (used when viscous != 0) */
    double prandtl;   /* Prandtl number, > 0; 1 leaves the BGK heat flux unchanged */
    double eps_tau;   /* epsilon of the numerical collision time (paper: 0.01) */
    double c_tau;     /* C of the pressure-jump term (paper: 1) */
    double eps_weno;  /* epsilon of the nonlinear weights (paper: 1e-8) */
    double lw2[3];    /* linear weights gamma_{2,2} : gamma_{1,2} : gamma_{0,2} (ratios) */
    double lw1[2];    /* linear weights gamma_{1,1} : gamma_{0,1} (ratios) */
    int32_t viscous;  /* 0: Euler, tau = 0; 1: Navier-Stokes, tau = mu / p */
    int32_t nonlinear;/* 1: multi-resolution WENO weights; 0: linear (R = P^2) */
    int32_t precision;/* GKS_FP64 or GKS_FP32_BULK */
    int32_t order;    /* 3: third-order scheme (default); 2: second-order scheme, R from P^1 and
                         P^0 only (eq. final_weno_expression-2nd) */
    int32_t flux;     /* GKS_FLUX_FULL (default) or GKS_FLUX_SMOOTH */
    double wall_T;    /* temperature of isothermal no-slip walls as p / rho (> 0; default 1) */
    double farfield[5]; /* free stream of far-field faces, conservative (rho, rho u, rho v, rho w, rho E);
                           default (1, 0, 0, 0, 2.5) */
} gks_config;

/* Fill cfg with the paper's defaults: gamma 1.4, Euler, Pr 1, eps_tau 0.01,
 * C 1, eps_weno 1e-8, weights 100:10:1 and 10:1, nonlinear, FP64, third order,
 * full flux distribution, wall_T 1, far-field state (1, 0, 0, 0, 2.5). */
void gks_default_config(gks_config *cfg);

/* Tetrahedral mesh, host arrays.  face_vert lists the face's vertices as seen
 * from the owner face_cell[2f]; face_cell[2f+1] is the neighbour or -1 on a
 * wall.  face_shift[3f..3f+2] is the translation that carries the
 * neighbour's geometry into the owner's frame (periodic seams; else 0).
 * A boundary face is tagged GKS_FACE_SLIP, GKS_FACE_NOSLIP_ADIABATIC,
 * GKS_FACE_NOSLIP_ISOTHERMAL or GKS_FACE_FARFIELD; face_wall_u[3f..3f+2] is the velocity of a
 * no-slip wall face (global frame; NULL: every wall at rest).
 *
 * Quadratic elements (Sec. 2.1 six-node triangles, Sec. 4.1 ten-node
 * tetrahedra; curved walls and bent cells): tet_mid[(6i + e) * 3 + d] is the
 * control point on edge e of cell i, edges in the order (0,1), (1,2), (0,2),
 * (0,3), (1,3), (2,3) of tet[4i..4i+3].  A point within 1e-14 of the edge
 * length of the midpoint is taken as the midpoint (a straight edge).  A cell
 * with a bent edge takes |Omega|, centroid and moments from the five-point
 * rule on its map (eq. base-int-change); a face with a bent edge takes the
 * owner's control points, and each of its Gauss points its own normal and
 * weight (eq. flux-para-coord-gauss).  GKS_E_MESH if det J <= 0 at a
 * quadrature point or the two cells of a face disagree on its control
 * points (after the periodic shift).  The adjoint covers them (the quadratic
 * faces' points with their own normals and weights).  NULL: straight-sided
 * tetrahedra. */
typedef struct {
    int64_t n_vert;
    const double *xyz;        /* [n_vert][3] */
    int64_t n_cell;
    const int64_t *tet;       /* [n_cell][4] */
    int64_t n_face;
    const int64_t *face_vert; /* [n_face][3] */
    const int64_t *face_cell; /* [n_face][2] */
    const int32_t *face_tag;  /* [n_face] */
    const double *face_shift; /* [n_face][3] */
    const double *face_wall_u;/* [n_face][3] or NULL */
    const double *tet_mid;    /* [n_cell][6][3] or NULL: quadratic elements (below) */
} gks_mesh;

typedef struct gks_ctx gks_ctx;

/* Create a context; cfg is copied.  GKS_E_INVAL on gamma <= 1, mu < 0,
 * prandtl <= 0, non-positive weights or unknown enums. */
gks_status gks_create(const gks_config *cfg, gks_ctx **out);
/* Release everything the context owns (not the caller's workspace). */
void gks_destroy(gks_ctx *ctx);
/* All later device work is enqueued on this HIP stream (hipStream_t). */
gks_status gks_set_stream(gks_ctx *ctx, void *stream);

/* Geometry and the per-cell least-squares operators are formed in FP64 on
 * the host (Sec. 2.1 face rule, Sec. 4.1 constrained least squares, Sec. 4.3
 * step-1 least squares, Sec. 5 inscribed radius).  The arrays are copied;
 * the caller may free them on return.  GKS_E_MESH on a malformed mesh. */
gks_status gks_mesh_upload(gks_ctx *ctx, const gks_mesh *mesh);
/* Device bytes the library needs for this mesh (after gks_mesh_upload). */
gks_status gks_workspace_bytes(const gks_ctx *ctx, size_t *bytes);
/* Give the library a device buffer of at least gks_workspace_bytes bytes
 * (256-byte aligned; the caller keeps it alive until gks_destroy).  Copies
 * the mesh data into it and blocks until the copy is complete. */
gks_status gks_bind_workspace(gks_ctx *ctx, void *device_ptr, size_t bytes);

/* Set the state W[5][n], gW[15][n] (host pointers if on_device == 0, device
 * pointers otherwise).  GKS_E_NONPHYSICAL if a cell has rho <= 0 or p <= 0. */
gks_status gks_init(gks_ctx *ctx, const double *W, const double *gW, int32_t on_device);
/* eq. time-step: dt = cfl * min_i min(dr_i / (|U_i| + a_i), dr_i^2 / (3 nu_i)).
 * Blocking (one 8-byte device-to-host copy). */
gks_status gks_compute_dt(gks_ctx *ctx, double cfl, double *dt);
/* One stage (1 or 2) of eq. s2o4 with step dt (asynchronous).  Stage 2 must
 * follow stage 1 with the same dt; GKS_E_ORDER otherwise. */
gks_status gks_stage(gks_ctx *ctx, int32_t stage, double dt);
/* Stage 1 followed by stage 2. */
gks_status gks_step(gks_ctx *ctx, double dt);
/* One whole step whose time step never leaves the device (asynchronous, no
 * host synchronisation): dt = cfl * the bound of gks_compute_dt on the
 * current state, then stage 1 and stage 2 with that dt.  Same arithmetic as
 * gks_compute_dt followed by gks_step.  GKS_E_INVAL for a cfl that is not
 * positive and finite, GKS_E_ORDER while a stage 1 is pending.  A
 * non-physical state surfaces at the next blocking call. */
gks_status gks_step_cfl(gks_ctx *ctx, double cfl);
/* The time step of the last gks_step_cfl or gks_compute_dt (blocking). */
gks_status gks_last_dt(gks_ctx *ctx, double *dt);
/* Discrete adjoint (hand-written reverse of the forward kernels; not part of
 * the paper, which has no adjoint).
 *
 * gks_adjoint_workspace_bytes / gks_bind_adjoint_workspace: a second device
 * buffer (256-byte aligned, caller-owned, kept alive until gks_destroy) for
 * the adjoint's recomputed forward quantities and adjoint arrays, about 5 KB
 * per cell in FP64.  Bind after gks_bind_workspace.
 *
 * gks_step_adjoint: the transpose of the Jacobian of one step of eq. s2o4
 * with the time step dt held fixed (dt is not differentiated).  Given the
 * state before the step (W_n[5][n], gW_n[15][n]) and the adjoints of the
 * state after it (Wbar_np1, gWbar_np1), writes the adjoints of the state
 * before it (Wbar_n, gWbar_n).  All six are DEVICE pointers in the caller's
 * cell order, component-major as in gks_init; the outputs may alias the
 * inputs.  Stage 1 and stage 2's reconstruction are recomputed from W_n; the
 * reconstruction is differentiated as implemented (the WENO weights with
 * d|x|/dx = sign(x), sign(0) = 0, and x^(4/3) -> (4/3) x^(1/3); the
 * positivity fallback as taken).  Asynchronous on the context's stream; it
 * leaves the context's own state untouched.  GKS_E_STATE without an adjoint
 * workspace, GKS_E_INVAL on a null pointer or a dt that is not positive and
 * finite.  Every boundary kind is differentiated: the slip mirror, the
 * no-slip walls (the constrained wall fits, through the density they take
 * their wall values from, and the reflected ghost state) and the far-field
 * state (its branch as taken, the free stream held constant). */
gks_status gks_adjoint_workspace_bytes(const gks_ctx *ctx, size_t *bytes);
gks_status gks_bind_adjoint_workspace(gks_ctx *ctx, void *device_ptr, size_t bytes);
gks_status gks_step_adjoint(gks_ctx *ctx, double dt, const double *W_n, const double *gW_n,
                            const double *Wbar_np1, const double *gWbar_np1, double *Wbar_n,
                            double *gWbar_n);

/* Copy the state out (blocking when on_device == 0).  Reports a pending
 * non-physical flag as GKS_E_NONPHYSICAL. */
gks_status gks_read_state(gks_ctx *ctx, double *W, double *gW, int32_t on_device);
/* sum_i |Omega_i| W_i for the five components, fixed-order FP64 reduction
 * (blocking). */
gks_status gks_conservation_sums(gks_ctx *ctx, double out[5]);

/* For callers that cannot allocate device memory or synchronise with the
 * host (code under HIP graph capture, tight serving loops): the sums of
 * gks_conservation_sums written to out_device[5], a DEVICE pointer, on the
 * context's stream without a host synchronisation and without any
 * allocation.  The per-block partial sums live in a fixed device array of the
 * library (2.5 MiB per device, kept until the process ends), which limits the
 * mesh to 16,777,216 cells (GKS_E_INVAL beyond, with the limit in
 * gks_last_error).  Every call on a device shares that array: calls that
 * overlap on one GPU (several streams or threads) race.  Same sums as
 * gks_conservation_sums up to rounding order (a fixed order per mesh, so
 * bitwise reproducible).  The non-physical flag is not read here. */
gks_status gks_conservation_sums_noalloc(gks_ctx *ctx, double *out_device);

/* Intermediate results of the current state, for parity checks, in the
 * caller's order (host or device pointers as on_device says):
 *   slopes[15][n]  reconstruction step 1 (component c, direction d at 3c+d);
 *   coef[50][n]    final polynomial per component about the cell centroid,
 *                  (c0, Gx, Gy, Gz, Hxx, Hyy, Hzz, Hxy, Hxz, Hyz), i.e.
 *                  R(r) = c0 + G.r + r^T H r / 2;
 *   flag[n]        1 where the positivity fallback replaced R by P^0.
 * Any output pointer may be NULL.  Blocking. */
gks_status gks_debug_reconstruct(gks_ctx *ctx, double *slopes, double *coef, int32_t *flag,
                                 int32_t on_device);
/* Face terms of the current state for step dt, out[20][n_face] =
 * |Gamma| sum_k w_k of (F_k (5), dF_k/dt (5), W_k(0) (5), W_k(dt) (5)) in the
 * global frame, normal outward from the owner.  Blocking. */
gks_status gks_debug_face_terms(gks_ctx *ctx, double dt, double *out, int32_t on_device);
/* The same launch with the flux rows before the linear-in-time fit of eq.
 * linear-system: out[20][n_face] = |Gamma| sum_k w_k of (F_k(dt) (5),
 * F_k(dt/2) (5), W_k(0) (5), W_k(dt) (5)), F_k(delta) the time integral over
 * [0, delta] of the flux of eq. 2nd-flux (Sec. 2.2).  Comparing these
 * un-cancelled integrals bounds the fitted dF/dt = 4 (F(dt) - 2 F(dt/2)) /
 * dt^2, a difference of nearly equal terms.  Blocking. */
gks_status gks_debug_flux_integrals(gks_ctx *ctx, double dt, double *out, int32_t on_device);

/* Per-kernel timing for measurement: while enabled, every kernel launch of
 * the context is bracketed by HIP events on its stream.  gks_timing_read
 * blocks, then returns the accumulated milliseconds and launch counts per
 * kernel id (GKS_K_*; arrays of GKS_NKERNELS) and optionally resets them. */
#define GKS_K_SLOPES 0     /* A1 */
#define GKS_K_RECON 1      /* A2 */
#define GKS_K_FLUX1 2      /* B, stage 1 */
#define GKS_K_FLUX2 3      /* B, stage 2 */
#define GKS_K_UPDATE1 4    /* C, stage 1 */
#define GKS_K_UPDATE2 5    /* C, stage 2 */
#define GKS_K_DT 6         /* CFL reduction (both passes) */
#define GKS_NKERNELS 7
gks_status gks_timing_enable(gks_ctx *ctx, int32_t on);
gks_status gks_timing_read(gks_ctx *ctx, double ms[GKS_NKERNELS], int64_t counts[GKS_NKERNELS],
                           int32_t reset);

/* Algorithmic floating-point operations of the flux kernel for one face
 * under cfg: counts[0] adds/subtracts, [1] multiplies, [2] divides, [3]
 * special functions (exp, erfc, sqrt), obtained by running the kernel's face
 * routine on the host with a counting scalar.  Host only. */
gks_status gks_flux_op_count(const gks_config *cfg, double counts[4]);

/* Derivative checks of the flux routines, run on the host (no device work).
 * Each evaluates the flux with a forward-mode dual number (the exact
 * Jacobian-vector product J v) and its hand-written reverse (the
 * vector-Jacobian product J^T ybar) on the same inputs, for tests.
 *
 * gks_flux_point_check: the time-dependent distribution at one interface point
 * in the face frame (Sec. 2.2, eq. 2nd-flux).  x[40] = (W_l[5], dW_l/dx_d[3][5],
 * W_r[5], dW_r/dx_d[3][5]); y[20] = (F(dt)[5], F(dt/2)[5], W(0)[5], W(dt)[5]).
 * Outputs y, jv = J v, xbar = J^T ybar.
 *
 * gks_flux_face_check: the terms of one Gauss point of a face (eq.
 * linear-system), acc[20] = (F, dF/dt, W(0), W(dt)) x |Gamma|/3, as functions of
 * the two cells' coefficients coef[100] (owner [5][10], then neighbour [5][10],
 * as gks_debug_reconstruct orders them).  geo[10] = (unit normal[3], area,
 * Gauss point minus owner centroid[3], owner centroid minus neighbour
 * centroid[3]).  Outputs acc, jv = J v, coefbar = J^T accbar.
 * GKS_E_INVAL on a null pointer or dt <= 0. */
gks_status gks_flux_point_check(const gks_config *cfg, double dt, const double x[40], const double v[40],
                                const double ybar[20], double y[20], double jv[20], double xbar[40]);
gks_status gks_flux_face_check(const gks_config *cfg, double dt, const double geo[10], const double coef[100],
                               const double v[100], const double accbar[20], double acc[20], double jv[20],
                               double coefbar[100]);
/* The same check for the nonlinear combination of reconstruction step 2
 * (Secs. 4.2-4.3) of one cell and component: x[25] = (Q0, the fit
 * (g, H)[9], the cell's step-1 slopes[3], its four neighbours' slopes[4][3]);
 * geo[8] = (centroid second moments / |Omega| [6], |Omega|^(2/3),
 * |Omega|^(4/3)); bit a of has_mask set when neighbour a exists.  r[10] =
 * the coefficients (c0, G, H).  Outputs r, jv = J v, xbar = J^T rbar. */
gks_status gks_weno_check(const gks_config *cfg, const double geo[8], int32_t has_mask, const double x[25],
                          const double v[25], const double rbar[10], double r[10], double jv[10],
                          double xbar[25]);
/* The same check for the ghost state of a boundary point, in the face frame
 * (normal e1): tag GKS_FACE_NOSLIP_ADIABATIC or _ISOTHERMAL (Sec. 4.4; uw the
 * wall velocity, face frame) or GKS_FACE_FARFIELD (the free stream cfg->farfield,
 * taken as given in the face frame); x[20] = (interior W[5], its derivatives
 * along the three axes [3][5]); y[20] the ghost in the same layout.  Outputs
 * y, jv = J v, xbar = J^T ybar.  GKS_E_INVAL for another tag. */
gks_status gks_wall_ghost_check(const gks_config *cfg, int32_t tag, const double uw[3], const double x[20],
                                const double v[20], const double ybar[20], double y[20], double jv[20],
                                double xbar[20]);

/* Message of the last failure on this context (never NULL). */
const char *gks_last_error(const gks_ctx *ctx);
/* Name of a status code (never NULL). */
const char *gks_strerror(gks_status status);

#ifdef __cplusplus
}
#endif
#endif
