// Internal definitions shared by the host side of libgks (gks_api.cpp) and
// its HIP kernels (gks_kernels.hip, gks_flux_*.hip, gks_adjoint*.hip).  Not part of the public interface.
//
// Two precision forms share one layout: in FP64 every bulk array holds
// doubles; in FP32-bulk the per-stage bulk arrays (least-squares operators,
// reconstruction geometry, slopes, coefficients, face geometry and face
// terms) hold floats, while the state (W, grad W, stage-1 copies), the
// geometry the cell update, time step and conservation sums read, and the
// normals of the Gauss-theorem sums stay in FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gks {

// Scheme parameters as the kernels see them (linear weights normalised).
struct Params {
    double gamma, K, mu, prandtl, eps_tau, c_tau, eps_weno;
    double g22, g12, g02, g11, g01;
    int viscous, nonlinear;
    int order;  // 3 or 2
    int flux;   // FLUX_KIND_FULL or FLUX_KIND_SMOOTH
    double wall_T;  // p / rho of isothermal no-slip walls
    double farfield[5];  // free stream of far-field faces (conservative)
};

// distribution of the flux: eq. 2nd-flux, or its smooth-flow form eq. 2nd-smooth-flux
enum FluxKind { FLUX_KIND_FULL = 0, FLUX_KIND_SMOOTH = 1 };

// Rows of DevMesh::geoR ([NGEO_R][nc], bulk precision): what the
// reconstruction reads.
enum GeoRRow {
    G_VOL23 = 0,   // |Omega|^(2/3)
    G_VOL43 = 1,   // |Omega|^(4/3)
    G_C = 2,       // 6 rows: centroid second moments / |Omega| (xx,yy,zz,xy,xz,yz)
    G_RV = 8,      // 12 rows: vertex a, direction d at G_RV + 3a + d, relative to the centroid
    NGEO_R = 20
};

// Rows of DevMesh::geoD ([NGEO_D][nc], FP64).
enum GeoDRow {
    G_INVVOL = 0,  // 1 / |Omega|
    G_DR = 1,      // 3 |Omega| / sum |Gamma|
    G_VOL = 2,     // |Omega|
    NGEO_D = 3
};

// Rows of DevMesh::fgeo ([NFGEO][nf], bulk precision, internal face order).
enum FaceRow {
    F_N = 0,       // 3 rows: unit normal, outward from the owner
    F_AREA = 3,    // |Gamma|
    F_RL = 4,      // 9 rows: Gauss point k, direction d at F_RL + 3k + d, relative to the owner centroid
    F_D = 13,      // 3 rows: owner centroid - (neighbour centroid + shift)
    NFGEO = 16
};

// No-slip walls (Sec. 4.4).  A cell with at least one no-slip face (a wall
// cell) has two constraint sets: momentum, constrained at every no-slip face,
// and energy, constrained at the isothermal ones.  Per set, rows of
// DevMesh::wop ([kWallRows][nwc], bulk precision):
//   step 1: b_d = sum_a K1N[4d+a] (Q_a - Q_0) + sum_j K1C[3d+j] (c_j - Q_0)
//           over the face centres j (X1, relative to the centroid; U1 their
//           wall velocity);
//   step 2: (g, H)_r = sum_k K2N[16r+k] d_k + sum_g K2C[9r+g] (c_g - Q_0)
//           over the faces' Gauss points g (X2, U2), d as for M2;
// c = rho U_wall (momentum) or rho (|U_wall|^2/2 + T_wall/(gamma-1)) (energy)
// from the density reconstructed at the point.  Unused constraint columns are
// zero.  DevMesh::wmode ([4][nwc]): step 1 momentum, step 1 energy, step 2
// momentum, step 2 energy, each a WallMode.
enum WallRow {
    WR_K1N = 0,
    WR_K1C = 12,
    WR_X1 = 21,
    WR_U1 = 30,
    WR_K2N = 39,
    WR_K2C = 183,
    WR_X2 = 264,
    WR_U2 = 291,
    WR_SET = 318
};
// after the two sets: the cell's unconstrained step-2 operator (the 144 rows
// of M2), so that the wall kernel reads every operator coalesced
constexpr int WR_M2 = 2 * WR_SET;
constexpr int kWallRows = WR_M2 + 144;
enum WallMode {
    WM_KEEP = 0,  // no constraint: the unconstrained result stands
    WM_OWN = 1,   // step 1 with fewer than three neighbours and constraints: own averaged gradient
    WM_FIT = 2    // the operators above (a fallback is an operator without K1C / K2C)
};
enum WallTag { WALL_SLIP = 2, WALL_ADIABATIC = 3, WALL_ISOTHERMAL = 4, WALL_FARFIELD = 5 };

// Device view of the mesh (all pointers into the caller's workspace).
// Quadratic elements (Sec. 2.1, eq. flux-para-coord-gauss): faces [nfc, nf)
// carry per Gauss point k a unit normal (rows 4k..4k+2 of cgeo) and the area
// scale |X_xi x X_eta| / 2 (row 4k+3; the point's weight is a third of it);
// a bent cell's positivity check reads its faces' Gauss points (cpts row
// 9a + 3k + d: slot a, point k, direction d, relative to the centroid).
constexpr int kCurvedFaceRows = 12;
constexpr int kCurvedCellRows = 36;

struct DevMesh {
    int nc, nf;
    int nfi;            // faces [0, nfi) are interior, [nfi, nf) walls
    int nfc;            // faces [nfc, nf) take the quadratic path (nfc <= nfi, or nf without bent edges)
    const void *cgeo;   // [kCurvedFaceRows][nf - nfc]
    const double *cnrm; // [9][nf - nfc] the same normals in FP64 (row 3k + d), for the cell update
    const int *ccell;   // [nc] row of a bent cell in cpts, -1 for a straight one
    const void *cpts;   // [kCurvedCellRows][ncc]
    int ncc;
    const int *nbr;     // [4][nc] neighbour internal id, -1 on a wall
    const int *cface;   // [4][nc] 2 * face + side (side 1: the cell is the face's neighbour)
    const void *M1;     // [12][nc] slopes b_d = sum_m M1[4d+m] (Q_m - Q_0)
    const void *M2;     // tiled [ceil(nc/64)][144][64]: (g, H) = M2 . (Q_m - Q_0 (4);
                        // dQ_m/dx_d (12, index 4+3m+d)); entry (row, i) at m2_index(row, i)
    const void *geoR;   // [NGEO_R][nc]
    const double *geoD; // [NGEO_D][nc]
    const int *fcell;   // [2][nf] owner, neighbour (-1 on a wall)
    const void *fgeo;   // [NFGEO][nf]
    const double *fnrm; // [3][nf] unit normal in FP64 (the Gauss sums of the cell update); zero on
                        // the quadratic faces [nfc, nf), which use cnrm
    const int *bslot;   // [4][nc] slot of neighbour a whose face is the cell's slot a (-1 on a wall)
    const int *bmode;   // [nc] 1: fewer than three neighbours, step-1 slopes = own averaged gradient
    const int *wtag;    // [nf - nfi] WallTag of wall face nfi + k
    const void *wvel;   // [3][nf - nfi] wall velocity (global frame)
    int nwc;            // wall cells (cells with a no-slip face)
    const int *wcell;   // [nwc] their internal ids
    const int *widx;    // [nc] wall-cell index of a cell, -1 if it has no no-slip face
    const int *wmode;   // [4][nwc]
    const void *wop;    // [kWallRows][nwc]
};

// Device view of the state and per-stage scratch.
struct DevState {
    double *W, *gW;         // [5][nc], [15][nc] current state (stage input / output)
    double *Wn, *Ln, *Ltn;  // [5][nc] each: W^n and L, dL/dt of stage 1
    void *slopes;           // [15][nc]
    void *coef;             // [50][nc]
    int *flag;              // [nc] positivity fallback taken
    void *FF, *FT, *FW0, *FWs; // [5][nf] each: face flux, its time derivative,
                               // interface W(0) of stage 1, interface W for the gradient
    void *GC0, *GCs;           // [15][nf - nfc] each: the quadratic faces' weighted interface values
                               // per Gauss point, as FW0 and FWs (component q, point k at 3q+k)
    double *red;            // reduction scratch
    int *nonphys;           // [1] set when a cell average is non-physical
};

// FLUX_DEBUG writes all four face terms; FLUX_DEBUG_RAW the same with the
// un-fitted time integrals F(dt), F(dt/2) in place of F and dF/dt
enum FluxMode { FLUX_STAGE1 = 0, FLUX_STAGE2 = 1, FLUX_DEBUG = 2, FLUX_DEBUG_RAW = 3 };

// kernel launchers (gks_kernels.hip); fp32 selects the FP32-bulk form;
// each returns the hipError_t of the launch
hipError_t launch_slopes(const DevMesh &m, const DevState &s, bool fp32, hipStream_t st);
hipError_t launch_reconstruct(const DevMesh &m, const DevState &s, const Params &p, bool fp32,
                              hipStream_t st);
// flux and update take the time step from *dtp when dtp is not null (a time
// step that stays on the device), else from dt
hipError_t launch_flux(const DevMesh &m, const DevState &s, const Params &p, double dt,
                       const double *dtp, int mode, bool fp32, hipStream_t st);
hipError_t launch_update(const DevMesh &m, const DevState &s, double dt, const double *dtp,
                         int stage, bool fp32, hipStream_t st);
// the flux launcher of one bulk type (gks_flux_f64.hip, gks_flux_f32.hip)
template <typename R>
hipError_t launch_flux_t(const DevMesh &m, const DevState &s, const Params &p, double dt, const double *dtp,
                         int mode, hipStream_t st);
// no-slip wall cells: the constrained step-1 slopes (after launch_slopes) and
// the step-2 reconstruction of the wall cells (after launch_reconstruct)
hipError_t launch_wall_slopes(const DevMesh &m, const DevState &s, const Params &p, bool fp32, hipStream_t st);
hipError_t launch_wall_reconstruct(const DevMesh &m, const DevState &s, const Params &p, bool fp32,
                                   hipStream_t st);
// dt: writes the min over cells of the CFL bound (without the CFL factor) to
// s.red[0] and cfl times it, the time step, to s.red[kRedDt]
hipError_t launch_dt(const DevMesh &m, const DevState &s, const Params &p, double cfl,
                     hipStream_t st);
// conservation sums: writes sum_i |Omega_i| W_i to s.red[0..4]
hipError_t launch_sums(const DevMesh &m, const DevState &s, hipStream_t st);
// conservation sums without allocation (gks_noalloc.hip): per-block partials
// in a fixed device array, the five sums written to out (device); at most
// noalloc_max_cells() cells (hipErrorInvalidValue beyond)
int64_t noalloc_max_cells();
hipError_t launch_sums_noalloc(const DevMesh &m, const DevState &s, double *out, hipStream_t st);
// physical check of the state: sets *s.nonphys when rho <= 0 or p <= 0
hipError_t launch_check(const DevMesh &m, const DevState &s, const Params &p, hipStream_t st);
// dst[r][perm[i]] = src[r][i] (scatter to caller order) or dst[r][i] = src[r][perm[i]]
// (gather); src_f32 reads floats and widens them
hipError_t launch_permute_rows(double *dst, const void *src, const int *perm, int n, int rows,
                               int scatter, bool src_f32, hipStream_t st);
hipError_t launch_permute_int(int *dst, const int *src, const int *perm, int n, int scatter,
                              hipStream_t st);
// *p = v (a one-thread kernel, so that no memset node is needed)
hipError_t launch_fill_int(int *p, int v, hipStream_t st);

// cells per tile of the second-step operator M2: the 144 rows of the 64 cells
// of a tile are contiguous, so that one reconstruction block streams its
// operators as a single block of memory; the last tile is zero-padded
constexpr int kM2Tile = 64;
constexpr int kM2Rows = 144;
__host__ __device__ inline size_t m2_index(int row, int i)
{
    return ((size_t)(i / kM2Tile) * kM2Rows + row) * kM2Tile + (size_t)(i % kM2Tile);
}
inline size_t m2_padded_cells(size_t nc) { return (nc + kM2Tile - 1) / kM2Tile * kM2Tile; }

// ---------------------------------------------------------------------------
// Discrete adjoint of one step (gks_adjoint.hip).  Adjoint arrays are FP64 in
// internal order.

// Flux stage of the adjoint: the adjoint of the face terms of a stage is
// formed from the cells' adjoints (the transpose of the cell update), and the
// flux's vector-Jacobian product is written per face side as the adjoint of
// that side's cell coefficients.
struct AdjFlux {
    const void *coef;           // [50][nc] the stage's reconstruction (bulk type)
    const double *Wb1, *Gb1;    // adjoint of W^{n+1}, grad W^{n+1}
    const double *Wbs, *Gbs;    // adjoint of W*, grad W* (stage 1 only)
    double *CB;                 // [2][50][nf] out: coefficient adjoints of owner / neighbour
    double *EQ;                 // [kEqRec][3 nf] per Gauss point: the equilibrium part's adjoints
    double *SB;                 // [kSideRec][2 x 3 nf] per Gauss point and side: a kinetic side's adjoints
};

// Reconstruction stage of the adjoint: the stage's input state and step-1
// slopes, the coefficient adjoints per face side, and the per-cell results.
struct AdjRecon {
    const double *W, *G;        // the stage's input state
    const void *slopes;         // [15][nc] its step-1 slopes (bulk type)
    const int *flag;            // [nc] positivity fallback taken
    const double *CB;           // [2][50][nf]
    double *own_w, *own_s;      // [5][nc], [15][nc] adjoints of the cell's own W and slopes
    double *nb_w, *nb_g, *nb_s; // [4][5][nc], [4][15][nc], [4][15][nc] adjoints of
                                // neighbour a's W, grad W and slopes
    double *nb_w1;              // [4][5][nc] neighbour a's W through the step-1 slopes
    double *Wtmp;               // [5][nc]
    const int *bslot;           // [4][nc] slot of neighbour a that points back at the cell
};

enum FluxAdjMode { FLUX_ADJ_STAGE1 = 1, FLUX_ADJ_STAGE2 = 2 };
constexpr int kEqRec = 33;    // values of an AdjFlux::EQ record (per Gauss point)
constexpr int kSideRec = 35;  // values of an AdjFlux::SB record (per Gauss point and side)

// the flux stage's adjoint for one bulk type (gks_adjoint_flux_f64.hip, _f32.hip),
// and the dispatch on the bulk type (gks_adjoint.hip, which does not see the
// template's definition, so each type is compiled in its own unit only)
template <typename R>
hipError_t launch_flux_vjp_t(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, int mode,
                             hipStream_t st);
hipError_t launch_flux_vjp(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, int mode, bool fp32,
                           hipStream_t st);
// adjoints of the reconstruction's inputs: own / neighbour terms
hipError_t launch_recon_vjp(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32,
                            hipStream_t st);  // either order
// gathers the neighbour terms (fixed slot order) and applies the reverse of the
// step-1 slopes: Gout = adjoint of the stage's input gradient (complete); then
// Wout = adjoint of its input W + X1 + X2 (X1, X2 may be null)
hipError_t launch_recon_gather(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, double *Gout,
                               double *Wout, const double *X1, const double *X2, hipStream_t st);
// the step-2 reverse of the no-slip wall cells (after launch_recon_vjp, which
// it overwrites for them)
hipError_t launch_wall_recon_vjp(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, hipStream_t st);

// block size for the one-thread-per-item kernels
constexpr int kBlock = 256;
// number of blocks of the reduction kernels' first pass
constexpr int kRedBlocks = 1024;
// slot of s.red that holds the last time step (slots 0..4 take the sums)
constexpr int kRedDt = 6;

}  // namespace gks
