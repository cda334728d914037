// Host side of libgks: the C interface of include/gks.h.
//
// Mesh upload forms, in FP64 on the host, everything the kernels stream per
// stage: cell volumes, centroids and second moments (closed forms for a
// straight tetrahedron), the inscribed-sphere estimate (Sec. 5), face
// normals, areas and Gauss points (Sec. 2.1), and per cell the step-1
// least-squares operator (3x4, Sec. 4.3) and the step-2 constrained
// least-squares operator (9x16, Sec. 4.1).  The operators are formed with
// Householder QR (pseudo-inverse for step 1, null-space method for step 2),
// in coordinates centred at the cell centroid and scaled by |Omega|^(1/3).
// Cells are renumbered along a Morton curve of their centroids and faces are
// sorted by their lower internal cell, so that neighbouring threads touch
// neighbouring memory.
#include "../../include/gks.h"
#include "gks_internal.h"
#include "gks_params.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

using gks::DevMesh;
using gks::DevState;

struct gks_ctx {
    gks_config cfg{};
    gks::Params par{};
    hipStream_t stream = nullptr;
    std::string err;
    bool device_failed = false;
    // mesh, prepared on the host in device layout
    bool have_mesh = false;
    int nc = 0, nf = 0, nfi = 0;  // nfi: interior faces (internal ids below it)
    bool fp32 = false;              // FP32-bulk form
    std::vector<int> cperm, fperm;  // internal -> caller
    std::vector<int> nbr, cface, fcell, bslot, bmode;
    // no-slip walls: wall faces' tags and velocities (internal wall order),
    // wall cells, their modes and operators (host copies until bound)
    int nwc = 0;
    bool farfield = false;  // the mesh has far-field faces (no adjoint)
    std::vector<int> wtag, wcell, wmode;
    std::vector<double> wvel, wop;
    std::vector<double> M1, M2, geoR, geoD, fgeo, fnrm;
    // quadratic elements: faces [nfc, nf) with a normal and a weight per Gauss
    // point (cgeo), and the ncc bent cells' face Gauss points (cpts, ccell)
    bool curved = false;
    int nfc = 0, ncc = 0;
    std::vector<double> cgeo, cnrm, cpts;
    std::vector<int> ccell;
    // workspace
    bool bound = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    DevMesh dm{};
    DevState ds{};
    int *d_cperm = nullptr, *d_fperm = nullptr;
    // adjoint workspace (gks_bind_adjoint_workspace)
    bool adj_bound = false;
    struct Adj {
        double *Wchk, *Gchk, *Ws, *Gs, *Wn, *Ln, *Ltn, *Wb1, *Gb1, *Wbs, *Gbs, *Wbn, *Gbn;
        void *slopes1, *slopes2, *coef1, *coef2, *FF, *FT, *FW0, *FWs;
        int *flag1, *flag2, *nonphys;
        double *CB, *own_w, *own_s, *nb_w, *nb_g, *nb_s, *nb_w1, *Wtmp, *red, *EQ, *SB;
        void *GC0, *GCs;
    } adj{};
    double *staging = nullptr;
    int *istaging = nullptr;
    bool have_state = false;
    bool stage1_done = false;
    double stage1_dt = 0.0;
    // per-kernel event timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kernel;  // kernel id of each recorded (start, stop) pair
    double t_ms[GKS_NKERNELS] = {0};
    int64_t t_cnt[GKS_NKERNELS] = {0};
    ~gks_ctx()
    {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace {

gks_status fail(gks_ctx *c, gks_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

#define HIP_TRY(ctx, expr)                                                                  \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            (ctx)->device_failed = true;                                                    \
            return fail((ctx), GKS_E_DEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
        }                                                                                   \
    } while (0)

// ---------------------------------------------------------------------------
// small dense linear algebra (row-major)
// ---------------------------------------------------------------------------

// Householder QR of an m x n matrix (m >= n): A is overwritten by R in its
// upper triangle; Q (m x m) is returned explicitly.
void householder_qr(int m, int n, double *A, double *Q)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Q[i * m + j] = i == j ? 1.0 : 0.0;
    std::vector<double> v(m);
    for (int k = 0; k < n; ++k) {
        double nrm = 0.0;
        for (int i = k; i < m; ++i) nrm += A[i * n + k] * A[i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        const double alpha = A[k * n + k] > 0 ? -nrm : nrm;
        for (int i = 0; i < m; ++i) v[i] = 0.0;
        for (int i = k; i < m; ++i) v[i] = A[i * n + k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < m; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        // A <- (I - 2 v v^T / vv) A
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < m; ++i) s += v[i] * A[i * n + j];
            s *= 2.0 / vv;
            for (int i = k; i < m; ++i) A[i * n + j] -= s * v[i];
        }
        // Q <- Q (I - 2 v v^T / vv)
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = k; j < m; ++j) s += Q[i * m + j] * v[j];
            s *= 2.0 / vv;
            for (int j = k; j < m; ++j) Q[i * m + j] -= s * v[j];
        }
    }
}

// X = R^{-1} B for upper-triangular R (n x n, leading dimension ldr), B n x k
bool upper_solve(int n, const double *R, int ldr, double *B, int k)
{
    for (int i = n - 1; i >= 0; --i) {
        const double d = R[i * ldr + i];
        if (d == 0.0) return false;
        for (int j = 0; j < k; ++j) {
            double s = B[i * k + j];
            for (int l = i + 1; l < n; ++l) s -= R[i * ldr + l] * B[l * k + j];
            B[i * k + j] = s / d;
        }
    }
    return true;
}

// X = R^{-T} B for upper-triangular R (n x n), B n x k
bool lower_solve_transposed(int n, const double *R, int ldr, double *B, int k)
{
    for (int i = 0; i < n; ++i) {
        const double d = R[i * ldr + i];
        if (d == 0.0) return false;
        for (int j = 0; j < k; ++j) {
            double s = B[i * k + j];
            for (int l = 0; l < i; ++l) s -= R[l * ldr + i] * B[l * k + j];
            B[i * k + j] = s / d;
        }
    }
    return true;
}

// pseudo-inverse of a full-column-rank m x n matrix (n x m result)
bool pseudo_inverse(int m, int n, const double *A, double *Ap)
{
    std::vector<double> R(A, A + m * n), Q(m * m);
    householder_qr(m, n, R.data(), Q.data());
    // Ap = R^{-1} Q1^T
    std::vector<double> B(n * m);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) B[i * m + j] = Q[j * m + i];
    if (!upper_solve(n, R.data(), n, B.data(), m)) return false;
    std::copy(B.begin(), B.end(), Ap);
    return true;
}

// A X = I for a square n x n matrix (row-major, destroyed) by Gauss-Jordan
// elimination with partial pivoting; Ainv n x n.  False if a pivot vanishes.
bool invert(int n, double *A, double *Ainv)
{
    for (int r = 0; r < n; ++r)
        for (int t = 0; t < n; ++t) Ainv[r * n + t] = r == t ? 1.0 : 0.0;
    double scale = 0.0;
    for (int k = 0; k < n * n; ++k) scale = std::max(scale, std::fabs(A[k]));
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
        if (!(std::fabs(A[piv * n + col]) > 1e-13 * scale)) return false;
        if (piv != col)
            for (int t = 0; t < n; ++t) {
                std::swap(A[piv * n + t], A[col * n + t]);
                std::swap(Ainv[piv * n + t], Ainv[col * n + t]);
            }
        const double ip = 1.0 / A[col * n + col];
        for (int t = 0; t < n; ++t) {
            A[col * n + t] *= ip;
            Ainv[col * n + t] *= ip;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double fct = A[r * n + col];
            if (fct == 0.0) continue;
            for (int t = 0; t < n; ++t) {
                A[r * n + t] -= fct * A[col * n + t];
                Ainv[r * n + t] -= fct * Ainv[col * n + t];
            }
        }
    }
    return true;
}

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
inline void sub3(const double *a, const double *b, double *o)
{
    o[0] = a[0] - b[0];
    o[1] = a[1] - b[1];
    o[2] = a[2] - b[2];
}

inline void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

uint64_t spread_bits(uint64_t x)
{
    x &= 0x1fffff;
    x = (x | x << 32) & 0x1f00000000ffffULL;
    x = (x | x << 16) & 0x1f0000ff0000ffULL;
    x = (x | x << 8) & 0x100f00f00f00f00fULL;
    x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
    x = (x | x << 2) & 0x1249249249249249ULL;
    return x;
}

// ---------------------------------------------------------------------------
// quadratic elements (Sec. 2.1 six-node triangles, Sec. 4.1 ten-node
// tetrahedra) in barycentric form: a vertex node has the shape function
// l (2 l - 1), an edge node 4 l_a l_b
// ---------------------------------------------------------------------------

// the tetrahedron's edges in the order of gks_mesh::tet_mid
const int kTetEdge[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

int tet_edge_index(int a, int b)
{
    for (int e = 0; e < 6; ++e)
        if ((kTetEdge[e][0] == a && kTetEdge[e][1] == b) || (kTetEdge[e][0] == b && kTetEdge[e][1] == a)) return e;
    return -1;
}

// X(lambda) and det dX/d(xi, eta, zeta) of a ten-node tetrahedron, nodes
// x[0..3] the vertices and x[4 + e] the point on edge e; lambda_0 = 1 - xi -
// eta - zeta, lambda_k = (xi, eta, zeta)_k
double qtet_eval(const double x[10][3], const double lam[4], double X[3])
{
    // d lambda_k / d xi_j
    static const double dl[4][3] = {{-1, -1, -1}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    double J[3][3] = {};
    for (int d = 0; d < 3; ++d) X[d] = 0.0;
    for (int k = 0; k < 4; ++k) {
        const double N = lam[k] * (2.0 * lam[k] - 1.0), dN = 4.0 * lam[k] - 1.0;
        for (int d = 0; d < 3; ++d) {
            X[d] += N * x[k][d];
            for (int j = 0; j < 3; ++j) J[d][j] += dN * dl[k][j] * x[k][d];
        }
    }
    for (int e = 0; e < 6; ++e) {
        const int a = kTetEdge[e][0], b = kTetEdge[e][1];
        const double N = 4.0 * lam[a] * lam[b];
        for (int d = 0; d < 3; ++d) {
            X[d] += N * x[4 + e][d];
            for (int j = 0; j < 3; ++j) J[d][j] += 4.0 * (dl[a][j] * lam[b] + lam[a] * dl[b][j]) * x[4 + e][d];
        }
    }
    double c0[3];
    cross3(J[1], J[2], c0);  // rows: det = J0 . (J1 x J2)
    return dot3(J[0], c0);
}

// the five-point volume rule of Sec. 4.1 in barycentric form: the centre
// (weight -2/15; the weight that makes the rule exact for cubics), and the
// four points with one coordinate 1/2 and the others 1/6 (weight 3/40);
// weights include the reference volume 1/6
void volume_rule(double lam[5][4], double w[5])
{
    for (int k = 0; k < 4; ++k) lam[0][k] = 0.25;
    w[0] = -2.0 / 15.0;
    for (int q = 1; q < 5; ++q) {
        for (int k = 0; k < 4; ++k) lam[q][k] = k == q - 1 ? 0.5 : 1.0 / 6.0;
        w[q] = 3.0 / 40.0;
    }
}

// |Omega|, centroid and second central moments (xx, yy, zz, xy, xz, yz,
// divided by |Omega|) of a ten-node tetrahedron by the five-point rule on
// its map (eq. base-int-change); false unless det J has the sign of the
// straight element's at every point
bool qtet_moments(const double x[10][3], double &V, double cen[3], double C[6])
{
    double lam[5][4], w[5], X[5][3], wj[5], e1[3], e2[3], e3[3], cr[3];
    sub3(x[1], x[0], e1);
    sub3(x[2], x[0], e2);
    sub3(x[3], x[0], e3);
    cross3(e2, e3, cr);
    const double orient = dot3(e1, cr) > 0.0 ? 1.0 : -1.0;
    volume_rule(lam, w);
    V = 0.0;
    for (int q = 0; q < 5; ++q) {
        const double dj = orient * qtet_eval(x, lam[q], X[q]);
        if (!(dj > 0.0)) return false;
        wj[q] = w[q] * dj;
        V += wj[q];
    }
    if (!(V > 0.0)) return false;
    for (int d = 0; d < 3; ++d) {
        double t = 0.0;
        for (int q = 0; q < 5; ++q) t += wj[q] * X[q][d];
        cen[d] = t / V;
    }
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k) C[k] = 0.0;
    for (int q = 0; q < 5; ++q) {
        double r[3];
        sub3(X[q], cen, r);
        for (int k = 0; k < 6; ++k) C[k] += wj[q] * r[ia[k]] * r[ib[k]];
    }
    for (int k = 0; k < 6; ++k) C[k] /= V;
    return true;
}

// a six-node triangle at (xi, eta): X, and the unnormalised normal X_xi x
// X_eta; nodes t[0..2] the vertices, t[3], t[4], t[5] the points on the
// edges (0,1), (1,2), (0,2)
void qtri_eval(const double t[6][3], double xi, double eta, double X[3], double cr[3])
{
    const double mu[3] = {1.0 - xi - eta, xi, eta};
    static const double dm[3][2] = {{-1, -1}, {1, 0}, {0, 1}};
    static const int edge[3][2] = {{0, 1}, {1, 2}, {0, 2}};
    double Xa[3] = {0, 0, 0}, Xb[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) X[d] = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double N = mu[k] * (2.0 * mu[k] - 1.0), dN = 4.0 * mu[k] - 1.0;
        for (int d = 0; d < 3; ++d) {
            X[d] += N * t[k][d];
            Xa[d] += dN * dm[k][0] * t[k][d];
            Xb[d] += dN * dm[k][1] * t[k][d];
        }
    }
    for (int e = 0; e < 3; ++e) {
        const int a = edge[e][0], b = edge[e][1];
        const double N = 4.0 * mu[a] * mu[b];
        for (int d = 0; d < 3; ++d) {
            X[d] += N * t[3 + e][d];
            Xa[d] += 4.0 * (dm[a][0] * mu[b] + mu[a] * dm[b][0]) * t[3 + e][d];
            Xb[d] += 4.0 * (dm[a][1] * mu[b] + mu[a] * dm[b][1]) * t[3 + e][d];
        }
    }
    cross3(Xa, Xb, cr);
}

// quadratic basis of the step-2 fit, in scaled coordinates y about the
// centroid: y_x, y_y, y_z, y_x^2, y_y^2, y_z^2, y_x y_y, y_x y_z, y_y y_z
const int QA[6] = {0, 1, 2, 0, 0, 1};
const int QB[6] = {0, 1, 2, 1, 2, 2};

struct Layout {
    size_t off[48];
    size_t total;
};

enum Slot {
    S_NBR, S_CFACE, S_M1, S_M2, S_GEOR, S_GEOD, S_FCELL, S_FGEO, S_FNRM, S_W, S_GW, S_WN, S_LN, S_LTN,
    S_SLOPES, S_COEF, S_FLAG, S_FF, S_FT, S_FW0, S_FWS, S_RED, S_NONPHYS, S_CPERM, S_FPERM,
    S_STAGING, S_ISTAGING, S_BSLOT, S_BMODE, S_WTAG, S_WVEL, S_WCELL, S_WMODE, S_WOP, S_WIDX,
    S_CGEO, S_CCELL, S_CPTS, S_GC0, S_GCS, S_CNRM, S_COUNT
};

// bs: bytes of a bulk element (8 in FP64, 4 in FP32-bulk); nwf wall faces,
// nwc no-slip wall cells, ncf quadratic-path faces, ncc bent cells
Layout make_layout(size_t nc, size_t nf, size_t bs, size_t nwf, size_t nwc, size_t ncf, size_t ncc)
{
    const size_t sz[S_COUNT] = {
        4 * nc * sizeof(int), 4 * nc * sizeof(int), 12 * nc * bs,
        (size_t)gks::kM2Rows * gks::m2_padded_cells(nc) * bs,
        (size_t)gks::NGEO_R * nc * bs, (size_t)gks::NGEO_D * nc * 8, 2 * nf * sizeof(int),
        (size_t)gks::NFGEO * nf * bs, 3 * nf * 8,
        5 * nc * 8, 15 * nc * 8, 5 * nc * 8, 5 * nc * 8, 5 * nc * 8, 15 * nc * bs, 50 * nc * bs,
        nc * sizeof(int), 5 * nf * bs, 5 * nf * bs, 5 * nf * bs, 5 * nf * bs,
        (8 + 5 * (size_t)gks::kRedBlocks) * 8, 64, nc * sizeof(int), nf * sizeof(int),
        std::max(50 * nc, 20 * nf) * 8, nc * sizeof(int), 4 * nc * sizeof(int), nc * sizeof(int),
        nwf * sizeof(int), 3 * nwf * bs, nwc * sizeof(int), 4 * nwc * sizeof(int), (size_t)gks::kWallRows * nwc * bs,
        nc * sizeof(int), (size_t)gks::kCurvedFaceRows * ncf * bs, nc * sizeof(int),
        (size_t)gks::kCurvedCellRows * ncc * bs, 15 * ncf * bs, 15 * ncf * bs, 9 * ncf * 8};
    Layout L;
    size_t o = 0;
    for (int k = 0; k < S_COUNT; ++k) {
        L.off[k] = o;
        o += (sz[k] + 255) & ~size_t(255);
    }
    L.total = o;
    return L;
}

bool config_ok(const gks_config *c, std::string &why)
{
    if (!(c->gamma > 1.0)) { why = "gamma must be > 1"; return false; }
    if (!(c->mu >= 0.0)) { why = "mu must be >= 0"; return false; }
    if (!(c->prandtl > 0.0)) { why = "prandtl must be > 0"; return false; }
    if (!(c->eps_tau >= 0.0) || !(c->c_tau >= 0.0) || !(c->eps_weno > 0.0)) {
        why = "collision-time and WENO epsilons must be non-negative (eps_weno > 0)";
        return false;
    }
    for (int k = 0; k < 3; ++k)
        if (!(c->lw2[k] > 0.0)) { why = "linear weights must be positive"; return false; }
    for (int k = 0; k < 2; ++k)
        if (!(c->lw1[k] > 0.0)) { why = "linear weights must be positive"; return false; }
    if (c->viscous != 0 && c->viscous != 1) { why = "viscous must be 0 or 1"; return false; }
    if (c->nonlinear != 0 && c->nonlinear != 1) { why = "nonlinear must be 0 or 1"; return false; }
    if (c->precision != GKS_FP64 && c->precision != GKS_FP32_BULK) { why = "unknown precision"; return false; }
    if (c->order != 2 && c->order != 3) { why = "order must be 2 or 3"; return false; }
    if (c->flux != GKS_FLUX_FULL && c->flux != GKS_FLUX_SMOOTH) { why = "unknown flux"; return false; }
    if (!(c->wall_T > 0.0) || !std::isfinite(c->wall_T)) { why = "wall_T must be positive"; return false; }
    {
        const double *w = c->farfield;
        const double r = w[0], k = r > 0.0 ? 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / r : 0.0;
        if (!(r > 0.0) || !((c->gamma - 1.0) * (w[4] - k) > 0.0) || !std::isfinite(w[4])) {
            why = "the far-field state must have rho > 0 and p > 0";
            return false;
        }
    }
    return true;
}

}  // namespace

// Reconstruction steps 1 and 2 (Secs. 4.1-4.4): every cell, then the
// constrained fits of the no-slip wall cells.
static hipError_t slopes_step(const gks::DevMesh &m, const gks::DevState &s, const gks::Params &p, bool fp32,
                              hipStream_t st)
{
    hipError_t e = gks::launch_slopes(m, s, fp32, st);
    if (e == hipSuccess && m.nwc > 0) e = gks::launch_wall_slopes(m, s, p, fp32, st);
    return e;
}
static hipError_t reconstruct_step(const gks::DevMesh &m, const gks::DevState &s, const gks::Params &p, bool fp32,
                                   hipStream_t st)
{
    hipError_t e = gks::launch_reconstruct(m, s, p, fp32, st);
    if (e == hipSuccess && m.nwc > 0) e = gks::launch_wall_reconstruct(m, s, p, fp32, st);
    return e;
}

// Record an event on the context's stream when timing is on.
static gks_status mark(gks_ctx *c)
{
    if (!c->timing) return GKS_OK;
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        HIP_TRY(c, hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    HIP_TRY(c, hipEventRecord(c->ev_pool[c->ev_used++], c->stream));
    return GKS_OK;
}

// Launch one kernel group, bracketed by timing events when enabled.
template <typename F>
static gks_status timed(gks_ctx *c, int kernel, F &&launch)
{
    gks_status st = mark(c);
    if (st) return st;
    HIP_TRY(c, launch());
    if ((st = mark(c))) return st;
    if (c->timing) c->ev_kernel.push_back(kernel);
    return GKS_OK;
}

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

void gks_default_config(gks_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->gamma = 1.4;
    cfg->mu = 0.0;
    cfg->prandtl = 1.0;
    cfg->eps_tau = 0.01;
    cfg->c_tau = 1.0;
    cfg->eps_weno = 1e-8;
    cfg->lw2[0] = 100.0;
    cfg->lw2[1] = 10.0;
    cfg->lw2[2] = 1.0;
    cfg->lw1[0] = 10.0;
    cfg->lw1[1] = 1.0;
    cfg->viscous = 0;
    cfg->nonlinear = 1;
    cfg->precision = GKS_FP64;
    cfg->order = 3;
    cfg->flux = GKS_FLUX_FULL;
    cfg->wall_T = 1.0;
    cfg->farfield[0] = 1.0;
    cfg->farfield[4] = 2.5;
}

gks_status gks_create(const gks_config *cfg, gks_ctx **out)
{
    if (!cfg || !out) return GKS_E_INVAL;
    *out = nullptr;
    std::string why;
    if (!config_ok(cfg, why)) return GKS_E_INVAL;
    gks_ctx *c = new (std::nothrow) gks_ctx();
    if (!c) return GKS_E_NOMEM;
    c->cfg = *cfg;
    c->par = gks::params_from_config(cfg);
    c->fp32 = cfg->precision == GKS_FP32_BULK;
    *out = c;
    return GKS_OK;
}

void gks_destroy(gks_ctx *ctx) { delete ctx; }

gks_status gks_set_stream(gks_ctx *ctx, void *stream)
{
    if (!ctx) return GKS_E_INVAL;
    ctx->stream = (hipStream_t)stream;
    return GKS_OK;
}

gks_status gks_mesh_upload(gks_ctx *c, const gks_mesh *m)
{
    if (!c || !m) return GKS_E_INVAL;
    if (c->bound) return fail(c, GKS_E_STATE, "a workspace is already bound; create a new context");
    if (m->n_cell <= 0 || m->n_face <= 0 || m->n_vert <= 0 || !m->xyz || !m->tet || !m->face_vert ||
        !m->face_cell || !m->face_tag || !m->face_shift)
        return fail(c, GKS_E_INVAL, "empty mesh or missing array");
    if (m->n_cell > INT_MAX / 64 || m->n_face > INT_MAX / 64)
        return fail(c, GKS_E_INVAL, "mesh too large for 32-bit indexing");
    const int nc = (int)m->n_cell, nf = (int)m->n_face;
    c->wcell.clear();
    c->wmode.clear();
    c->wop.clear();

    // --- cells: vertices, volume, centroid -------------------------------
    std::vector<double> cen(3 * (size_t)nc), vol(nc);
    for (int i = 0; i < nc; ++i) {
        double v[4][3];
        for (int a = 0; a < 4; ++a) {
            const int64_t id = m->tet[4 * (size_t)i + a];
            if (id < 0 || id >= m->n_vert) return fail(c, GKS_E_MESH, "tet vertex id out of range");
            for (int d = 0; d < 3; ++d) v[a][d] = m->xyz[3 * id + d];
        }
        double e1[3], e2[3], e3[3], cr[3];
        sub3(v[1], v[0], e1);
        sub3(v[2], v[0], e2);
        sub3(v[3], v[0], e3);
        cross3(e2, e3, cr);
        const double V = std::fabs(dot3(e1, cr)) / 6.0;
        if (!(V > 0.0) || !std::isfinite(V)) return fail(c, GKS_E_MESH, "degenerate tetrahedron");
        vol[i] = V;
        for (int d = 0; d < 3; ++d) cen[3 * i + d] = 0.25 * (v[0][d] + v[1][d] + v[2][d] + v[3][d]);
    }

    // second central moments / |Omega| of the straight cells: (1/20) sum_a r_a r_a^T
    std::vector<double> cmom(6 * (size_t)nc);
    for (int i = 0; i < nc; ++i) {
        double C[6] = {0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 4; ++a) {
            const int64_t id = m->tet[4 * (size_t)i + a];
            double r[3];
            for (int d = 0; d < 3; ++d) r[d] = m->xyz[3 * id + d] - cen[3 * (size_t)i + d];
            for (int k = 0; k < 6; ++k) C[k] += r[QA[k]] * r[QB[k]];
        }
        for (int k = 0; k < 6; ++k) cmom[6 * (size_t)i + k] = C[k] / 20.0;
    }

    // --- quadratic elements (Secs. 2.1, 4.1): control points on the edges; a
    // point within 1e-14 of its edge length of the midpoint is the midpoint
    // (a straight edge); a cell with a bent edge takes its volume, centroid
    // and moments from the five-point rule on its map
    std::vector<double> cx;  // [nc][10][3]
    std::vector<char> ecurv(m->tet_mid ? 6 * (size_t)nc : 0, 0), ccurv(nc, 0);
    if (m->tet_mid) {
        cx.resize(30 * (size_t)nc);
        for (int i = 0; i < nc; ++i) {
            double(*x)[3] = reinterpret_cast<double(*)[3]>(&cx[30 * (size_t)i]);
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d) x[a][d] = m->xyz[3 * m->tet[4 * (size_t)i + a] + d];
            for (int e = 0; e < 6; ++e) {
                const int a = kTetEdge[e][0], b = kTetEdge[e][1];
                double mid[3], ed[3], dev = 0.0;
                sub3(x[b], x[a], ed);
                for (int d = 0; d < 3; ++d) {
                    const double t = m->tet_mid[(6 * (size_t)i + e) * 3 + d];
                    if (!std::isfinite(t)) return fail(c, GKS_E_MESH, "tet_mid is not finite");
                    mid[d] = 0.5 * (x[a][d] + x[b][d]);
                    dev = std::max(dev, std::fabs(t - mid[d]));
                    x[4 + e][d] = t;
                }
                if (dev <= 1e-14 * std::sqrt(dot3(ed, ed))) {
                    for (int d = 0; d < 3; ++d) x[4 + e][d] = mid[d];
                } else {
                    ecurv[6 * (size_t)i + e] = 1;
                    ccurv[i] = 1;
                }
            }
            if (ccurv[i] && !qtet_moments(x, vol[i], &cen[3 * (size_t)i], &cmom[6 * (size_t)i]))
                return fail(c, GKS_E_MESH, "a quadratic tetrahedron has det J <= 0 at a quadrature point");
        }
    }

    // --- faces: validation, incidence in caller face order ---------------
    std::vector<int> nslots(nc, 0), slot_face(4 * (size_t)nc, -1), slot_side(4 * (size_t)nc, 0);
    for (int f = 0; f < nf; ++f) {
        const int64_t L = m->face_cell[2 * (size_t)f], R = m->face_cell[2 * (size_t)f + 1];
        const int tag = m->face_tag[f];
        if (L < 0 || L >= nc || R >= nc || R == L) return fail(c, GKS_E_MESH, "bad face_cell entry");
        if (tag != GKS_FACE_INTERIOR && tag != GKS_FACE_PERIODIC && tag != GKS_FACE_SLIP &&
            tag != GKS_FACE_NOSLIP_ADIABATIC && tag != GKS_FACE_NOSLIP_ISOTHERMAL && tag != GKS_FACE_FARFIELD)
            return fail(c, GKS_E_MESH, "unknown face tag");
        const bool wall_tag = tag == GKS_FACE_SLIP || tag == GKS_FACE_NOSLIP_ADIABATIC ||
                              tag == GKS_FACE_NOSLIP_ISOTHERMAL || tag == GKS_FACE_FARFIELD;
        if ((R < 0) != wall_tag)
            return fail(c, GKS_E_MESH, "a wall face needs face_cell[2f+1] = -1 and a wall tag");
        if (m->face_wall_u)
            for (int d = 0; d < 3; ++d)
                if (!std::isfinite(m->face_wall_u[3 * (size_t)f + d]))
                    return fail(c, GKS_E_MESH, "face_wall_u is not finite");
        for (int s = 0; s < (R < 0 ? 1 : 2); ++s) {
            const int cell = (int)(s == 0 ? L : R);
            if (nslots[cell] >= 4) return fail(c, GKS_E_MESH, "a cell has more than four faces");
            slot_face[4 * (size_t)cell + nslots[cell]] = f;
            slot_side[4 * (size_t)cell + nslots[cell]] = s;
            ++nslots[cell];
        }
    }
    for (int i = 0; i < nc; ++i)
        if (nslots[i] != 4) return fail(c, GKS_E_MESH, "a cell does not have four faces");

    // a face is quadratic if one of its edges is bent in its owner; the
    // control points of its edges are the owner's and must be the
    // neighbour's (translated by the periodic shift)
    std::vector<char> fcurv(nf, 0);
    std::vector<double> fctrl(m->tet_mid ? 18 * (size_t)nf : 0);  // [nf][6][3] face control points
    if (m->tet_mid) {
        for (int f = 0; f < nf; ++f) {
            const int L = (int)m->face_cell[2 * (size_t)f], R = (int)m->face_cell[2 * (size_t)f + 1];
            int loc[3];
            for (int a = 0; a < 3; ++a) {
                loc[a] = -1;
                for (int k = 0; k < 4; ++k)
                    if (m->tet[4 * (size_t)L + k] == m->face_vert[3 * (size_t)f + a]) loc[a] = k;
                if (loc[a] < 0) return fail(c, GKS_E_MESH, "a face vertex is not a vertex of its owner");
            }
            double *t = &fctrl[18 * (size_t)f];
            for (int a = 0; a < 3; ++a)
                for (int d = 0; d < 3; ++d) t[3 * a + d] = cx[30 * (size_t)L + 3 * loc[a] + d];
            static const int fe[3][2] = {{0, 1}, {1, 2}, {0, 2}};
            for (int e = 0; e < 3; ++e) {
                const int te = tet_edge_index(loc[fe[e][0]], loc[fe[e][1]]);
                fcurv[f] |= ecurv[6 * (size_t)L + te];
                for (int d = 0; d < 3; ++d) t[9 + 3 * e + d] = cx[30 * (size_t)L + 3 * (4 + te) + d];
            }
            if (R < 0) continue;
            // the neighbour's vertices matched by position
            int nl[3];
            double h2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                nl[a] = -1;
                double best = INFINITY;
                for (int k = 0; k < 4; ++k) {
                    double dd = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const double u = cx[30 * (size_t)R + 3 * k + d] + m->face_shift[3 * (size_t)f + d] - t[3 * a + d];
                        dd += u * u;
                    }
                    if (dd < best) { best = dd; nl[a] = k; }
                }
                for (int d = 0; d < 3; ++d) {
                    const double u = t[3 * a + d] - t[3 * ((a + 1) % 3) + d];
                    h2 = std::max(h2, u * u);
                }
            }
            for (int e = 0; e < 3; ++e) {
                const int te = tet_edge_index(nl[fe[e][0]], nl[fe[e][1]]);
                if (te < 0) return fail(c, GKS_E_MESH, "a shared face's vertices do not match");
                double dd = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const double u = cx[30 * (size_t)R + 3 * (4 + te) + d] + m->face_shift[3 * (size_t)f + d] - t[9 + 3 * e + d];
                    dd += u * u;
                }
                if (dd > 1e-20 * h2)
                    return fail(c, GKS_E_MESH, "the quadratic control points of a shared face differ between its cells");
            }
        }
    }
    bool curved = false;
    for (int f = 0; f < nf; ++f) curved = curved || fcurv[f];

    // --- renumbering: Morton order of centroids --------------------------
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < nc; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], cen[3 * i + d]);
            hi[d] = std::max(hi[d], cen[3 * i + d]);
        }
    std::vector<uint64_t> key(nc);
    for (int i = 0; i < nc; ++i) {
        uint64_t k = 0;
        for (int d = 0; d < 3; ++d) {
            const double span = hi[d] - lo[d];
            const double t = span > 0 ? (cen[3 * i + d] - lo[d]) / span : 0.0;
            const uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, t * 2097151.0));
            k |= spread_bits(q) << d;
        }
        key[i] = k;
    }
    std::vector<int> cperm(nc), cinv(nc);
    std::iota(cperm.begin(), cperm.end(), 0);
    std::stable_sort(cperm.begin(), cperm.end(), [&](int a, int b) { return key[a] < key[b]; });
    for (int i = 0; i < nc; ++i) cinv[cperm[i]] = i;
    std::vector<int> fkey(nf);
    for (int f = 0; f < nf; ++f)
    {
        // interior faces by their lower internal cell; on a mesh with quadratic
        // faces those after the flat ones; wall faces after all of them (by
        // owner), so that the flux runs each group as a launch of its own
        const int64_t L = m->face_cell[2 * (size_t)f], R = m->face_cell[2 * (size_t)f + 1];
        fkey[f] = R < 0 ? (curved ? 2 : 1) * nc + cinv[L] : (fcurv[f] ? nc : 0) + std::min(cinv[L], cinv[R]);
    }
    std::vector<int> fperm(nf), finv(nf);
    std::iota(fperm.begin(), fperm.end(), 0);
    std::stable_sort(fperm.begin(), fperm.end(), [&](int a, int b) { return fkey[a] < fkey[b]; });
    for (int j = 0; j < nf; ++j) finv[fperm[j]] = j;
    // faces [nfc, nf) take the quadratic path: a normal and a weight per
    // Gauss point; on a mesh without bent edges nfc = nf
    int nfc = nf;
    if (curved) {
        nfc = 0;
        for (int f = 0; f < nf; ++f) nfc += (m->face_cell[2 * (size_t)f + 1] >= 0 && !fcurv[f]) ? 1 : 0;
    }
    const int ncf = nf - nfc;

    // --- face geometry (internal order) ----------------------------------
    std::vector<double> fgeo((size_t)gks::NFGEO * nf), fnrm64(3 * (size_t)nf);
    std::vector<int> fcell(2 * (size_t)nf);
    std::vector<double> farea(nf), fnrm(3 * (size_t)nf), avec(3 * (size_t)nf), gpa(9 * (size_t)nf);
    std::vector<double> cgeo((size_t)gks::kCurvedFaceRows * ncf), cnrm(9 * (size_t)ncf);
    for (int j = 0; j < nf; ++j) {
        const int f = fperm[j];
        const int L = (int)m->face_cell[2 * (size_t)f], R = (int)m->face_cell[2 * (size_t)f + 1];
        double x[3][3];
        for (int a = 0; a < 3; ++a) {
            const int64_t id = m->face_vert[3 * (size_t)f + a];
            if (id < 0 || id >= m->n_vert) return fail(c, GKS_E_MESH, "face vertex id out of range");
            for (int d = 0; d < 3; ++d) x[a][d] = m->xyz[3 * id + d];
        }
        double e1[3], e2[3], cr[3];
        sub3(x[1], x[0], e1);
        sub3(x[2], x[0], e2);
        cross3(e1, e2, cr);
        const double nrm = std::sqrt(dot3(cr, cr));
        if (!(nrm > 0.0)) return fail(c, GKS_E_MESH, "degenerate face");
        // Gauss points (1/6,1/6), (2/3,1/6), (1/6,2/3) of the reference triangle
        const double gpw[3][2] = {{1.0 / 6.0, 1.0 / 6.0}, {2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}};
        double gp[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d)
                gp[k][d] = x[0][d] * (1.0 - gpw[k][0] - gpw[k][1]) + x[1][d] * gpw[k][0] +
                           x[2][d] * gpw[k][1];
        double out = 0.0;
        for (int d = 0; d < 3; ++d) out += cr[d] * (gp[0][d] - cen[3 * L + d]);
        const double sg = out > 0 ? 1.0 : -1.0;
        for (int d = 0; d < 3; ++d) {
            const double nd = sg * cr[d] / nrm;
            fgeo[(size_t)(gks::F_N + d) * nf + j] = nd;
            fnrm64[(size_t)d * nf + j] = nd;
            fnrm[3 * (size_t)f + d] = nd;
        }
        farea[f] = 0.5 * nrm;
        double pn[3][3], pa[3];  // per Gauss point: unit normal, area scale |X_xi x X_eta| / 2
        for (int k = 0; k < 3; ++k) {
            pa[k] = farea[f];
            for (int d = 0; d < 3; ++d) pn[k][d] = fnrm[3 * (size_t)f + d];
        }
        if (fcurv[f]) {
            // eq. flux-para-coord-gauss on the six-node triangle: weight
            // (1/2)(1/3)|X_xi x X_eta| and normal X_xi x X_eta / |.| per point
            const double(*t)[3] = reinterpret_cast<const double(*)[3]>(&fctrl[18 * (size_t)f]);
            double area = 0.0;
            for (int k = 0; k < 3; ++k) {
                double cq[3];
                qtri_eval(t, gpw[k][0], gpw[k][1], gp[k], cq);
                const double jq = std::sqrt(dot3(cq, cq));
                if (!(jq > 0.0)) return fail(c, GKS_E_MESH, "degenerate quadratic face");
                pa[k] = 0.5 * jq;
                area += pa[k] / 3.0;
                for (int d = 0; d < 3; ++d) pn[k][d] = sg * cq[d] / jq;
            }
            farea[f] = area;
        }
        for (int d = 0; d < 3; ++d)
            avec[3 * (size_t)f + d] = (pa[0] * pn[0][d] + pa[1] * pn[1][d] + pa[2] * pn[2][d]) / 3.0;
        if (j >= nfc) {
            // the cell update takes this face's gradient terms per Gauss point
            for (int d = 0; d < 3; ++d) fnrm64[(size_t)d * nf + j] = 0.0;
        }
        if (j >= nfc)
            for (int k = 0; k < 3; ++k) {
                for (int d = 0; d < 3; ++d) {
                    cgeo[(size_t)(4 * k + d) * ncf + (j - nfc)] = pn[k][d];
                    cnrm[(size_t)(3 * k + d) * ncf + (j - nfc)] = pn[k][d];
                }
                cgeo[(size_t)(4 * k + 3) * ncf + (j - nfc)] = pa[k];
            }
        fgeo[(size_t)gks::F_AREA * nf + j] = farea[f];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) {
                gpa[9 * (size_t)f + 3 * k + d] = gp[k][d];
                fgeo[(size_t)(gks::F_RL + 3 * k + d) * nf + j] = gp[k][d] - cen[3 * L + d];
            }
        for (int d = 0; d < 3; ++d)
            fgeo[(size_t)(gks::F_D + d) * nf + j] =
                R < 0 ? 0.0 : cen[3 * L + d] - (cen[3 * R + d] + m->face_shift[3 * (size_t)f + d]);
        fcell[j] = cinv[L];
        fcell[(size_t)nf + j] = R < 0 ? -1 : cinv[R];
    }

    // --- cells: geometry rows, neighbours, operators (internal order) ----
    std::vector<double> geoR((size_t)gks::NGEO_R * nc), geoD((size_t)gks::NGEO_D * nc);
    std::vector<double> M1(12 * (size_t)nc), M2(gks::kM2Rows * gks::m2_padded_cells(nc), 0.0);
    std::vector<int> nbr(4 * (size_t)nc), cface(4 * (size_t)nc), bmode(nc, 0), ccell(nc, -1);
    std::vector<double> cpts_host;  // [ncc][36], transposed at binding
    for (int ii = 0; ii < nc; ++ii) {
        const int i = cperm[ii];
        const double V = vol[i];
        const double *ci = &cen[3 * (size_t)i];
        double rv[4][3];
        for (int a = 0; a < 4; ++a) {
            const int64_t id = m->tet[4 * (size_t)i + a];
            for (int d = 0; d < 3; ++d) rv[a][d] = m->xyz[3 * id + d] - ci[d];
        }
        // second moments about the centroid
        double C[6];
        for (int k = 0; k < 6; ++k) C[k] = cmom[6 * (size_t)i + k];
        double sumA = 0.0, closure[3] = {0, 0, 0};
        double delta[4][3], Cm[4][6];
        for (int a = 0; a < 4; ++a) {
            const int f = slot_face[4 * (size_t)i + a], side = slot_side[4 * (size_t)i + a];
            const int L = (int)m->face_cell[2 * (size_t)f], R = (int)m->face_cell[2 * (size_t)f + 1];
            const int other = side == 0 ? R : L;
            const double sgn = side == 0 ? 1.0 : -1.0;
            sumA += farea[f];
            for (int d = 0; d < 3; ++d) closure[d] += sgn * avec[3 * (size_t)f + d];
            nbr[(size_t)a * nc + ii] = other < 0 ? -1 : cinv[other];
            cface[(size_t)a * nc + ii] = 2 * finv[f] + side;
            if (other < 0) {
                for (int d = 0; d < 3; ++d) delta[a][d] = 0.0;
                for (int k = 0; k < 6; ++k) Cm[a][k] = 0.0;
                continue;
            }
            // neighbour centroid next to this cell
            for (int d = 0; d < 3; ++d) {
                const double off = side == 0 ? m->face_shift[3 * (size_t)f + d] : -m->face_shift[3 * (size_t)f + d];
                delta[a][d] = cen[3 * (size_t)other + d] + off - ci[d];
            }
            for (int k = 0; k < 6; ++k) Cm[a][k] = cmom[6 * (size_t)other + k];
        }
        if (std::sqrt(dot3(closure, closure)) > 1e-10 * sumA)
            return fail(c, GKS_E_MESH, "a cell surface is not closed");
        const double h = std::cbrt(V);
        double *g = geoR.data(), *gd = geoD.data();
        gd[(size_t)gks::G_INVVOL * nc + ii] = 1.0 / V;
        gd[(size_t)gks::G_DR * nc + ii] = 3.0 * V / sumA;
        gd[(size_t)gks::G_VOL * nc + ii] = V;
        g[(size_t)gks::G_VOL23 * nc + ii] = std::pow(V, 2.0 / 3.0);
        g[(size_t)gks::G_VOL43 * nc + ii] = std::pow(V, 4.0 / 3.0);
        for (int k = 0; k < 6; ++k) g[(size_t)(gks::G_C + k) * nc + ii] = C[k];
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d) g[(size_t)(gks::G_RV + 3 * a + d) * nc + ii] = rv[a][d];
        if (ccurv[i]) {
            // the positivity check of a quadratic cell runs at its faces' Gauss
            // points, which its vertices no longer give
            ccell[ii] = (int)(cpts_host.size() / gks::kCurvedCellRows);
            for (int a = 0; a < 4; ++a) {
                const int f = slot_face[4 * (size_t)i + a], side = slot_side[4 * (size_t)i + a];
                for (int k = 0; k < 3; ++k)
                    for (int d = 0; d < 3; ++d)
                        cpts_host.push_back(gpa[9 * (size_t)f + 3 * k + d] -
                                            (side ? m->face_shift[3 * (size_t)f + d] : 0.0) - ci[d]);
            }
        }

        // the neighbours present (a cell at a wall has fewer than four)
        int pres[4], np = 0;
        for (int a = 0; a < 4; ++a)
            if (nbr[(size_t)a * nc + ii] >= 0) pres[np++] = a;

        // step 1: least squares of the neighbour averages, D b' = dQ, D = delta / h;
        // fewer than three neighbours: the cell's own averaged gradient (bmode);
        // a singular stencil: zero slopes
        if (np >= 3) {
            double D[12], Dp[12];
            for (int k = 0; k < np; ++k)
                for (int d = 0; d < 3; ++d) D[3 * k + d] = delta[pres[k]][d] / h;
            if (pseudo_inverse(np, 3, D, Dp))
                for (int d = 0; d < 3; ++d)
                    for (int k = 0; k < np; ++k) M1[(size_t)(4 * d + pres[k]) * nc + ii] = Dp[d * np + k] / h;
        } else {
            bmode[ii] = 1;
        }

        // step 2: constrained least squares in y = (x - c) / h for the 9
        // coefficients of the basis y^k - <y^k>_0: equality rows E (neighbour
        // averages), least-squares rows A (neighbour averaged derivatives)
        double E[4][9], A[12][9];
        for (int k = 0; k < np; ++k) {
            const int a = pres[k];
            double dl[3];
            for (int d = 0; d < 3; ++d) dl[d] = delta[a][d] / h;
            for (int d = 0; d < 3; ++d) E[k][d] = dl[d];
            for (int t = 0; t < 6; ++t)
                E[k][3 + t] = dl[QA[t]] * dl[QB[t]] + (Cm[a][t] - C[t]) / (h * h);
            for (int j = 0; j < 3; ++j) {
                double *row = A[3 * k + j];
                for (int d = 0; d < 3; ++d) row[d] = j == d ? 1.0 : 0.0;
                for (int t = 0; t < 6; ++t) {
                    const int p = QA[t], q = QB[t];
                    double v = 0.0;
                    if (j == p) v += dl[q];
                    if (j == q) v += dl[p];
                    row[3 + t] = v;
                }
            }
        }
        // physical outputs: g = a_lin / h; H_pp = 2 a / h^2; H_pq = a / h^2; inputs e, h * dQ/dx
        const double osc[9] = {1 / h, 1 / h, 1 / h, 2 / (h * h), 2 / (h * h), 2 / (h * h),
                               1 / (h * h), 1 / (h * h), 1 / (h * h)};
        bool fitted = false;
        if (np >= 3) {
            // null-space method: E^T = Q [R; 0]; a = Q1 R^{-T} e + Q2 z,
            // z = (A Q2)^+ (b - A Q1 R^{-T} e)
            const int nz = 9 - np, na = 3 * np;
            double Et[9 * 4], Q[81];
            for (int r = 0; r < 9; ++r)
                for (int k = 0; k < np; ++k) Et[r * np + k] = E[k][r];
            householder_qr(9, np, Et, Q);
            double Rinv_t[16];
            for (int r = 0; r < np; ++r)
                for (int t = 0; t < np; ++t) Rinv_t[r * np + t] = r == t ? 1.0 : 0.0;
            double AQ2[12 * 6], AQ2p[6 * 12];
            if (lower_solve_transposed(np, Et, np, Rinv_t, np)) {
                double Y[9 * 4];  // Q1 R^{-T}
                for (int r = 0; r < 9; ++r)
                    for (int t = 0; t < np; ++t) {
                        double v = 0.0;
                        for (int k = 0; k < np; ++k) v += Q[r * 9 + k] * Rinv_t[k * np + t];
                        Y[r * np + t] = v;
                    }
                for (int r = 0; r < na; ++r)
                    for (int t = 0; t < nz; ++t) {
                        double v = 0.0;
                        for (int k = 0; k < 9; ++k) v += A[r][k] * Q[k * 9 + np + t];
                        AQ2[r * nz + t] = v;
                    }
                if (pseudo_inverse(na, nz, AQ2, AQ2p)) {
                    double Mb[9 * 12], Me[9 * 4];
                    for (int r = 0; r < 9; ++r)
                        for (int t = 0; t < na; ++t) {
                            double v = 0.0;
                            for (int k = 0; k < nz; ++k) v += Q[r * 9 + np + k] * AQ2p[k * na + t];
                            Mb[r * na + t] = v;
                        }
                    for (int r = 0; r < 9; ++r)
                        for (int t = 0; t < np; ++t) {
                            double v = 0.0;
                            for (int k = 0; k < na; ++k) {
                                double ay = 0.0;
                                for (int l = 0; l < 9; ++l) ay += A[k][l] * Y[l * np + t];
                                v += Mb[r * na + k] * ay;
                            }
                            Me[r * np + t] = Y[r * np + t] - v;
                        }
                    for (int r = 0; r < 9; ++r)
                        for (int k = 0; k < np; ++k) {
                            const int a = pres[k];
                            M2[gks::m2_index(16 * r + a, ii)] = osc[r] * Me[r * np + k];
                            for (int j = 0; j < 3; ++j)
                                M2[gks::m2_index(16 * r + 4 + 3 * a + j, ii)] = osc[r] * h * Mb[r * na + 3 * k + j];
                        }
                    fitted = true;
                }
            }
        }
        // the linear polynomial fitted to the step-2 data in the least-squares
        // sense (H = 0), as rows of a (g, H) operator on d
        auto linear_fallback = [&](auto put) {
            if (np == 0) return;
            const int nr = 4 * np;
            double Lr[16 * 3], Lp[3 * 16];
            for (int k = 0; k < np; ++k)
                for (int d = 0; d < 3; ++d) Lr[3 * k + d] = E[k][d];
            for (int r = 0; r < 3 * np; ++r)
                for (int d = 0; d < 3; ++d) Lr[3 * (np + r) + d] = A[r][d];
            if (pseudo_inverse(nr, 3, Lr, Lp))
                for (int d = 0; d < 3; ++d)
                    for (int k = 0; k < np; ++k) {
                        const int a = pres[k];
                        put(16 * d + a, osc[d] * Lp[d * nr + k]);
                        for (int j = 0; j < 3; ++j) put(16 * d + 4 + 3 * a + j, osc[d] * h * Lp[d * nr + np + 3 * k + j]);
                    }
        };
        if (!fitted) {
            // fewer than three neighbours or a singular system (boundary cells,
            // Sec. 4.4)
            linear_fallback([&](int row, double v) { M2[gks::m2_index(row, ii)] = v; });
        }

        // no-slip walls (Sec. 4.4): constrained fits of the momentum set (every
        // no-slip face) and the energy set (isothermal faces)
        int ws_slot[2][4], ws_n[2] = {0, 0};
        for (int a = 0; a < 4; ++a) {
            if (nbr[(size_t)a * nc + ii] >= 0) continue;
            const int t = m->face_tag[slot_face[4 * (size_t)i + a]];
            if (t == GKS_FACE_NOSLIP_ADIABATIC || t == GKS_FACE_NOSLIP_ISOTHERMAL) ws_slot[0][ws_n[0]++] = a;
            if (t == GKS_FACE_NOSLIP_ISOTHERMAL) ws_slot[1][ws_n[1]++] = a;
        }
        if (ws_n[0] > 0) {
            const size_t w = c->wcell.size();
            c->wcell.push_back(ii);
            c->wmode.resize(4 * (w + 1), gks::WM_KEEP);
            c->wop.resize(gks::kWallRows * (w + 1), 0.0);
            double *op = &c->wop[gks::kWallRows * w];
            for (int r = 0; r < gks::kM2Rows; ++r) op[gks::WR_M2 + r] = M2[gks::m2_index(r, ii)];
            for (int set = 0; set < 2; ++set) {
                const int ns = ws_n[set];
                double *o = op + set * gks::WR_SET;
                // constraint points: face centres (step 1), Gauss points (step 2)
                double xc[3][3] = {}, xg[9][3] = {}, uf[3][3] = {};
                for (int j = 0; j < ns && j < 3; ++j) {
                    const int f = slot_face[4 * (size_t)i + ws_slot[set][j]], jj = finv[f];
                    for (int d = 0; d < 3; ++d) {
                        uf[j][d] = m->face_wall_u ? m->face_wall_u[3 * (size_t)f + d] : 0.0;
                        for (int k = 0; k < 3; ++k) {
                            xg[3 * j + k][d] = fgeo[(size_t)(gks::F_RL + 3 * k + d) * nf + jj];
                            xc[j][d] += xg[3 * j + k][d] / 3.0;
                        }
                    }
                }
                for (int j = 0; j < 3; ++j)
                    for (int d = 0; d < 3; ++d) {
                        o[gks::WR_X1 + 3 * j + d] = xc[j][d];
                        o[gks::WR_U1 + 3 * j + d] = uf[j][d];
                        for (int k = 0; k < 3; ++k) {
                            o[gks::WR_X2 + 3 * (3 * j + k) + d] = xg[3 * j + k][d];
                            o[gks::WR_U2 + 3 * (3 * j + k) + d] = uf[j][d];
                        }
                    }
                // step 1: least squares on the neighbour averages with one
                // equality row per face centre: [D^T D  C^T; C  0]
                int &mode1 = c->wmode[4 * w + set];
                if (ns == 0 || ns > 3) {
                    mode1 = gks::WM_KEEP;
                } else if (np + ns < 3) {
                    mode1 = gks::WM_OWN;
                } else {
                    mode1 = gks::WM_FIT;
                    const int N = 3 + ns;
                    double K[36] = {}, Ki[36];
                    for (int r = 0; r < 3; ++r)
                        for (int t = 0; t < 3; ++t)
                            for (int k = 0; k < np; ++k) K[r * N + t] += delta[pres[k]][r] * delta[pres[k]][t] / (h * h);
                    for (int j = 0; j < ns; ++j)
                        for (int r = 0; r < 3; ++r) K[r * N + 3 + j] = K[(3 + j) * N + r] = xc[j][r] / h;
                    if (invert(N, K, Ki)) {
                        for (int d = 0; d < 3; ++d) {
                            for (int k = 0; k < np; ++k) {
                                double v = 0.0;
                                for (int r = 0; r < 3; ++r) v += Ki[d * N + r] * delta[pres[k]][r] / h;
                                o[gks::WR_K1N + 4 * d + pres[k]] = v / h;
                            }
                            for (int j = 0; j < ns; ++j) o[gks::WR_K1C + 3 * d + j] = Ki[d * N + 3 + j] / h;
                        }
                    }
                }
                // step 2: least squares on the neighbour averages and averaged
                // derivatives with one equality row per wall Gauss point
                int &mode2 = c->wmode[4 * w + 2 + set];
                const int ng = 3 * ns;
                if (ns == 0) {
                    mode2 = gks::WM_KEEP;
                    continue;
                }
                mode2 = gks::WM_FIT;
                bool ok = false;
                if (ng <= 9 && 4 * np + ng >= 9) {
                    const int N = 9 + ng;
                    double K[18 * 18] = {}, Ki[18 * 18];
                    for (int r = 0; r < 9; ++r)
                        for (int t = 0; t < 9; ++t) {
                            double v = 0.0;
                            for (int k = 0; k < np; ++k) v += E[k][r] * E[k][t];
                            for (int l = 0; l < 3 * np; ++l) v += A[l][r] * A[l][t];
                            K[r * N + t] = v;
                        }
                    for (int g = 0; g < ng; ++g) {
                        double y[3], row[9];
                        for (int d = 0; d < 3; ++d) y[d] = xg[g][d] / h;
                        for (int d = 0; d < 3; ++d) row[d] = y[d];
                        for (int t = 0; t < 6; ++t) row[3 + t] = y[QA[t]] * y[QB[t]] - C[t] / (h * h);
                        for (int r = 0; r < 9; ++r) K[r * N + 9 + g] = K[(9 + g) * N + r] = row[r];
                    }
                    if (invert(N, K, Ki)) {
                        ok = true;
                        for (int r = 0; r < 9; ++r) {
                            for (int k = 0; k < np; ++k) {
                                const int a = pres[k];
                                double v = 0.0;
                                for (int t = 0; t < 9; ++t) v += Ki[r * N + t] * E[k][t];
                                o[gks::WR_K2N + 16 * r + a] = osc[r] * v;
                                for (int j = 0; j < 3; ++j) {
                                    double u = 0.0;
                                    for (int t = 0; t < 9; ++t) u += Ki[r * N + t] * A[3 * k + j][t];
                                    o[gks::WR_K2N + 16 * r + 4 + 3 * a + j] = osc[r] * h * u;
                                }
                            }
                            for (int g = 0; g < ng; ++g) o[gks::WR_K2C + 9 * r + g] = osc[r] * Ki[r * N + 9 + g];
                        }
                    }
                }
                if (!ok) linear_fallback([&](int row, double v) { o[gks::WR_K2N + row] = v; });
            }
        }
    }

    int nwall = 0;
    for (int f = 0; f < nf; ++f) nwall += m->face_cell[2 * (size_t)f + 1] < 0 ? 1 : 0;
    c->wtag.assign(nwall, gks::WALL_SLIP);
    c->wvel.assign(3 * (size_t)nwall, 0.0);
    c->farfield = false;
    for (int j = nf - nwall; j < nf; ++j) {
        const int f = fperm[j], k = j - (nf - nwall);
        c->wtag[k] = m->face_tag[f];
        c->farfield = c->farfield || m->face_tag[f] == GKS_FACE_FARFIELD;
        for (int d = 0; d < 3; ++d)
            c->wvel[(size_t)d * nwall + k] = m->face_wall_u ? m->face_wall_u[3 * (size_t)f + d] : 0.0;
    }
    c->nwc = (int)c->wcell.size();
    c->nc = nc;
    c->nf = nf;
    c->nfi = nf - nwall;
    c->cperm.swap(cperm);
    c->fperm.swap(fperm);
    // back slots: slot b of neighbour j = nbr[a][i] is the same face as slot a of i
    std::vector<int> bslot(4 * (size_t)nc, -1);
    for (int ii = 0; ii < nc; ++ii)
        for (int a = 0; a < 4; ++a) {
            const int j = nbr[(size_t)a * nc + ii];
            if (j < 0) continue;
            const int f = cface[(size_t)a * nc + ii] >> 1;
            for (int b = 0; b < 4; ++b)
                if ((cface[(size_t)b * nc + j] >> 1) == f) {
                    bslot[(size_t)a * nc + ii] = b;
                    break;
                }
            if (bslot[(size_t)a * nc + ii] < 0) return fail(c, GKS_E_MESH, "inconsistent face-cell adjacency");
        }
    c->bslot.swap(bslot);
    c->bmode.swap(bmode);
    c->nbr.swap(nbr);
    c->cface.swap(cface);
    c->fcell.swap(fcell);
    c->M1.swap(M1);
    c->M2.swap(M2);
    c->geoR.swap(geoR);
    c->geoD.swap(geoD);
    c->fgeo.swap(fgeo);
    c->fnrm.swap(fnrm64);
    c->curved = curved;
    c->nfc = nfc;
    c->ncc = (int)(cpts_host.size() / gks::kCurvedCellRows);
    c->cgeo.swap(cgeo);
    c->cnrm.swap(cnrm);
    c->cpts.swap(cpts_host);
    c->ccell.swap(ccell);
    c->have_mesh = true;
    return GKS_OK;
}

gks_status gks_workspace_bytes(const gks_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return GKS_E_INVAL;
    if (!c->have_mesh) return GKS_E_STATE;
    *bytes = make_layout(c->nc, c->nf, c->fp32 ? 4 : 8, c->nf - c->nfi, c->nwc, c->nf - c->nfc, c->ncc).total;
    return GKS_OK;
}

gks_status gks_bind_workspace(gks_ctx *c, void *dev, size_t bytes)
{
    if (!c || !dev) return GKS_E_INVAL;
    if (!c->have_mesh) return fail(c, GKS_E_STATE, "no mesh uploaded");
    if (c->bound) return fail(c, GKS_E_STATE, "workspace already bound");
    if (((uintptr_t)dev) & 255) return fail(c, GKS_E_INVAL, "workspace must be 256-byte aligned");
    const Layout L = make_layout(c->nc, c->nf, c->fp32 ? 4 : 8, c->nf - c->nfi, c->nwc, c->nf - c->nfc, c->ncc);
    if (bytes < L.total) return fail(c, GKS_E_NOMEM, "workspace too small");
    char *w = (char *)dev;
    auto P = [&](int slot) { return (void *)(w + L.off[slot]); };
    DevMesh &dm = c->dm;
    DevState &ds = c->ds;
    dm.nc = c->nc;
    dm.nf = c->nf;
    dm.nfi = c->nfi;
    dm.nbr = (const int *)P(S_NBR);
    dm.cface = (const int *)P(S_CFACE);
    dm.M1 = P(S_M1);
    dm.M2 = P(S_M2);
    dm.geoR = P(S_GEOR);
    dm.geoD = (const double *)P(S_GEOD);
    dm.fcell = (const int *)P(S_FCELL);
    dm.fgeo = P(S_FGEO);
    dm.fnrm = (const double *)P(S_FNRM);
    dm.bslot = (const int *)P(S_BSLOT);
    dm.bmode = (const int *)P(S_BMODE);
    dm.wtag = (const int *)P(S_WTAG);
    dm.wvel = P(S_WVEL);
    dm.nwc = c->nwc;
    dm.wcell = (const int *)P(S_WCELL);
    dm.wmode = (const int *)P(S_WMODE);
    dm.wop = P(S_WOP);
    dm.widx = (const int *)P(S_WIDX);
    dm.nfc = c->nfc;
    dm.ncc = c->ncc;
    dm.cgeo = P(S_CGEO);
    dm.cnrm = (const double *)P(S_CNRM);
    dm.ccell = (const int *)P(S_CCELL);
    dm.cpts = P(S_CPTS);
    ds.W = (double *)P(S_W);
    ds.gW = (double *)P(S_GW);
    ds.Wn = (double *)P(S_WN);
    ds.Ln = (double *)P(S_LN);
    ds.Ltn = (double *)P(S_LTN);
    ds.slopes = P(S_SLOPES);
    ds.coef = P(S_COEF);
    ds.flag = (int *)P(S_FLAG);
    ds.FF = P(S_FF);
    ds.FT = P(S_FT);
    ds.FW0 = P(S_FW0);
    ds.FWs = P(S_FWS);
    ds.GC0 = P(S_GC0);
    ds.GCs = P(S_GCS);
    ds.red = (double *)P(S_RED);
    ds.nonphys = (int *)P(S_NONPHYS);
    c->d_cperm = (int *)P(S_CPERM);
    c->d_fperm = (int *)P(S_FPERM);
    c->staging = (double *)P(S_STAGING);
    c->istaging = (int *)P(S_ISTAGING);
    const hipStream_t st = c->stream;
    auto up = [&](void *dst, const void *src, size_t n) {
        return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
    };
    const size_t nc = c->nc, nf = c->nf;
    // bulk arrays are formed in FP64 and, in the FP32-bulk form, rounded once here
    std::vector<float> tmp;
    auto up_bulk = [&](const void *dst, const std::vector<double> &src) {
        if (!c->fp32) return up((void *)dst, src.data(), src.size() * 8);
        tmp.assign(src.begin(), src.end());
        hipError_t e = up((void *)dst, tmp.data(), tmp.size() * 4);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        return e;
    };
    HIP_TRY(c, up((void *)dm.nbr, c->nbr.data(), 4 * nc * sizeof(int)));
    HIP_TRY(c, up((void *)dm.cface, c->cface.data(), 4 * nc * sizeof(int)));
    HIP_TRY(c, up_bulk(dm.M1, c->M1));
    HIP_TRY(c, up_bulk(dm.M2, c->M2));
    HIP_TRY(c, up_bulk(dm.geoR, c->geoR));
    HIP_TRY(c, up((void *)dm.geoD, c->geoD.data(), gks::NGEO_D * nc * 8));
    HIP_TRY(c, up((void *)dm.fcell, c->fcell.data(), 2 * nf * sizeof(int)));
    HIP_TRY(c, up_bulk(dm.fgeo, c->fgeo));
    HIP_TRY(c, up((void *)dm.fnrm, c->fnrm.data(), 3 * nf * 8));
    HIP_TRY(c, up((void *)dm.bslot, c->bslot.data(), 4 * nc * sizeof(int)));
    HIP_TRY(c, up((void *)dm.bmode, c->bmode.data(), nc * sizeof(int)));
    if (!c->wtag.empty()) {
        HIP_TRY(c, up((void *)dm.wtag, c->wtag.data(), c->wtag.size() * sizeof(int)));
        HIP_TRY(c, up_bulk(dm.wvel, c->wvel));
    }
    {
        // every cell's wall-cell index (-1 for most), read by the adjoint
        std::vector<int> widx(nc, -1);
        for (int w = 0; w < c->nwc; ++w) widx[c->wcell[w]] = w;
        HIP_TRY(c, up((void *)dm.widx, widx.data(), nc * sizeof(int)));
        HIP_TRY(c, hipStreamSynchronize(st));
    }
    if (c->nwc > 0) {
        // operators per wall cell on the host, [kWallRows][nwc] on the device
        std::vector<double> wt((size_t)gks::kWallRows * c->nwc);
        for (int w = 0; w < c->nwc; ++w)
            for (int r = 0; r < gks::kWallRows; ++r)
                wt[(size_t)r * c->nwc + w] = c->wop[(size_t)gks::kWallRows * w + r];
        std::vector<int> wm(4 * (size_t)c->nwc);
        for (int w = 0; w < c->nwc; ++w)
            for (int k = 0; k < 4; ++k) wm[(size_t)k * c->nwc + w] = c->wmode[4 * (size_t)w + k];
        HIP_TRY(c, up((void *)dm.wcell, c->wcell.data(), c->nwc * sizeof(int)));
        HIP_TRY(c, up((void *)dm.wmode, wm.data(), wm.size() * sizeof(int)));
        HIP_TRY(c, up_bulk(dm.wop, wt));
        HIP_TRY(c, hipStreamSynchronize(st));
    }
    HIP_TRY(c, up((void *)dm.ccell, c->ccell.data(), nc * sizeof(int)));
    if (c->nf > c->nfc) {
        HIP_TRY(c, up_bulk(dm.cgeo, c->cgeo));
        HIP_TRY(c, up((void *)dm.cnrm, c->cnrm.data(), c->cnrm.size() * 8));
    }
    if (c->ncc > 0) {
        std::vector<double> ct((size_t)gks::kCurvedCellRows * c->ncc);
        for (int k = 0; k < c->ncc; ++k)
            for (int r = 0; r < gks::kCurvedCellRows; ++r)
                ct[(size_t)r * c->ncc + k] = c->cpts[(size_t)gks::kCurvedCellRows * k + r];
        HIP_TRY(c, up_bulk(dm.cpts, ct));
    }
    HIP_TRY(c, hipStreamSynchronize(st));
    HIP_TRY(c, up(c->d_cperm, c->cperm.data(), nc * sizeof(int)));
    HIP_TRY(c, up(c->d_fperm, c->fperm.data(), nf * sizeof(int)));
    HIP_TRY(c, gks::launch_fill_int(ds.nonphys, 0, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    // the host copies are no longer needed
    std::vector<int>().swap(c->nbr);
    std::vector<int>().swap(c->cface);
    std::vector<int>().swap(c->fcell);
    std::vector<int>().swap(c->bslot);
    std::vector<int>().swap(c->bmode);
    std::vector<int>().swap(c->wtag);
    std::vector<int>().swap(c->wcell);
    std::vector<int>().swap(c->wmode);
    std::vector<double>().swap(c->wvel);
    std::vector<double>().swap(c->wop);
    std::vector<double>().swap(c->M1);
    std::vector<double>().swap(c->M2);
    std::vector<double>().swap(c->geoR);
    std::vector<double>().swap(c->geoD);
    std::vector<double>().swap(c->fgeo);
    std::vector<double>().swap(c->fnrm);
    std::vector<double>().swap(c->cgeo);
    std::vector<double>().swap(c->cnrm);
    std::vector<double>().swap(c->cpts);
    std::vector<int>().swap(c->ccell);
    c->ws = w;
    c->ws_bytes = bytes;
    c->bound = true;
    return GKS_OK;
}

static gks_status ready(gks_ctx *c, bool need_state)
{
    if (!c) return GKS_E_INVAL;
    if (c->device_failed) return fail(c, GKS_E_DEVICE, "an earlier device error is pending: " + c->err);
    if (!c->bound) return fail(c, GKS_E_STATE, "no workspace bound");
    if (need_state && !c->have_state) return fail(c, GKS_E_STATE, "no state set (gks_init)");
    return GKS_OK;
}

static gks_status read_nonphys(gks_ctx *c, bool reset)
{
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&flag, c->ds.nonphys, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag) {
        if (reset) HIP_TRY(c, gks::launch_fill_int(c->ds.nonphys, 0, c->stream));
        return fail(c, GKS_E_NONPHYSICAL, "a cell average has non-positive density or pressure");
    }
    return GKS_OK;
}

gks_status gks_init(gks_ctx *c, const double *W, const double *gW, int32_t on_device)
{
    gks_status st = ready(c, false);
    if (st) return st;
    if (!W || !gW) return fail(c, GKS_E_INVAL, "null state pointer");
    const int nc = c->nc;
    const hipStream_t s = c->stream;
    const double *srcW = W, *srcG = gW;
    if (!on_device) {
        double *stW = c->staging, *stG = c->staging + 5 * (size_t)nc;
        HIP_TRY(c, hipMemcpyAsync(stW, W, 5 * (size_t)nc * 8, hipMemcpyHostToDevice, s));
        HIP_TRY(c, hipMemcpyAsync(stG, gW, 15 * (size_t)nc * 8, hipMemcpyHostToDevice, s));
        srcW = stW;
        srcG = stG;
    }
    HIP_TRY(c, gks::launch_permute_rows(c->ds.W, srcW, c->d_cperm, nc, 5, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(c->ds.gW, srcG, c->d_cperm, nc, 15, 0, false, s));
    HIP_TRY(c, gks::launch_fill_int(c->ds.nonphys, 0, s));
    HIP_TRY(c, gks::launch_check(c->dm, c->ds, c->par, s));
    c->have_state = false;
    c->stage1_done = false;
    st = read_nonphys(c, true);
    if (st) return st;
    c->have_state = true;
    return GKS_OK;
}

gks_status gks_compute_dt(gks_ctx *c, double cfl, double *dt)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!dt || !(cfl > 0.0) || !std::isfinite(cfl)) return fail(c, GKS_E_INVAL, "cfl must be positive and finite");
    st = timed(c, GKS_K_DT, [&] { return gks::launch_dt(c->dm, c->ds, c->par, cfl, c->stream); });
    if (st) return st;
    double v = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&v, c->ds.red + gks::kRedDt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    st = read_nonphys(c, false);
    if (st) return st;
    *dt = v;
    return GKS_OK;
}

// One stage; the time step is dt, or *dtp when dtp is not null.
static gks_status stage_impl(gks_ctx *c, int stage, double dt, const double *dtp)
{
    gks_status st;
    const hipStream_t s = c->stream;
    if ((st = timed(c, GKS_K_SLOPES, [&] { return slopes_step(c->dm, c->ds, c->par, c->fp32, s); }))) return st;
    if ((st = timed(c, GKS_K_RECON, [&] { return reconstruct_step(c->dm, c->ds, c->par, c->fp32, s); })))
        return st;
    const int mode = stage == 1 ? gks::FLUX_STAGE1 : gks::FLUX_STAGE2;
    if ((st = timed(c, stage == 1 ? GKS_K_FLUX1 : GKS_K_FLUX2, [&] {
             return gks::launch_flux(c->dm, c->ds, c->par, dt, dtp, mode, c->fp32, s);
         })))
        return st;
    return timed(c, stage == 1 ? GKS_K_UPDATE1 : GKS_K_UPDATE2,
                 [&] { return gks::launch_update(c->dm, c->ds, dt, dtp, stage, c->fp32, s); });
}

gks_status gks_stage(gks_ctx *c, int32_t stage, double dt)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, GKS_E_INVAL, "dt must be positive and finite");
    if (stage == 1) {
        if ((st = stage_impl(c, 1, dt, nullptr))) return st;
        c->stage1_done = true;
        c->stage1_dt = dt;
        return GKS_OK;
    }
    if (stage == 2) {
        if (!c->stage1_done || dt != c->stage1_dt)
            return fail(c, GKS_E_ORDER, "stage 2 needs a preceding stage 1 with the same dt");
        if ((st = stage_impl(c, 2, dt, nullptr))) return st;
        c->stage1_done = false;
        return GKS_OK;
    }
    return fail(c, GKS_E_INVAL, "stage must be 1 or 2");
}

gks_status gks_step(gks_ctx *c, double dt)
{
    gks_status st = gks_stage(c, 1, dt);
    if (st) return st;
    return gks_stage(c, 2, dt);
}

gks_status gks_step_cfl(gks_ctx *c, double cfl)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(c, GKS_E_INVAL, "cfl must be positive and finite");
    if (c->stage1_done) return fail(c, GKS_E_ORDER, "a stage 1 is pending: finish it with stage 2 first");
    st = timed(c, GKS_K_DT, [&] { return gks::launch_dt(c->dm, c->ds, c->par, cfl, c->stream); });
    if (st) return st;
    const double *dtp = c->ds.red + gks::kRedDt;
    if ((st = stage_impl(c, 1, 0.0, dtp))) return st;
    return stage_impl(c, 2, 0.0, dtp);
}

gks_status gks_last_dt(gks_ctx *c, double *dt)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!dt) return fail(c, GKS_E_INVAL, "null output");
    double v = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&v, c->ds.red + gks::kRedDt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    st = read_nonphys(c, false);
    if (st) return st;
    *dt = v;
    return GKS_OK;
}

// ---------------------------------------------------------------------------
// Discrete adjoint of one step

namespace {

// slots of the adjoint workspace; bulk arrays take bs bytes per element
enum AdjSlot {
    A_WCHK, A_GCHK, A_WS, A_GS, A_WN, A_LN, A_LTN, A_WB1, A_GB1, A_WBS, A_GBS, A_WBN, A_GBN,
    A_SLOPES1, A_SLOPES2, A_COEF1, A_COEF2, A_FF, A_FT, A_FW0, A_FWS, A_FLAG1, A_FLAG2, A_NONPHYS,
    A_CB, A_OWNW, A_OWNS, A_NBW, A_NBG, A_NBS, A_NBW1, A_WTMP, A_RED, A_EQ, A_SB, A_GC0, A_GCS, A_COUNT
};

// ncf: faces on the quadratic path (their per-point interface values)
Layout make_adj_layout(size_t nc, size_t nf, size_t bs, size_t ncf)
{
    const size_t d5 = 5 * nc * 8, d15 = 15 * nc * 8;
    const size_t sz[A_COUNT] = {
        d5, d15, d5, d15, d5, d5, d5, d5, d15, d5, d15, d5, d15,
        15 * nc * bs, 15 * nc * bs, 50 * nc * bs, 50 * nc * bs,
        5 * nf * bs, 5 * nf * bs, 5 * nf * bs, 5 * nf * bs,
        nc * sizeof(int), nc * sizeof(int), 64,
        100 * nf * 8, d5, d15, 4 * d5, 4 * d15, 4 * d15, 4 * d5, d5,
        (8 + 5 * (size_t)gks::kRedBlocks) * 8, gks::kEqRec * 3 * nf * 8, gks::kSideRec * 6 * nf * 8,
        15 * ncf * bs, 15 * ncf * bs};
    Layout L;
    size_t o = 0;
    for (int k = 0; k < A_COUNT; ++k) {
        L.off[k] = o;
        o += (sz[k] + 255) & ~size_t(255);
    }
    L.total = o;
    return L;
}

}  // namespace

gks_status gks_adjoint_workspace_bytes(const gks_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return GKS_E_INVAL;
    if (!c->have_mesh) return GKS_E_STATE;
    *bytes = make_adj_layout(c->nc, c->nf, c->fp32 ? 4 : 8, c->nf - c->nfc).total;
    return GKS_OK;
}

gks_status gks_bind_adjoint_workspace(gks_ctx *c, void *dev, size_t bytes)
{
    if (!c || !dev) return GKS_E_INVAL;
    if (!c->bound) return fail(c, GKS_E_STATE, "bind the forward workspace first");
    if (c->adj_bound) return fail(c, GKS_E_STATE, "adjoint workspace already bound");
    if (((uintptr_t)dev) & 255) return fail(c, GKS_E_INVAL, "workspace must be 256-byte aligned");
    const Layout L = make_adj_layout(c->nc, c->nf, c->fp32 ? 4 : 8, c->nf - c->nfc);
    if (bytes < L.total) return fail(c, GKS_E_NOMEM, "adjoint workspace too small");
    char *w = (char *)dev;
    auto P = [&](int k) { return (void *)(w + L.off[k]); };
    gks_ctx::Adj &a = c->adj;
    a.Wchk = (double *)P(A_WCHK);
    a.Gchk = (double *)P(A_GCHK);
    a.Ws = (double *)P(A_WS);
    a.Gs = (double *)P(A_GS);
    a.Wn = (double *)P(A_WN);
    a.Ln = (double *)P(A_LN);
    a.Ltn = (double *)P(A_LTN);
    a.Wb1 = (double *)P(A_WB1);
    a.Gb1 = (double *)P(A_GB1);
    a.Wbs = (double *)P(A_WBS);
    a.Gbs = (double *)P(A_GBS);
    a.Wbn = (double *)P(A_WBN);
    a.Gbn = (double *)P(A_GBN);
    a.slopes1 = P(A_SLOPES1);
    a.slopes2 = P(A_SLOPES2);
    a.coef1 = P(A_COEF1);
    a.coef2 = P(A_COEF2);
    a.FF = P(A_FF);
    a.FT = P(A_FT);
    a.FW0 = P(A_FW0);
    a.FWs = P(A_FWS);
    a.flag1 = (int *)P(A_FLAG1);
    a.flag2 = (int *)P(A_FLAG2);
    a.nonphys = (int *)P(A_NONPHYS);
    a.CB = (double *)P(A_CB);
    a.own_w = (double *)P(A_OWNW);
    a.own_s = (double *)P(A_OWNS);
    a.nb_w = (double *)P(A_NBW);
    a.nb_g = (double *)P(A_NBG);
    a.nb_s = (double *)P(A_NBS);
    a.nb_w1 = (double *)P(A_NBW1);
    a.Wtmp = (double *)P(A_WTMP);
    a.red = (double *)P(A_RED);
    a.EQ = (double *)P(A_EQ);
    a.SB = (double *)P(A_SB);
    a.GC0 = P(A_GC0);
    a.GCs = P(A_GCS);
    HIP_TRY(c, gks::launch_fill_int(a.nonphys, 0, c->stream));
    c->adj_bound = true;
    return GKS_OK;
}

gks_status gks_step_adjoint(gks_ctx *c, double dt, const double *W_n, const double *gW_n,
                            const double *Wbar_np1, const double *gWbar_np1, double *Wbar_n,
                            double *gWbar_n)
{
    if (!c) return GKS_E_INVAL;
    gks_status st = ready(c, false);
    if (st) return st;
    if (!c->adj_bound) return fail(c, GKS_E_STATE, "no adjoint workspace bound");
    if (!W_n || !gW_n || !Wbar_np1 || !gWbar_np1 || !Wbar_n || !gWbar_n)
        return fail(c, GKS_E_INVAL, "null pointer");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, GKS_E_INVAL, "dt must be positive and finite");
    const hipStream_t s = c->stream;
    const int nc = c->nc;
    const bool f32 = c->fp32;
    gks_ctx::Adj &a = c->adj;
    const DevMesh &dm = c->dm;
    // caller order -> internal order
    HIP_TRY(c, gks::launch_permute_rows(a.Wchk, W_n, c->d_cperm, nc, 5, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(a.Gchk, gW_n, c->d_cperm, nc, 15, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(a.Ws, W_n, c->d_cperm, nc, 5, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(a.Gs, gW_n, c->d_cperm, nc, 15, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(a.Wb1, Wbar_np1, c->d_cperm, nc, 5, 0, false, s));
    HIP_TRY(c, gks::launch_permute_rows(a.Gb1, gWbar_np1, c->d_cperm, nc, 15, 0, false, s));
    // forward recomputation of stage 1 (W*, grad W* into Ws, Gs) and of
    // stage 2's reconstruction, on the adjoint workspace
    DevState f1 = c->ds;
    f1.W = a.Ws;
    f1.gW = a.Gs;
    f1.Wn = a.Wn;
    f1.Ln = a.Ln;
    f1.Ltn = a.Ltn;
    f1.slopes = a.slopes1;
    f1.coef = a.coef1;
    f1.flag = a.flag1;
    f1.FF = a.FF;
    f1.FT = a.FT;
    f1.FW0 = a.FW0;
    f1.FWs = a.FWs;
    f1.GC0 = a.GC0;
    f1.GCs = a.GCs;
    f1.red = a.red;
    f1.nonphys = a.nonphys;
    HIP_TRY(c, slopes_step(dm, f1, c->par, f32, s));
    HIP_TRY(c, reconstruct_step(dm, f1, c->par, f32, s));
    HIP_TRY(c, gks::launch_flux(dm, f1, c->par, dt, nullptr, gks::FLUX_STAGE1, f32, s));
    HIP_TRY(c, gks::launch_update(dm, f1, dt, nullptr, 1, f32, s));
    DevState f2 = f1;
    f2.slopes = a.slopes2;
    f2.coef = a.coef2;
    f2.flag = a.flag2;
    HIP_TRY(c, slopes_step(dm, f2, c->par, f32, s));
    HIP_TRY(c, reconstruct_step(dm, f2, c->par, f32, s));
    // stage 2 in reverse: W^{n+1}, grad W^{n+1} -> W*, grad W*
    gks::AdjRecon r{};
    r.CB = a.CB;
    r.own_w = a.own_w;
    r.own_s = a.own_s;
    r.nb_w = a.nb_w;
    r.nb_g = a.nb_g;
    r.nb_s = a.nb_s;
    r.nb_w1 = a.nb_w1;
    r.Wtmp = a.Wtmp;
    r.bslot = dm.bslot;
    gks::AdjFlux fx{a.coef2, a.Wb1, a.Gb1, nullptr, nullptr, a.CB, a.EQ, a.SB};
    HIP_TRY(c, gks::launch_flux_vjp(dm, fx, c->par, dt, gks::FLUX_ADJ_STAGE2, f32, s));
    r.W = a.Ws;
    r.G = a.Gs;
    r.slopes = a.slopes2;
    r.flag = a.flag2;
    HIP_TRY(c, gks::launch_recon_vjp(dm, r, c->par, f32, s));
    HIP_TRY(c, gks::launch_wall_recon_vjp(dm, r, c->par, f32, s));
    HIP_TRY(c, gks::launch_recon_gather(dm, r, c->par, f32, a.Gbs, a.Wbs, nullptr, nullptr, s));
    // stage 1 in reverse: -> W^n, grad W^n (W^n also enters both updates directly)
    fx = gks::AdjFlux{a.coef1, a.Wb1, a.Gb1, a.Wbs, a.Gbs, a.CB, a.EQ, a.SB};
    HIP_TRY(c, gks::launch_flux_vjp(dm, fx, c->par, dt, gks::FLUX_ADJ_STAGE1, f32, s));
    r.W = a.Wchk;
    r.G = a.Gchk;
    r.slopes = a.slopes1;
    r.flag = a.flag1;
    HIP_TRY(c, gks::launch_recon_vjp(dm, r, c->par, f32, s));
    HIP_TRY(c, gks::launch_wall_recon_vjp(dm, r, c->par, f32, s));
    HIP_TRY(c, gks::launch_recon_gather(dm, r, c->par, f32, a.Gbn, a.Wbn, a.Wb1, a.Wbs, s));
    // internal order -> caller order
    HIP_TRY(c, gks::launch_permute_rows(Wbar_n, a.Wbn, c->d_cperm, nc, 5, 1, false, s));
    HIP_TRY(c, gks::launch_permute_rows(gWbar_n, a.Gbn, c->d_cperm, nc, 15, 1, false, s));
    return GKS_OK;
}

gks_status gks_read_state(gks_ctx *c, double *W, double *gW, int32_t on_device)
{
    gks_status st = ready(c, true);
    if (st) return st;
    const int nc = c->nc;
    const hipStream_t s = c->stream;
    if (on_device) {
        if (W) HIP_TRY(c, gks::launch_permute_rows(W, c->ds.W, c->d_cperm, nc, 5, 1, false, s));
        if (gW) HIP_TRY(c, gks::launch_permute_rows(gW, c->ds.gW, c->d_cperm, nc, 15, 1, false, s));
    } else {
        double *stW = c->staging, *stG = c->staging + 5 * (size_t)nc;
        if (W) {
            HIP_TRY(c, gks::launch_permute_rows(stW, c->ds.W, c->d_cperm, nc, 5, 1, false, s));
            HIP_TRY(c, hipMemcpyAsync(W, stW, 5 * (size_t)nc * 8, hipMemcpyDeviceToHost, s));
        }
        if (gW) {
            HIP_TRY(c, gks::launch_permute_rows(stG, c->ds.gW, c->d_cperm, nc, 15, 1, false, s));
            HIP_TRY(c, hipMemcpyAsync(gW, stG, 15 * (size_t)nc * 8, hipMemcpyDeviceToHost, s));
        }
    }
    return read_nonphys(c, false);
}

gks_status gks_conservation_sums(gks_ctx *c, double out[5])
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!out) return GKS_E_INVAL;
    HIP_TRY(c, gks::launch_sums(c->dm, c->ds, c->stream));
    HIP_TRY(c, hipMemcpyAsync(out, c->ds.red, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return GKS_OK;
}

gks_status gks_conservation_sums_noalloc(gks_ctx *c, double *out_device)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!out_device) return fail(c, GKS_E_INVAL, "null output pointer");
    if ((int64_t)c->nc > gks::noalloc_max_cells())
        return fail(c, GKS_E_INVAL, "gks_conservation_sums_noalloc: " + std::to_string(c->nc) +
                                        " cells exceed the fixed scratch of " +
                                        std::to_string(gks::noalloc_max_cells()) + " cells");
    HIP_TRY(c, gks::launch_sums_noalloc(c->dm, c->ds, out_device, c->stream));
    return GKS_OK;
}

// scatter bulk rows (widened to double) to the caller's order
static gks_status export_rows(gks_ctx *c, double *dst, const void *src, const int *perm, int n,
                              int rows, int on_device)
{
    const hipStream_t s = c->stream;
    if (on_device) {
        HIP_TRY(c, gks::launch_permute_rows(dst, src, perm, n, rows, 1, c->fp32, s));
    } else {
        HIP_TRY(c, gks::launch_permute_rows(c->staging, src, perm, n, rows, 1, c->fp32, s));
        HIP_TRY(c, hipMemcpyAsync(dst, c->staging, (size_t)rows * n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipStreamSynchronize(s));
    }
    return GKS_OK;
}

gks_status gks_debug_reconstruct(gks_ctx *c, double *slopes, double *coef, int32_t *flag,
                                 int32_t on_device)
{
    gks_status st = ready(c, true);
    if (st) return st;
    const hipStream_t s = c->stream;
    HIP_TRY(c, slopes_step(c->dm, c->ds, c->par, c->fp32, s));
    HIP_TRY(c, reconstruct_step(c->dm, c->ds, c->par, c->fp32, s));
    if (slopes && (st = export_rows(c, slopes, c->ds.slopes, c->d_cperm, c->nc, 15, on_device))) return st;
    if (coef && (st = export_rows(c, coef, c->ds.coef, c->d_cperm, c->nc, 50, on_device))) return st;
    if (flag) {
        if (on_device) {
            HIP_TRY(c, gks::launch_permute_int(flag, c->ds.flag, c->d_cperm, c->nc, 1, s));
        } else {
            HIP_TRY(c, gks::launch_permute_int(c->istaging, c->ds.flag, c->d_cperm, c->nc, 1, s));
            HIP_TRY(c, hipMemcpyAsync(flag, c->istaging, (size_t)c->nc * sizeof(int),
                                      hipMemcpyDeviceToHost, s));
        }
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return GKS_OK;
}

static gks_status debug_faces(gks_ctx *c, double dt, double *out, int32_t on_device, int mode)
{
    gks_status st = ready(c, true);
    if (st) return st;
    if (!out || !(dt > 0.0)) return fail(c, GKS_E_INVAL, "null output or non-positive dt");
    const hipStream_t s = c->stream;
    HIP_TRY(c, slopes_step(c->dm, c->ds, c->par, c->fp32, s));
    HIP_TRY(c, reconstruct_step(c->dm, c->ds, c->par, c->fp32, s));
    HIP_TRY(c, gks::launch_flux(c->dm, c->ds, c->par, dt, nullptr, mode, c->fp32, s));
    c->stage1_done = false;  // the face buffers of a pending stage 1 are overwritten
    const int nf = c->nf;
    const void *src[4] = {c->ds.FF, c->ds.FT, c->ds.FW0, c->ds.FWs};
    for (int k = 0; k < 4; ++k) {
        double *dst = out + (size_t)5 * k * nf;
        if ((st = export_rows(c, dst, src[k], c->d_fperm, nf, 5, on_device))) return st;
    }
    HIP_TRY(c, hipStreamSynchronize(s));
    return GKS_OK;
}

gks_status gks_debug_face_terms(gks_ctx *c, double dt, double *out, int32_t on_device)
{
    return debug_faces(c, dt, out, on_device, gks::FLUX_DEBUG);
}

gks_status gks_debug_flux_integrals(gks_ctx *c, double dt, double *out, int32_t on_device)
{
    return debug_faces(c, dt, out, on_device, gks::FLUX_DEBUG_RAW);
}

gks_status gks_timing_enable(gks_ctx *c, int32_t on)
{
    if (!c) return GKS_E_INVAL;
    c->timing = on != 0;
    return GKS_OK;
}

gks_status gks_timing_read(gks_ctx *c, double ms[GKS_NKERNELS], int64_t counts[GKS_NKERNELS],
                           int32_t reset)
{
    if (!c) return GKS_E_INVAL;
    if (c->ev_used) HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < c->ev_kernel.size(); ++k) {
        float t = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&t, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
        c->t_ms[c->ev_kernel[k]] += t;
        c->t_cnt[c->ev_kernel[k]] += 1;
    }
    c->ev_kernel.clear();
    c->ev_used = 0;
    for (int k = 0; k < GKS_NKERNELS; ++k) {
        if (ms) ms[k] = c->t_ms[k];
        if (counts) counts[k] = c->t_cnt[k];
        if (reset) {
            c->t_ms[k] = 0.0;
            c->t_cnt[k] = 0;
        }
    }
    return GKS_OK;
}

const char *gks_last_error(const gks_ctx *c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

const char *gks_strerror(gks_status st)
{
    switch (st) {
    case GKS_OK: return "GKS_OK";
    case GKS_E_INVAL: return "GKS_E_INVAL";
    case GKS_E_MESH: return "GKS_E_MESH";
    case GKS_E_NONPHYSICAL: return "GKS_E_NONPHYSICAL";
    case GKS_E_ORDER: return "GKS_E_ORDER";
    case GKS_E_DEVICE: return "GKS_E_DEVICE";
    case GKS_E_STATE: return "GKS_E_STATE";
    case GKS_E_NOMEM: return "GKS_E_NOMEM";
    default: return "unknown status";
    }
}

}  // extern "C"
