// HIP kernels of libgks for gfx950 (MI355X): one stage of the third-order
// compact gas-kinetic scheme on tetrahedra (Ji, Zhao, Shyy & Xu).
//
// Data are structure-of-arrays in internal (renumbered) order, so that
// consecutive lanes of a wavefront read consecutive addresses.  Every output
// element is written by exactly one thread; the cell update gathers its four
// faces in a fixed order, so results are bitwise reproducible.  No MFMA: the
// per-cell operators are small matrix-vector products used once per stage.
#include "gks_flux.h"
#include "gks_internal.h"

#include <cmath>

namespace gks {

__device__ __forceinline__ int gid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// ===========================================================================
// A1: reconstruction step 1 (Sec. 4.3) -- P^1 slopes b = M1 (Q_m - Q_0)
// ===========================================================================
__global__ __launch_bounds__(kBlock) void slopes_kernel(DevMesh m, DevState s)
{
    const int i = gid();
    const int n = m.nc;
    if (i >= n) return;
    int nb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) nb[a] = m.nbr[a * n + i];
    double M[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) M[k] = m.M1[(size_t)k * n + i];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double Q0 = s.W[(size_t)q * n + i];
        double dq[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) dq[a] = nb[a] >= 0 ? s.W[(size_t)q * n + nb[a]] - Q0 : 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double b = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) b += M[4 * d + a] * dq[a];
            s.slopes[(size_t)(3 * q + d) * n + i] = b;
        }
    }
}

// ===========================================================================
// A2: reconstruction step 2 (Secs. 4.1-4.3)
//   P^2 = (g, H) = M2 d about the centroid, c0 keeps the cell mean;
//   indicators beta_1 (P^1), beta_2 (P^2) in closed form for a straight
//   tetrahedron, beta_0 from the neighbours' slopes; nonlinear weights;
//   R = Q0 + alpha (P^2 - Q0) + lin (P^1 - Q0); positivity at the 12 face
//   Gauss points, else P^0 for all components.
// ===========================================================================
__device__ __forceinline__ double pow43(double x) { return pow(x, 4.0 / 3.0); }

// One block reconstructs kRecCells cells with one wavefront per conservative
// component: thread (q, l) fits component q of cell l, so each thread holds a
// single component's stencil and coefficients.  The five wavefronts read the
// same rows of M2 (one HBM read, four cache hits).  The coefficients meet in
// LDS for the cell-wide positivity check: wavefront a evaluates the three
// Gauss points of the face opposite vertex a, wavefront 4 checks the cell
// average.
constexpr int kRecCells = 64;
constexpr int kRecThreads = 5 * kRecCells;

__global__ __launch_bounds__(kRecThreads) void reconstruct_kernel(DevMesh m, DevState s, Params p)
{
    __shared__ double sR[5][10][kRecCells];
    __shared__ double sQ0[5][kRecCells];
    __shared__ int sBad[5][kRecCells];
    const int n = m.nc;
    const int q = threadIdx.x / kRecCells;  // component, uniform over the wavefront
    const int l = threadIdx.x % kRecCells;
    const int i = blockIdx.x * kRecCells + l;
    const bool live = i < n;
    const double *geo = m.geo;

    if (live) {
        const double vol23 = geo[(size_t)G_VOL23 * n + i];
        const double vol43 = geo[(size_t)G_VOL43 * n + i];
        double C[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) C[k] = geo[(size_t)(G_C + k) * n + i];
        int nb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) nb[a] = m.nbr[a * n + i];
        const double Q0 = s.W[(size_t)q * n + i];
        double d[16];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const bool has = nb[a] >= 0;
            d[a] = has ? s.W[(size_t)q * n + nb[a]] - Q0 : 0.0;
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                d[4 + 3 * a + dd] = has ? s.gW[(size_t)(3 * q + dd) * n + nb[a]] : 0.0;
        }
        double c[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += m.M2[(size_t)(16 * r + k) * n + i] * d[k];
            c[r] = acc;
        }
        // P^2 about the centroid: its value at the centroid keeps the mean
        const double c0 = Q0 - 0.5 * (c[3] * C[0] + c[4] * C[1] + c[5] * C[2]) -
                          (c[6] * C[3] + c[7] * C[4] + c[8] * C[5]);
        double R[10];
        if (!p.nonlinear) {
            R[0] = c0;
#pragma unroll
            for (int k = 0; k < 9; ++k) R[1 + k] = c[k];
        } else {
            double b[3];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) b[dd] = s.slopes[(size_t)(3 * q + dd) * n + i];
            // beta_1 = |Omega|^(2/3) |b|^2
            const double beta1 = vol23 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
            // beta_2 = |Omega|^(2/3) (|g|^2 + tr(H C H)) + |Omega|^(4/3) sum of the six H^2
            const double Hm[3][3] = {{c[3], c[6], c[7]}, {c[6], c[4], c[8]}, {c[7], c[8], c[5]}};
            const double Cm[3][3] = {{C[0], C[3], C[4]}, {C[3], C[1], C[5]}, {C[4], C[5], C[2]}};
            double trHCH = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    double hc = 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) hc += Hm[a][k] * Cm[k][bb];
                    trHCH += hc * Hm[bb][a];
                }
            double h2 = 0.0;
#pragma unroll
            for (int k = 3; k < 9; ++k) h2 += c[k] * c[k];
            const double beta2 = vol23 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + trHCH) + vol43 * h2;
            // beta_0 from the neighbours' slopes (eq. p0-non-linear-weight), over
            // the neighbours present, pairs (j, k < j) in slot order
            double b0[4];
            bool hv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                hv[a] = nb[a] >= 0;
                double ss = 0.0;
                if (hv[a]) {
#pragma unroll
                    for (int dd = 0; dd < 3; ++dd) {
                        const double v = s.slopes[(size_t)(3 * q + dd) * n + nb[a]];
                        ss += v * v;
                    }
                }
                b0[a] = vol23 * ss;
            }
            double beta0 = 0.0;
            {
                double sum = 0.0;
                int np = 0, nn = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    nn += hv[j] ? 1 : 0;
#pragma unroll
                    for (int k = 0; k < j; ++k)
                        if (hv[j] && hv[k]) {
                            sum += fabs(b0[j] - b0[k]);
                            ++np;
                        }
                }
                if (nn > 0) {
                    const double sig1 = np ? pow43(sum / np) : 0.0;
                    double w[4], ws = 0.0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        w[j] = hv[j] ? 1.0 + sig1 / (p.eps_weno + b0[j]) : 0.0;
                        if (hv[j]) ws += w[j];
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (hv[j]) beta0 += (w[j] / ws) * b0[j];
                }
            }
            const double sig = pow43(0.5 * (fabs(beta2 - beta1) + fabs(beta2 - beta0)));
            const double r2 = sig / (p.eps_weno + beta2), r1 = sig / (p.eps_weno + beta1),
                         r0 = sig / (p.eps_weno + beta0);
            double w2 = p.g22 * (1.0 + r2 * r2);
            double w1 = p.g12 * (1.0 + r1 * r1);
            const double w0 = p.g02 * (1.0 + r0 * r0);
            const double ws = w0 + w1 + w2;
            w2 /= ws;
            w1 /= ws;
            // R = w22 p2 + w12 p1 + w02 p0 collapsed: Q0 + alpha (P^2 - Q0) + lin (P^1 - Q0)
            const double alpha = w2 / p.g22;
            const double lin = w1 / p.g11 - w2 * p.g12 / (p.g22 * p.g11);
            R[0] = Q0 + alpha * (c0 - Q0);
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) R[1 + dd] = alpha * c[dd] + lin * b[dd];
#pragma unroll
            for (int k = 3; k < 9; ++k) R[1 + k] = alpha * c[k];
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) sR[q][k][l] = R[k];
        sQ0[q][l] = Q0;
    }
    __syncthreads();

    int bad = 0;
    if (live) {
        if (q < 4) {
            // Gauss points of the face opposite vertex q: r_k / 2 - r_q / 6, k != q
            double rv[4][3];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) rv[a][dd] = geo[(size_t)(G_RV + 3 * a + dd) * n + i];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k == q) continue;
                double r[3];
#pragma unroll
                for (int dd = 0; dd < 3; ++dd) r[dd] = 0.5 * rv[k][dd] - rv[q][dd] / 6.0;
                double v[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    double cf[10];
#pragma unroll
                    for (int kk = 0; kk < 10; ++kk) cf[kk] = sR[c][kk][l];
                    v[c] = cf[0] + cf[1] * r[0] + cf[2] * r[1] + cf[3] * r[2] +
                           0.5 * (cf[4] * r[0] * r[0] + cf[5] * r[1] * r[1] + cf[6] * r[2] * r[2]) +
                           cf[7] * r[0] * r[1] + cf[8] * r[0] * r[2] + cf[9] * r[1] * r[2];
                }
                const double pr =
                    (p.gamma - 1.0) * (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0]);
                if (!(v[0] > 0.0) || !(pr > 0.0)) bad = 1;
            }
        } else {
            // a non-physical cell average cannot be repaired by the fallback
            const double rho = sQ0[0][l];
            const double pr = (p.gamma - 1.0) *
                              (sQ0[4][l] - 0.5 * (sQ0[1][l] * sQ0[1][l] + sQ0[2][l] * sQ0[2][l] +
                                                  sQ0[3][l] * sQ0[3][l]) / rho);
            if (!(rho > 0.0) || !(pr > 0.0)) *s.nonphys = 1;
        }
    }
    sBad[q][l] = bad;
    __syncthreads();
    if (live) {
        const bool anybad = (sBad[0][l] | sBad[1][l] | sBad[2][l] | sBad[3][l]) != 0;
#pragma unroll
        for (int k = 0; k < 10; ++k)
            s.coef[(size_t)(10 * q + k) * n + i] = anybad ? (k == 0 ? sQ0[q][l] : 0.0) : sR[q][k][l];
        if (q == 0) s.flag[i] = anybad ? 1 : 0;
    }
}

// ===========================================================================
// B: gas-kinetic flux (Sec. 2.2) at the three Gauss points of each face
// ===========================================================================
struct DevCoef {
    const double *coef;
    int n, cell;
    __device__ __forceinline__ double operator()(int q, int k) const
    {
        return coef[(size_t)(10 * q + k) * n + cell];
    }
};

// Three lanes per face, one per Gauss point: 21 faces per wavefront (lane 63
// idle).  The lanes of a face are summed in Gauss-point order by shuffles and
// the first lane writes the face.
constexpr int kFluxThreads = 256;
constexpr int kFacesPerWave = 21;
constexpr int kFacesPerBlock = kFacesPerWave * (kFluxThreads / 64);

template <int MODE, bool VISC, bool PRFIX>
__global__ __launch_bounds__(kFluxThreads) void flux_kernel(DevMesh m, DevState s, Params p, double dt)
{
    const int nf = m.nf, n = m.nc;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f = blockIdx.x * kFacesPerBlock + wave * kFacesPerWave + slot;
    const bool live = slot < kFacesPerWave && f < nf;
    double acc[4][5];
    if (live) {
        const int L = m.fcell[f], R = m.fcell[nf + f];
        const double *fg = m.fgeo;
        double nrm[3], dv[3], r[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            nrm[d] = fg[(size_t)(F_N + d) * nf + f];
            dv[d] = fg[(size_t)(F_D + d) * nf + f];
            r[d] = fg[(size_t)(F_RL + 3 * k + d) * nf + f];
        }
        const double area = fg[(size_t)F_AREA * nf + f];
        gauss_point_terms<double, VISC, PRFIX>(p, dt, nrm, area, r, dv, DevCoef{s.coef, n, L},
                                               DevCoef{s.coef, n, R}, acc);
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[a][q] = 0.0;
    }
    // sum the three Gauss points of each face onto its first lane
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double v1 = __shfl_down(acc[a][q], 1, 64);
            const double v2 = __shfl_down(acc[a][q], 2, 64);
            acc[a][q] = (acc[a][q] + v1) + v2;
        }
    if (!live || k != 0) return;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const size_t o = (size_t)q * nf + f;
        if (MODE == FLUX_STAGE1) {
            s.FF[o] = acc[0][q];
            s.FT[o] = acc[1][q];
            s.FW0[o] = acc[2][q];
            s.FWs[o] = 0.5 * (acc[2][q] + acc[3][q]);
        } else if (MODE == FLUX_STAGE2) {
            s.FT[o] = acc[1][q];
            s.FWs[o] = acc[3][q] - acc[2][q];
        } else {
            s.FF[o] = acc[0][q];
            s.FT[o] = acc[1][q];
            s.FW0[o] = acc[2][q];
            s.FWs[o] = acc[3][q];
        }
    }
}

template <int MODE>
static void launch_flux_mode(const DevMesh &m, const DevState &s, const Params &p, double dt,
                             hipStream_t st)
{
    const dim3 grid((unsigned)((m.nf + kFacesPerBlock - 1) / kFacesPerBlock)), block(kFluxThreads);
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (visc && prfix)
        hipLaunchKernelGGL((flux_kernel<MODE, true, true>), grid, block, 0, st, m, s, p, dt);
    else if (visc)
        hipLaunchKernelGGL((flux_kernel<MODE, true, false>), grid, block, 0, st, m, s, p, dt);
    else if (prfix)
        hipLaunchKernelGGL((flux_kernel<MODE, false, true>), grid, block, 0, st, m, s, p, dt);
    else
        hipLaunchKernelGGL((flux_kernel<MODE, false, false>), grid, block, 0, st, m, s, p, dt);
}

// ===========================================================================
// C: cell update (eqs. flux-operator, s2o4, gauss-formula, step-du)
// ===========================================================================
template <int STAGE>
__global__ __launch_bounds__(kBlock) void update_kernel(DevMesh m, DevState s, double dt)
{
    const int i = gid();
    const int n = m.nc, nf = m.nf;
    if (i >= n) return;
    double L[5] = {0, 0, 0, 0, 0}, Lt[5] = {0, 0, 0, 0, 0}, G[15];
#pragma unroll
    for (int k = 0; k < 15; ++k) G[k] = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int code = m.cface[a * n + i];
        const int f = code >> 1;
        const double sg = (code & 1) ? -1.0 : 1.0;
        double nrm[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) nrm[d] = m.fgeo[(size_t)(F_N + d) * nf + f];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const size_t o = (size_t)q * nf + f;
            if (STAGE == 1) L[q] -= sg * s.FF[o];
            Lt[q] -= sg * s.FT[o];
            const double wf = STAGE == 1 ? s.FWs[o] : s.FW0[o] + s.FWs[o];
#pragma unroll
            for (int d = 0; d < 3; ++d) G[3 * q + d] += sg * wf * nrm[d];
        }
    }
    const double iv = m.geo[(size_t)G_INVVOL * n + i];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const size_t o = (size_t)q * n + i;
        const double lt = Lt[q] * iv;
        if (STAGE == 1) {
            const double l = L[q] * iv;
            const double w = s.W[o];
            s.Wn[o] = w;
            s.Ln[o] = l;
            s.Ltn[o] = lt;
            s.W[o] = w + 0.5 * dt * l + 0.125 * dt * dt * lt;
        } else {
            s.W[o] = s.Wn[o] + dt * s.Ln[o] + dt * dt / 6.0 * (s.Ltn[o] + 2.0 * lt);
        }
    }
#pragma unroll
    for (int k = 0; k < 15; ++k) s.gW[(size_t)k * n + i] = G[k] * iv;
}

// ===========================================================================
// reductions: CFL time step (exact min) and conservation sums (fixed order)
// ===========================================================================
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kBlock) void dt_pass1(DevMesh m, DevState s, Params p)
{
    __shared__ double sm[kBlock / 64];
    const int n = m.nc;
    double best = INFINITY;
    for (int i = gid(); i < n; i += gridDim.x * blockDim.x) {
        const double rho = s.W[i], ir = 1.0 / rho;
        const double u = s.W[n + i] * ir, v = s.W[2 * n + i] * ir, w = s.W[3 * n + i] * ir;
        const double pr = (p.gamma - 1.0) * (s.W[4 * n + i] - 0.5 * rho * (u * u + v * v + w * w));
        const double a = sqrt(p.gamma * pr / rho);
        const double dr = m.geo[(size_t)G_DR * n + i];
        double b = dr / (sqrt(u * u + v * v + w * w) + a);
        if (p.viscous && p.mu > 0.0) b = fmin(b, dr * dr / (3.0 * (p.mu / rho)));
        if (!(rho > 0.0) || !(pr > 0.0)) *s.nonphys = 1;
        best = fmin(best, b);
    }
    best = wave_min(best);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sm[wv] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sm[0];
        for (int k = 1; k < kBlock / 64; ++k) b = fmin(b, sm[k]);
        s.red[8 + blockIdx.x] = b;
    }
}

__global__ __launch_bounds__(kBlock) void min_pass2(DevState s, int nparts)
{
    __shared__ double sm[kBlock / 64];
    double best = INFINITY;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) best = fmin(best, s.red[8 + k]);
    best = wave_min(best);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sm[0];
        for (int k = 1; k < kBlock / 64; ++k) b = fmin(b, sm[k]);
        s.red[0] = b;
    }
}

__global__ __launch_bounds__(kBlock) void sums_pass1(DevMesh m, DevState s)
{
    __shared__ double sm[5][kBlock / 64];
    const int n = m.nc;
    double acc[5] = {0, 0, 0, 0, 0};
    for (int i = gid(); i < n; i += gridDim.x * blockDim.x) {
        const double v = m.geo[(size_t)G_VOL * n + i];
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[q] += v * s.W[(size_t)q * n + i];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const double t = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) sm[q][threadIdx.x >> 6] = t;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        double t = 0.0;
        for (int k = 0; k < kBlock / 64; ++k) t += sm[threadIdx.x][k];
        s.red[8 + (size_t)threadIdx.x * kRedBlocks + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kBlock) void sums_pass2(DevState s)
{
    __shared__ double sm[kBlock / 64];
    for (int q = 0; q < 5; ++q) {
        double t = 0.0;
        for (int k = threadIdx.x; k < kRedBlocks; k += blockDim.x) t += s.red[8 + (size_t)q * kRedBlocks + k];
        t = wave_sum(t);
        if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = t;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = 0.0;
            for (int k = 0; k < kBlock / 64; ++k) b += sm[k];
            s.red[q] = b;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void check_kernel(DevMesh m, DevState s, Params p)
{
    const int i = gid();
    const int n = m.nc;
    if (i >= n) return;
    const double rho = s.W[i];
    const double u = s.W[n + i], v = s.W[2 * n + i], w = s.W[3 * n + i];
    const double pr = (p.gamma - 1.0) * (s.W[4 * n + i] - 0.5 * (u * u + v * v + w * w) / rho);
    if (!(rho > 0.0) || !(pr > 0.0)) *s.nonphys = 1;
}

__global__ __launch_bounds__(kBlock) void permute_rows_kernel(double *dst, const double *src,
                                                              const int *perm, int n, int rows,
                                                              int scatter)
{
    const int i = gid();
    if (i >= n) return;
    const int j = perm[i];
    for (int r = 0; r < rows; ++r) {
        if (scatter)
            dst[(size_t)r * n + j] = src[(size_t)r * n + i];
        else
            dst[(size_t)r * n + i] = src[(size_t)r * n + j];
    }
}

__global__ __launch_bounds__(kBlock) void permute_int_kernel(int *dst, const int *src, const int *perm,
                                                             int n, int scatter)
{
    const int i = gid();
    if (i >= n) return;
    if (scatter)
        dst[perm[i]] = src[i];
    else
        dst[i] = src[perm[i]];
}

__global__ void fill_int_kernel(int *p, int v) { *p = v; }

// ===========================================================================
// launchers
// ===========================================================================
static inline dim3 grid_for(int n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

hipError_t launch_slopes(const DevMesh &m, const DevState &s, hipStream_t st)
{
    hipLaunchKernelGGL(slopes_kernel, grid_for(m.nc), dim3(kBlock), 0, st, m, s);
    return hipGetLastError();
}

hipError_t launch_reconstruct(const DevMesh &m, const DevState &s, const Params &p, hipStream_t st)
{
    hipLaunchKernelGGL(reconstruct_kernel, dim3((unsigned)((m.nc + kRecCells - 1) / kRecCells)),
                       dim3(kRecThreads), 0, st, m, s, p);
    return hipGetLastError();
}

hipError_t launch_flux(const DevMesh &m, const DevState &s, const Params &p, double dt, int mode,
                       hipStream_t st)
{
    if (mode == FLUX_STAGE1)
        launch_flux_mode<FLUX_STAGE1>(m, s, p, dt, st);
    else if (mode == FLUX_STAGE2)
        launch_flux_mode<FLUX_STAGE2>(m, s, p, dt, st);
    else
        launch_flux_mode<FLUX_DEBUG>(m, s, p, dt, st);
    return hipGetLastError();
}

hipError_t launch_update(const DevMesh &m, const DevState &s, double dt, int stage, hipStream_t st)
{
    if (stage == 1)
        hipLaunchKernelGGL(update_kernel<1>, grid_for(m.nc), dim3(kBlock), 0, st, m, s, dt);
    else
        hipLaunchKernelGGL(update_kernel<2>, grid_for(m.nc), dim3(kBlock), 0, st, m, s, dt);
    return hipGetLastError();
}

hipError_t launch_dt(const DevMesh &m, const DevState &s, const Params &p, hipStream_t st)
{
    int blocks = (m.nc + kBlock - 1) / kBlock;
    if (blocks > kRedBlocks) blocks = kRedBlocks;
    hipLaunchKernelGGL(dt_pass1, dim3(blocks), dim3(kBlock), 0, st, m, s, p);
    hipLaunchKernelGGL(min_pass2, dim3(1), dim3(kBlock), 0, st, s, blocks);
    return hipGetLastError();
}

hipError_t launch_sums(const DevMesh &m, const DevState &s, hipStream_t st)
{
    hipLaunchKernelGGL(sums_pass1, dim3(kRedBlocks), dim3(kBlock), 0, st, m, s);
    hipLaunchKernelGGL(sums_pass2, dim3(1), dim3(kBlock), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_check(const DevMesh &m, const DevState &s, const Params &p, hipStream_t st)
{
    hipLaunchKernelGGL(check_kernel, grid_for(m.nc), dim3(kBlock), 0, st, m, s, p);
    return hipGetLastError();
}

hipError_t launch_permute_rows(double *dst, const double *src, const int *perm, int n, int rows,
                               int scatter, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_rows_kernel, grid_for(n), dim3(kBlock), 0, st, dst, src, perm, n, rows,
                       scatter);
    return hipGetLastError();
}

hipError_t launch_permute_int(int *dst, const int *src, const int *perm, int n, int scatter,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(permute_int_kernel, grid_for(n), dim3(kBlock), 0, st, dst, src, perm, n, scatter);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int v, hipStream_t st)
{
    hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st, p, v);
    return hipGetLastError();
}

}  // namespace gks
