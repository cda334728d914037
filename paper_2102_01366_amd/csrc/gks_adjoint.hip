// HIP kernels of the discrete adjoint of one step: the reverse of the cell
// update, of the gas-kinetic flux and of both reconstruction steps, as the
// forward kernels implement them.  Face-to-cell and cell-to-neighbour
// accumulations are fixed-order gathers (each cell reads its four faces, each
// neighbour's contribution through the slot that points back at it), so the
// adjoint is bitwise reproducible.  Adjoint arrays are FP64; the forward
// quantities are recomputed in the bulk type R.
#include "gks_flux_adj.h"
#include "gks_internal.h"
#include "gks_recon_adj.h"

#include <cmath>

namespace gks {

namespace {

constexpr int kXcdsA = 8;
// The XCD-contiguous workgroup order of the forward kernels (a bijection of
// [0, gridDim.x)): each XCD takes one contiguous range of cells or faces.
__device__ __forceinline__ int xcd_block_a()
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int q = nb / kXcdsA, r = nb % kXcdsA, x = b % kXcdsA, k = b / kXcdsA;
    return x * q + (x < r ? x : r) + k;
}

template <typename R>
struct CoefView {
    const R *coef;
    int n, cell;
    __device__ __forceinline__ R operator()(int q, int k) const { return coef[(size_t)(10 * q + k) * n + cell]; }
};

// ===========================================================================
// Flux: three lanes per face (one per Gauss point), as the forward kernel.
// The adjoint of the face terms follows from the transpose of the update:
//   L_i = -(1/|Omega_i|) sum_f s_if F_f,  grad W_i = (1/|Omega_i|) sum_f s_if W_f n_f,
// s_if = +1 for the owner, -1 for the neighbour.
//   stage 2: W^{n+1} = W^n + dt L^n + dt^2/6 (L_t^n + 2 L_t*), grad W^{n+1} from
//            W(0) of stage 1 + (W(dt) - W(0)) of stage 2;
//   stage 1: W* = W^n + dt/2 L^n + dt^2/8 L_t^n, grad W* from (W(0) + W(dt))/2.
// ===========================================================================
constexpr int kFluxThreadsA = 256;
constexpr int kFacesPerWaveA = 21;
constexpr int kFacesPerBlockA = kFacesPerWaveA * (kFluxThreadsA / 64);

template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int nf = m.nf, n = m.nc;
    const R dt = R(dt_);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? nf : m.nfi;
    const int f = f0 + xcd_block_a() * kFacesPerBlockA + wave * kFacesPerWaveA + slot;
    const bool live = slot < kFacesPerWaveA && f < f1;
    R Wb[2][5], Gb[2][5][3], off[2][3];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Wb[sd][q] = R(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) Gb[sd][q][d] = R(0);
        }
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int d = 0; d < 3; ++d) off[sd][d] = R(0);
    if (live) {
        // a wall face has only its owner: the neighbour terms below vanish
        const int L = m.fcell[f], Rc = WALL ? L : m.fcell[nf + f];
        const double iL = m.geoD[(size_t)G_INVVOL * n + L];
        const double iR = WALL ? 0.0 : m.geoD[(size_t)G_INVVOL * n + Rc];
        double nn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) nn[d] = m.fnrm[(size_t)d * nf + f];
        const double dt2 = dt_ * dt_;
        R accb[4][5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            // sum_i s_i / |Omega_i| n . gradbar_i[q]
            double g1 = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                g1 += nn[d] * (iL * a.Gb1[(size_t)(3 * q + d) * n + L] - iR * a.Gb1[(size_t)(3 * q + d) * n + Rc]);
            const double wL = a.Wb1[(size_t)q * n + L], wR = a.Wb1[(size_t)q * n + Rc];
            if (MODE == FLUX_ADJ_STAGE2) {
                // L_t*: coefficient dt^2/3 of W^{n+1}
                accb[0][q] = R(0);
                accb[1][q] = R(dt2 / 3.0 * (-iL * wL + iR * wR));
                accb[2][q] = R(-g1);
                accb[3][q] = R(g1);
            } else {
                const double sL = a.Wbs[(size_t)q * n + L], sR = a.Wbs[(size_t)q * n + Rc];
                const double lbL = dt_ * wL + 0.5 * dt_ * sL, lbR = dt_ * wR + 0.5 * dt_ * sR;
                const double ltL = dt2 / 6.0 * wL + 0.125 * dt2 * sL, ltR = dt2 / 6.0 * wR + 0.125 * dt2 * sR;
                double gs = 0.0;
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    gs += nn[d] * (iL * a.Gbs[(size_t)(3 * q + d) * n + L] - iR * a.Gbs[(size_t)(3 * q + d) * n + Rc]);
                accb[0][q] = R(-iL * lbL + iR * lbR);
                accb[1][q] = R(-iL * ltL + iR * ltR);
                accb[2][q] = R(g1 + 0.5 * gs);
                accb[3][q] = R(0.5 * gs);
            }
        }
        const R *fg = static_cast<const R *>(m.fgeo);
        R nrm[3], dv[3], r[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            nrm[d] = fg[(size_t)(F_N + d) * nf + f];
            dv[d] = fg[(size_t)(F_D + d) * nf + f];
            r[d] = fg[(size_t)(F_RL + 3 * k + d) * nf + f];
        }
        const R area = fg[(size_t)F_AREA * nf + f];
        const R *coef = static_cast<const R *>(a.coef);
        gauss_point_vjp_point<R, VISC, PRFIX>(p, dt, nrm, area, r, dv, CoefView<R>{coef, n, L},
                                              CoefView<R>{coef, n, Rc}, accb, Wb, Gb, off, WALL);
    }
    // per side and component: the ten coefficient adjoints, summed over the
    // face's three Gauss points in order onto its first lane
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            R cb[10];
            coef_adjoint(off[sd], Wb[sd][q], Gb[sd][q], cb);
#pragma unroll
            for (int t = 0; t < 10; ++t) {
                const R v1 = __shfl_down(cb[t], 1, 64);
                const R v2 = __shfl_down(cb[t], 2, 64);
                cb[t] = (cb[t] + v1) + v2;
            }
            if (live && k == 0) {
#pragma unroll
                for (int t = 0; t < 10; ++t) a.CB[(size_t)(50 * sd + 10 * q + t) * nf + f] = double(cb[t]);
            }
        }
}

template <typename R, int MODE, bool WALL>
void launch_flux_vjp_part(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    const int nfaces = WALL ? m.nf - m.nfi : m.nfi;
    if (nfaces <= 0) return;
    const dim3 grid((unsigned)((nfaces + kFacesPerBlockA - 1) / kFacesPerBlockA)), block(kFluxThreadsA);
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (visc && prfix)
        hipLaunchKernelGGL((flux_vjp_kernel<R, MODE, true, true, WALL>), grid, block, 0, st, m, a, p, dt);
    else if (visc)
        hipLaunchKernelGGL((flux_vjp_kernel<R, MODE, true, false, WALL>), grid, block, 0, st, m, a, p, dt);
    else if (prfix)
        hipLaunchKernelGGL((flux_vjp_kernel<R, MODE, false, true, WALL>), grid, block, 0, st, m, a, p, dt);
    else
        hipLaunchKernelGGL((flux_vjp_kernel<R, MODE, false, false, WALL>), grid, block, 0, st, m, a, p, dt);
}

template <typename R, int MODE>
void launch_flux_vjp_mode(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    launch_flux_vjp_part<R, MODE, false>(m, a, p, dt, st);
    launch_flux_vjp_part<R, MODE, true>(m, a, p, dt, st);
}

// ===========================================================================
// Reconstruction step 2 (Secs. 4.1-4.3), reversed per (cell, component): the
// forward fit, indicators and weights are recomputed, then differentiated as
// implemented (|x| -> sign(x), x^(4/3) -> (4/3) x^(1/3), the normalisations,
// the positivity fallback as taken).  Thread (q, l) of a 5 x 64 block handles
// component q of cell l, as the forward kernel.
// ===========================================================================
constexpr int kRecCellsA = 64;
constexpr int kRecThreadsA = 5 * kRecCellsA;

template <typename R>
__global__ __launch_bounds__(kRecThreadsA) void recon_vjp_kernel(DevMesh m, AdjRecon a, Params p)
{
    const int n = m.nc, nf = m.nf;
    const int q = threadIdx.x / kRecCellsA;
    const int i = xcd_block_a() * kRecCellsA + (int)(threadIdx.x % kRecCellsA);
    if (i >= n) return;
    const R *geo = static_cast<const R *>(m.geoR);
    const R *M2 = static_cast<const R *>(m.M2);
    const R *slopes = static_cast<const R *>(a.slopes);

    // coefficient adjoint of (cell, component): sum over the cell's faces
    R cb[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) cb[t] = R(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int code = m.cface[s * n + i];
        const int f = code >> 1, side = code & 1;
#pragma unroll
        for (int t = 0; t < 10; ++t) cb[t] += R(a.CB[(size_t)(50 * side + 10 * q + t) * nf + f]);
    }
    int nb[4];
    bool has[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        nb[s] = m.nbr[s * n + i];
        has[s] = nb[s] >= 0;
    }
    R Q0b = R(0), bb[3] = {R(0), R(0), R(0)}, snb[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) snb[s][d] = R(0);
    R db[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) db[t] = R(0);
    if (a.flag[i]) {
        // P^0 fallback: the coefficients are (Q0, 0, ..., 0)
        Q0b = cb[0];
    } else {
        const double Q0 = a.W[(size_t)q * n + i];
        R d[16];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            d[s] = has[s] ? R(a.W[(size_t)q * n + nb[s]] - Q0) : R(0);
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                d[4 + 3 * s + dd] = has[s] ? R(a.G[(size_t)(3 * q + dd) * n + nb[s]]) : R(0);
        }
        R c[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            R acc = R(0);
#pragma unroll
            for (int t = 0; t < 16; ++t) acc += M2[m2_index(16 * r + t, i)] * d[t];
            c[r] = acc;
        }
        R C[6], b[3], sn[4][3];
#pragma unroll
        for (int t = 0; t < 6; ++t) C[t] = geo[(size_t)(G_C + t) * n + i];
        const R vol23 = geo[(size_t)G_VOL23 * n + i], vol43 = geo[(size_t)G_VOL43 * n + i];
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) b[dd] = slopes[(size_t)(3 * q + dd) * n + i];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) sn[s][dd] = has[s] ? slopes[(size_t)(3 * q + dd) * n + nb[s]] : R(0);
        WenoFwd<R> f;
        R Rq[10], cbar[9];
        weno_forward<R>(p, R(Q0), c, C, vol23, vol43, b, sn, has, f, Rq);
        weno_reverse<R>(p, c, C, vol23, vol43, b, sn, has, f, cb, Q0b, cbar, bb, snb);
        // c = M2 d
#pragma unroll
        for (int r = 0; r < 9; ++r)
#pragma unroll
            for (int t = 0; t < 16; ++t) db[t] += M2[m2_index(16 * r + t, i)] * cbar[r];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (has[s]) Q0b -= db[s];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        a.nb_w[(size_t)(5 * s + q) * n + i] = has[s] ? double(db[s]) : 0.0;
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) {
            a.nb_g[(size_t)(15 * s + 3 * q + dd) * n + i] = has[s] ? double(db[4 + 3 * s + dd]) : 0.0;
            a.nb_s[(size_t)(15 * s + 3 * q + dd) * n + i] = has[s] ? double(snb[s][dd]) : 0.0;
        }
    }
    a.own_w[(size_t)q * n + i] = double(Q0b);
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) a.own_s[(size_t)(3 * q + dd) * n + i] = double(bb[dd]);
}

// ===========================================================================
// Gathers of the neighbour terms, in slot order.  Pass 1 also reverses the
// step-1 slopes b = M1 (Q_m - Q_0) of the cell (Sec. 4.3).
// ===========================================================================
template <typename R>
__global__ __launch_bounds__(kBlock) void recon_gather1_kernel(DevMesh m, AdjRecon a, double *Gout)
{
    const int j = xcd_block_a() * kBlock + (int)threadIdx.x;
    const int n = m.nc;
    if (j >= n) return;
    const R *M1 = static_cast<const R *>(m.M1);
    int nb[4], bs[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        nb[s] = m.nbr[s * n + j];
        bs[s] = a.bslot[s * n + j];
    }
    double M[12];
#pragma unroll
    for (int t = 0; t < 12; ++t) M[t] = double(M1[(size_t)t * n + j]);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double W = a.own_w[(size_t)q * n + j];
        double G[3] = {0.0, 0.0, 0.0}, S[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) S[d] = a.own_s[(size_t)(3 * q + d) * n + j];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (nb[s] < 0) continue;
            const int i = nb[s], b = bs[s];
            W += a.nb_w[(size_t)(5 * b + q) * n + i];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                G[d] += a.nb_g[(size_t)(15 * b + 3 * q + d) * n + i];
                S[d] += a.nb_s[(size_t)(15 * b + 3 * q + d) * n + i];
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) Gout[(size_t)(3 * q + d) * n + j] = G[d];
        // a cell with fewer than three neighbours took its own averaged gradient
        // as slopes; otherwise b_d = sum_s M1[4d+s] (Q_s - Q_0) over the
        // neighbours present (M1 is zero for this cell in the first case)
        if (m.bmode[j])
#pragma unroll
            for (int d = 0; d < 3; ++d) Gout[(size_t)(3 * q + d) * n + j] += S[d];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double dqb = M[s] * S[0] + M[4 + s] * S[1] + M[8 + s] * S[2];
            const bool h = nb[s] >= 0;
            a.nb_w1[(size_t)(5 * s + q) * n + j] = h ? dqb : 0.0;
            if (h) W -= dqb;
        }
        a.Wtmp[(size_t)q * n + j] = W;
    }
}

__global__ __launch_bounds__(kBlock) void recon_gather2_kernel(DevMesh m, AdjRecon a, double *Wout,
                                                               const double *X1, const double *X2)
{
    const int j = xcd_block_a() * kBlock + (int)threadIdx.x;
    const int n = m.nc;
    if (j >= n) return;
    int nb[4], bs[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        nb[s] = m.nbr[s * n + j];
        bs[s] = a.bslot[s * n + j];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const size_t o = (size_t)q * n + j;
        double W = a.Wtmp[o];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (nb[s] >= 0) W += a.nb_w1[(size_t)(5 * bs[s] + q) * n + nb[s]];
        if (X1) W += X1[o];
        if (X2) W += X2[o];
        Wout[o] = W;
    }
}

}  // namespace

hipError_t launch_flux_vjp(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, int mode,
                           bool fp32, hipStream_t st)
{
    if (fp32) {
        if (mode == FLUX_ADJ_STAGE1)
            launch_flux_vjp_mode<float, FLUX_ADJ_STAGE1>(m, a, p, dt, st);
        else
            launch_flux_vjp_mode<float, FLUX_ADJ_STAGE2>(m, a, p, dt, st);
    } else {
        if (mode == FLUX_ADJ_STAGE1)
            launch_flux_vjp_mode<double, FLUX_ADJ_STAGE1>(m, a, p, dt, st);
        else
            launch_flux_vjp_mode<double, FLUX_ADJ_STAGE2>(m, a, p, dt, st);
    }
    return hipGetLastError();
}

hipError_t launch_recon_vjp(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, hipStream_t st)
{
    const dim3 grid((unsigned)((m.nc + kRecCellsA - 1) / kRecCellsA)), block(kRecThreadsA);
    if (fp32)
        hipLaunchKernelGGL(recon_vjp_kernel<float>, grid, block, 0, st, m, a, p);
    else
        hipLaunchKernelGGL(recon_vjp_kernel<double>, grid, block, 0, st, m, a, p);
    return hipGetLastError();
}

hipError_t launch_recon_gather(const DevMesh &m, const AdjRecon &a, bool fp32, double *Gout, double *Wout,
                               const double *X1, const double *X2, hipStream_t st)
{
    const dim3 grid((unsigned)((m.nc + kBlock - 1) / kBlock)), block(kBlock);
    if (fp32)
        hipLaunchKernelGGL(recon_gather1_kernel<float>, grid, block, 0, st, m, a, Gout);
    else
        hipLaunchKernelGGL(recon_gather1_kernel<double>, grid, block, 0, st, m, a, Gout);
    hipLaunchKernelGGL(recon_gather2_kernel, grid, block, 0, st, m, a, Wout, X1, X2);
    return hipGetLastError();
}

}  // namespace gks
