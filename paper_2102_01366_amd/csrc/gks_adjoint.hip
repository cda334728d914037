// HIP kernels of the discrete adjoint of one step: the reverse of both
// reconstruction steps, as the forward kernels implement them (the reverse
// of the cell update and of the gas-kinetic flux is in gks_flux_vjp.h).
// Cell-to-neighbour accumulations are fixed-order gathers (each neighbour's
// contribution through the slot that points back at it), so the adjoint is
// bitwise reproducible.  Adjoint arrays are FP64; the forward quantities are
// recomputed in the bulk type R.
#include "gks_device.h"
#include "gks_flux_adj.h"
#include "gks_internal.h"
#include "gks_m2stage.h"
#include "gks_recon_adj.h"

#include <cmath>

namespace gks {

namespace {

// ===========================================================================
// Reconstruction step 2 (Secs. 4.1-4.3), reversed per (cell, component): the
// forward fit, indicators and weights are recomputed, then differentiated as
// implemented (|x| -> sign(x), x^(4/3) -> (4/3) x^(1/3), the normalisations,
// the positivity fallback as taken).  Thread (q, l) of a 5 x 64 block handles
// component q of cell l, as the forward kernel.
// ===========================================================================
template <typename R>
__global__ __launch_bounds__(kRecThreads) void recon_vjp_kernel(DevMesh m, AdjRecon a, Params p)
{
    __shared__ __align__(16) R sBuf[kM2Chunk * kRecCells];
    const int n = m.nc, nf = m.nf;
    const int q = threadIdx.x / kRecCells;  // component, uniform over the wavefront
    const int l = threadIdx.x % kRecCells;
    const int tb = xcd_block();
    const int i = tb * kRecCells + l;
    const bool live = i < n;
    const R *geo = static_cast<const R *>(m.geoR);
    const R *tile = static_cast<const R *>(m.M2) + (size_t)tb * kM2Rows * kRecCells;
    const R *slopes = static_cast<const R *>(a.slopes);
    M2Chunk<R> pre;
    pre.load(tile, 0);

    // inputs of (cell, component): the coefficient adjoint summed over the
    // cell's faces, the fit's data d
    R cb[10], d[16];
#pragma unroll
    for (int t = 0; t < 10; ++t) cb[t] = R(0);
#pragma unroll
    for (int t = 0; t < 16; ++t) d[t] = R(0);
    int nb[4] = {-1, -1, -1, -1};
    bool has[4] = {false, false, false, false};
    bool fb = true;  // the P^0 fallback (or a padding lane): nothing to reverse but Q0
    double Q0 = 0.0;
    if (live) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int code = m.cface[s * n + i];
            const int f = code >> 1, side = code & 1;
#pragma unroll
            for (int t = 0; t < 10; ++t) cb[t] += R(a.CB[(size_t)(50 * side + 10 * q + t) * nf + f]);
            nb[s] = m.nbr[s * n + i];
            has[s] = nb[s] >= 0;
        }
        fb = a.flag[i] != 0;
        Q0 = a.W[(size_t)q * n + i];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            d[s] = has[s] ? R(a.W[(size_t)q * n + nb[s]] - Q0) : R(0);
#pragma unroll
            for (int dd = 0; dd < 3; ++dd)
                d[4 + 3 * s + dd] = has[s] ? R(a.G[(size_t)(3 * q + dd) * n + nb[s]]) : R(0);
        }
    }
    // the fit c = M2 d, operators streamed through LDS
    R c[9];
#pragma unroll
    for (int t = 0; t < kM2Chunks; ++t) {
        if (t > 0) __syncthreads();
        pre.store(sBuf);
        __syncthreads();
        if (t + 1 < kM2Chunks) pre.load(tile, t + 1);
#pragma unroll
        for (int rr = 0; rr < kM2Chunk / 16; ++rr) {
            R acc = R(0);
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += sBuf[(16 * rr + k) * kRecCells + l] * d[k];
            asm volatile("" : "+v"(acc));  // formed here, not sunk past the barriers
            c[t * (kM2Chunk / 16) + rr] = acc;
        }
    }
    pre.load(tile, 0);  // for the transposed product below
    R Q0b = fb ? cb[0] : R(0), bb[3] = {R(0), R(0), R(0)}, snb[4][3], cbar[9];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) snb[s][dd] = R(0);
#pragma unroll
    for (int r = 0; r < 9; ++r) cbar[r] = R(0);
    if (!fb) {
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
        R Rq[10];
        weno_forward<R>(p, R(Q0), c, C, vol23, vol43, b, sn, has, f, Rq);
        weno_reverse<R>(p, c, C, vol23, vol43, b, sn, has, f, cb, Q0b, cbar, bb, snb);
    }
    // db = M2^T cbar, the operators streamed again
    R db[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) db[k] = R(0);
#pragma unroll
    for (int t = 0; t < kM2Chunks; ++t) {
        __syncthreads();
        pre.store(sBuf);
        __syncthreads();
        if (t + 1 < kM2Chunks) pre.load(tile, t + 1);
#pragma unroll
        for (int rr = 0; rr < kM2Chunk / 16; ++rr) {
            const R cr = cbar[t * (kM2Chunk / 16) + rr];
#pragma unroll
            for (int k = 0; k < 16; ++k) db[k] += sBuf[(16 * rr + k) * kRecCells + l] * cr;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) asm volatile("" : "+v"(db[k]));
    }
    if (!live) return;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (has[s]) Q0b -= db[s];
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

// The second-order scheme's reconstruction reversed (weno2_reverse): no
// step-2 fit, so only the cell's own W and slopes and its neighbours' slopes
// receive adjoints.  One thread per cell.
template <typename R>
__global__ __launch_bounds__(kBlock) void recon2_vjp_kernel(DevMesh m, AdjRecon a, Params p)
{
    const int n = m.nc, nf = m.nf;
    const int i = xcd_block() * kBlock + (int)threadIdx.x;
    if (i >= n) return;
    const R *geo = static_cast<const R *>(m.geoR);
    const R *slopes = static_cast<const R *>(a.slopes);
    int nb[4];
    bool has[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        nb[s] = m.nbr[s * n + i];
        has[s] = nb[s] >= 0;
    }
    const bool fb = a.flag[i] != 0;
    const R vol23 = geo[(size_t)G_VOL23 * n + i];
#pragma unroll 1
    for (int q = 0; q < 5; ++q) {
        R cb[10];
#pragma unroll
        for (int t = 0; t < 10; ++t) cb[t] = R(0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int code = m.cface[s * n + i];
            const int f = code >> 1, side = code & 1;
#pragma unroll
            for (int t = 0; t < 4; ++t) cb[t] += R(a.CB[(size_t)(50 * side + 10 * q + t) * nf + f]);
        }
        R Q0b = cb[0], bb[3] = {R(0), R(0), R(0)}, snb[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int d = 0; d < 3; ++d) snb[s][d] = R(0);
        if (!fb) {
            R b[3], sn[4][3], Rq[10];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                b[d] = slopes[(size_t)(3 * q + d) * n + i];
#pragma unroll
                for (int s = 0; s < 4; ++s) sn[s][d] = has[s] ? slopes[(size_t)(3 * q + d) * n + nb[s]] : R(0);
            }
            Weno2Fwd<R> f;
            weno2_forward<R>(p, R(a.W[(size_t)q * n + i]), vol23, b, sn, has, f, Rq);
            weno2_reverse<R>(p, vol23, b, sn, has, f, cb, Q0b, bb, snb);
        }
        a.own_w[(size_t)q * n + i] = double(Q0b);
#pragma unroll
        for (int d = 0; d < 3; ++d) a.own_s[(size_t)(3 * q + d) * n + i] = double(bb[d]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            a.nb_w[(size_t)(5 * s + q) * n + i] = 0.0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                a.nb_g[(size_t)(15 * s + 3 * q + d) * n + i] = 0.0;
                a.nb_s[(size_t)(15 * s + 3 * q + d) * n + i] = has[s] ? double(snb[s][d]) : 0.0;
            }
        }
    }
}

// ===========================================================================
// Gathers of the neighbour terms, in slot order.  Pass 1 also reverses the
// step-1 slopes b = M1 (Q_m - Q_0) of the cell (Sec. 4.3).
// ===========================================================================
template <typename R>
__global__ __launch_bounds__(kBlock) void recon_gather1_kernel(DevMesh m, AdjRecon a, double *Gout)
{
    const int j = xcd_block() * kBlock + (int)threadIdx.x;
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
    const int j = xcd_block() * kBlock + (int)threadIdx.x;
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

hipError_t launch_recon_vjp(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, hipStream_t st)
{
    if (p.order == 2) {
        const dim3 g((unsigned)((m.nc + kBlock - 1) / kBlock)), b(kBlock);
        if (fp32)
            hipLaunchKernelGGL(recon2_vjp_kernel<float>, g, b, 0, st, m, a, p);
        else
            hipLaunchKernelGGL(recon2_vjp_kernel<double>, g, b, 0, st, m, a, p);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((m.nc + kRecCells - 1) / kRecCells)), block(kRecThreads);
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
