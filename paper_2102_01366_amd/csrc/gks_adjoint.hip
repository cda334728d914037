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
// No-slip wall cells (Sec. 4.4), step 2 reversed: the whole reconstruction of
// a wall cell as the forward fixup computes it (block of kRecCells wall cells,
// one wavefront per component), then its reverse.  A constrained component's
// wall values rho_rec(x_g) U_wall (or the energy's) feed the density's final
// polynomial, so the constrained components reverse first and hand their
// adjoint of that polynomial to the density through LDS.  The outputs replace
// what recon_vjp_kernel wrote for these cells.
// ===========================================================================
template <typename R>
__global__ __launch_bounds__(kRecThreads) void wall_recon_vjp_kernel(DevMesh m, AdjRecon a, Params p)
{
    __shared__ R sRho[10][kRecCells];
    __shared__ R sRb[4][10][kRecCells];
    const int nw = m.nwc, n = m.nc, nf = m.nf;
    const int q = threadIdx.x / kRecCells, l = threadIdx.x % kRecCells;
    const int w = blockIdx.x * kRecCells + l;
    const bool live = w < nw;
    const int i = live ? m.wcell[w] : 0;
    const R *op = static_cast<const R *>(m.wop);
    const R *geo = static_cast<const R *>(m.geoR);
    const R *slopes = static_cast<const R *>(a.slopes);
    const int set = q < 4 ? 0 : 1, base = set * WR_SET;
    const int mode = (q == 0 || !live) ? WM_KEEP : m.wmode[(size_t)(2 + set) * nw + w];
    R cb[10], d[16], c[9], Rq[10], b[3], sn[4][3], C[6], vol23 = R(0), vol43 = R(0);
    int nb[4] = {-1, -1, -1, -1};
    bool has[4] = {false, false, false, false}, fb = true;
    double Q0 = 0.0;
#pragma unroll
    for (int t = 0; t < 10; ++t) cb[t] = R(0);
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
            for (int dd = 0; dd < 3; ++dd) {
                d[4 + 3 * s + dd] = has[s] ? R(a.G[(size_t)(3 * q + dd) * n + nb[s]]) : R(0);
                sn[s][dd] = has[s] ? slopes[(size_t)(3 * q + dd) * n + nb[s]] : R(0);
            }
        }
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) b[dd] = slopes[(size_t)(3 * q + dd) * n + i];
#pragma unroll
        for (int t = 0; t < 6; ++t) C[t] = geo[(size_t)(G_C + t) * n + i];
        vol23 = geo[(size_t)G_VOL23 * n + i];
        vol43 = geo[(size_t)G_VOL43 * n + i];
    }
    // forward: the fits, the density's final polynomial first
    WenoFwd<R> f;
    R ec[9];
    if (live && mode == WM_KEEP) {
        for (int r = 0; r < 9; ++r) {
            R acc = R(0);
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += op[(size_t)(WR_M2 + 16 * r + k) * nw + w] * d[k];
            c[r] = acc;
        }
        weno_forward<R>(p, R(Q0), c, C, vol23, vol43, b, sn, has, f, Rq);
    }
    if (live && q == 0)
#pragma unroll
        for (int k = 0; k < 10; ++k) sRho[k][l] = Rq[k];
    __syncthreads();
    if (live && mode != WM_KEEP) {
        for (int g = 0; g < 9; ++g) {
            R x[3], u[3], Rr[10];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                x[dd] = op[(size_t)(base + WR_X2 + 3 * g + dd) * nw + w];
                u[dd] = op[(size_t)(base + WR_U2 + 3 * g + dd) * nw + w];
            }
#pragma unroll
            for (int k = 0; k < 10; ++k) Rr[k] = sRho[k][l];
            ec[g] = wall_value(q, quad_value(Rr, x), u, R(p.gamma), R(p.wall_T)) - R(Q0);
        }
        for (int r = 0; r < 9; ++r) {
            R acc = R(0);
#pragma unroll
            for (int k = 0; k < 16; ++k) acc += op[(size_t)(base + WR_K2N + 16 * r + k) * nw + w] * d[k];
#pragma unroll
            for (int g = 0; g < 9; ++g) acc += op[(size_t)(base + WR_K2C + 9 * r + g) * nw + w] * ec[g];
            c[r] = acc;
        }
        weno_forward<R>(p, R(Q0), c, C, vol23, vol43, b, sn, has, f, Rq);
    }
    // reverse of the non-density components
    R Q0b = fb ? cb[0] : R(0), bb[3] = {R(0), R(0), R(0)}, snb[4][3], db[16];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) snb[s][dd] = R(0);
#pragma unroll
    for (int k = 0; k < 16; ++k) db[k] = R(0);
    // cbar -> db (and, for a constrained component, the wall values' adjoints)
    auto reverse_fit = [&](const R cbar[9]) {
        if (mode == WM_KEEP) {
            for (int r = 0; r < 9; ++r)
#pragma unroll
                for (int k = 0; k < 16; ++k) db[k] += op[(size_t)(WR_M2 + 16 * r + k) * nw + w] * cbar[r];
            return;
        }
        for (int r = 0; r < 9; ++r)
#pragma unroll
            for (int k = 0; k < 16; ++k) db[k] += op[(size_t)(base + WR_K2N + 16 * r + k) * nw + w] * cbar[r];
        R Rrb[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) Rrb[k] = R(0);
        for (int g = 0; g < 9; ++g) {
            R ecb = R(0);
            for (int r = 0; r < 9; ++r) ecb += op[(size_t)(base + WR_K2C + 9 * r + g) * nw + w] * cbar[r];
            Q0b -= ecb;
            R x[3], u[3], e[10];
#pragma unroll
            for (int dd = 0; dd < 3; ++dd) {
                x[dd] = op[(size_t)(base + WR_X2 + 3 * g + dd) * nw + w];
                u[dd] = op[(size_t)(base + WR_U2 + 3 * g + dd) * nw + w];
            }
            quad_basis(x, e);
            const R fr = ecb * wall_factor(q, u, R(p.gamma), R(p.wall_T));
#pragma unroll
            for (int k = 0; k < 10; ++k) Rrb[k] += fr * e[k];
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) sRb[q - 1][k][l] = Rrb[k];
    };
    if (q > 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) sRb[q - 1][k][l] = R(0);
        if (live && !fb) {
            R cbar[9];
#pragma unroll
            for (int r = 0; r < 9; ++r) cbar[r] = R(0);
            weno_reverse<R>(p, c, C, vol23, vol43, b, sn, has, f, cb, Q0b, cbar, bb, snb);
            reverse_fit(cbar);
        }
    }
    __syncthreads();
    if (q == 0 && live && !fb) {
        // the density's final polynomial also fed the wall values
#pragma unroll
        for (int k = 0; k < 10; ++k) cb[k] += sRb[0][k][l] + sRb[1][k][l] + sRb[2][k][l] + sRb[3][k][l];
        R cbar[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) cbar[r] = R(0);
        weno_reverse<R>(p, c, C, vol23, vol43, b, sn, has, f, cb, Q0b, cbar, bb, snb);
        reverse_fit(cbar);
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

// ===========================================================================
// Gathers of the neighbour terms, in slot order.  Pass 1 also reverses the
// step-1 slopes b = M1 (Q_m - Q_0) of the cell (Sec. 4.3).
// ===========================================================================
template <typename R>
__global__ __launch_bounds__(kBlock) void recon_gather1_kernel(DevMesh m, AdjRecon a, Params p, double *Gout)
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
    // the gathered adjoints of the cell's W, grad W and step-1 slopes
    double W[5], G[5][3], S[5][3];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        W[q] = a.own_w[(size_t)q * n + j];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            G[q][d] = 0.0;
            S[q][d] = a.own_s[(size_t)(3 * q + d) * n + j];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (nb[s] < 0) continue;
            const int i = nb[s], b = bs[s];
            W[q] += a.nb_w[(size_t)(5 * b + q) * n + i];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                G[q][d] += a.nb_g[(size_t)(15 * b + 3 * q + d) * n + i];
                S[q][d] += a.nb_s[(size_t)(15 * b + 3 * q + d) * n + i];
            }
        }
    }
    // no-slip wall cells (Sec. 4.4): a constrained component's slopes
    // b = K1N (Q_s - Q_0) + K1C (rho_rec(x_j) f_j - Q_0), rho_rec = rho_0 +
    // b_rho . x_j the density's step-1 polynomial; reversed before the density
    int wmode1[5] = {WM_KEEP, WM_KEEP, WM_KEEP, WM_KEEP, WM_KEEP};
    double wdq[5][4];
    const int w = m.widx[j];
    if (w >= 0) {
        const R *op = static_cast<const R *>(m.wop);
        const int nw = m.nwc;
        for (int q = 1; q < 5; ++q) {
            const int set = q < 4 ? 0 : 1, base = set * WR_SET;
            wmode1[q] = m.wmode[(size_t)set * nw + w];
            if (wmode1[q] != WM_FIT) continue;
            for (int s = 0; s < 4; ++s) {
                double v = 0.0;
                for (int d = 0; d < 3; ++d) v += double(op[(size_t)(base + WR_K1N + 4 * d + s) * nw + w]) * S[q][d];
                wdq[q][s] = v;
            }
            for (int jj = 0; jj < 3; ++jj) {
                double ecb = 0.0;
                for (int d = 0; d < 3; ++d) ecb += double(op[(size_t)(base + WR_K1C + 3 * d + jj) * nw + w]) * S[q][d];
                W[q] -= ecb;
                R x[3], u[3];
                for (int d = 0; d < 3; ++d) {
                    x[d] = op[(size_t)(base + WR_X1 + 3 * jj + d) * nw + w];
                    u[d] = op[(size_t)(base + WR_U1 + 3 * jj + d) * nw + w];
                }
                const double fr = ecb * double(wall_factor(q, u, R(p.gamma), R(p.wall_T)));
                W[0] += fr;
                for (int d = 0; d < 3; ++d) S[0][d] += fr * double(x[d]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        double Wq = W[q];
#pragma unroll
        for (int d = 0; d < 3; ++d) Gout[(size_t)(3 * q + d) * n + j] = G[q][d];
        if (wmode1[q] == WM_FIT) {
            // the constrained fit replaced the unconstrained slopes
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool h = nb[s] >= 0;
                a.nb_w1[(size_t)(5 * s + q) * n + j] = h ? wdq[q][s] : 0.0;
                if (h) Wq -= wdq[q][s];
            }
            a.Wtmp[(size_t)q * n + j] = Wq;
            continue;
        }
        // a cell with fewer than three neighbours (or a constrained component
        // with too few neighbours and constraints) took its own averaged
        // gradient as slopes; otherwise b_d = sum_s M1[4d+s] (Q_s - Q_0) over
        // the neighbours present (M1 is zero for this cell in the first case)
        const bool own = m.bmode[j] || wmode1[q] == WM_OWN;
        if (own)
#pragma unroll
            for (int d = 0; d < 3; ++d) Gout[(size_t)(3 * q + d) * n + j] += S[q][d];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double dqb = own ? 0.0 : M[s] * S[q][0] + M[4 + s] * S[q][1] + M[8 + s] * S[q][2];
            const bool h = nb[s] >= 0;
            a.nb_w1[(size_t)(5 * s + q) * n + j] = h ? dqb : 0.0;
            if (h) Wq -= dqb;
        }
        a.Wtmp[(size_t)q * n + j] = Wq;
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

hipError_t launch_flux_vjp(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, int mode, bool fp32,
                           hipStream_t st)
{
    return fp32 ? launch_flux_vjp_t<float>(m, a, p, dt, mode, st) : launch_flux_vjp_t<double>(m, a, p, dt, mode, st);
}

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

hipError_t launch_wall_recon_vjp(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, hipStream_t st)
{
    if (m.nwc <= 0 || p.order == 2) return hipSuccess;
    const dim3 grid((unsigned)((m.nwc + kRecCells - 1) / kRecCells)), block(kRecThreads);
    if (fp32)
        hipLaunchKernelGGL(wall_recon_vjp_kernel<float>, grid, block, 0, st, m, a, p);
    else
        hipLaunchKernelGGL(wall_recon_vjp_kernel<double>, grid, block, 0, st, m, a, p);
    return hipGetLastError();
}

hipError_t launch_recon_gather(const DevMesh &m, const AdjRecon &a, const Params &p, bool fp32, double *Gout,
                               double *Wout, const double *X1, const double *X2, hipStream_t st)
{
    const dim3 grid((unsigned)((m.nc + kBlock - 1) / kBlock)), block(kBlock);
    if (fp32)
        hipLaunchKernelGGL(recon_gather1_kernel<float>, grid, block, 0, st, m, a, p, Gout);
    else
        hipLaunchKernelGGL(recon_gather1_kernel<double>, grid, block, 0, st, m, a, p, Gout);
    hipLaunchKernelGGL(recon_gather2_kernel, grid, block, 0, st, m, a, Wout, X1, X2);
    return hipGetLastError();
}

}  // namespace gks
