// HIP kernels of the discrete adjoint of one step: the reverse of the cell
// update, of the gas-kinetic flux and of both reconstruction steps, as the
// forward kernels implement them.  Face-to-cell and cell-to-neighbour
// accumulations are fixed-order gathers (each cell reads its four faces, each
// neighbour's contribution through the slot that points back at it), so the
// adjoint is bitwise reproducible.  Adjoint arrays are FP64; the forward
// quantities are recomputed in the bulk type R.
#include "gks_flux_adj.h"
#include "gks_internal.h"
#include "gks_m2stage.h"
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
constexpr int kEqRec = 32;    // values of an EqAdj record
constexpr int kSideRec = 35;  // values of a SideAdj record

// Per Gauss point k of face f: the face frame, both sides' point states in it
// (the slip ghost on a wall face) and the offsets of the polynomial
// evaluations; with ADJ also the adjoints Fob, Wob of the point outputs,
// formed from the cells' adjoints (the transpose of the cell update).
template <typename R, int MODE, bool WALL, bool ADJ>
__device__ __forceinline__ void gp_setup(const DevMesh &m, const AdjFlux &a, int f, int k, double dt_, R T[3][3],
                                         R wl[5], R gl[3][5], R wr[5], R gr[3][5], R off[2][3], R Fob[2][5],
                                         R Wob[2][5])
{
    const int nf = m.nf, n = m.nc;
    const int L = m.fcell[f], Rc = WALL ? L : m.fcell[nf + f];
    const R *fg = static_cast<const R *>(m.fgeo);
    R nrm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        nrm[d] = fg[(size_t)(F_N + d) * nf + f];
        off[0][d] = fg[(size_t)(F_RL + 3 * k + d) * nf + f];
        off[1][d] = off[0][d] + fg[(size_t)(F_D + d) * nf + f];
    }
    rotation(nrm, T);
    const R *coef = static_cast<const R *>(a.coef);
    eval_local(CoefView<R>{coef, n, L}, off[0], T, wl, gl);
    if (WALL)
        slip_ghost(wl, gl, wr, gr);
    else
        eval_local(CoefView<R>{coef, n, Rc}, off[1], T, wr, gr);
    if (!ADJ) return;
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
    // acc0 = w (4 Fh - F1)/dt, acc1 = 4 w (F1 - 2 Fh)/dt^2, acc2 = w W0, acc3 = w W1
    const R w = fg[(size_t)F_AREA * nf + f] * R(1.0 / 3.0);
    const R idt = R(1.0 / dt_);
    R gF1[5], gFh[5], gW0[5], gW1[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        gF1[q] = w * (-accb[0][q] * idt + R(4) * accb[1][q] * (idt * idt));
        gFh[q] = w * (R(4) * accb[0][q] * idt - R(8) * accb[1][q] * (idt * idt));
        gW0[q] = w * accb[2][q];
        gW1[q] = w * accb[3][q];
    }
    to_global_rev(T, gF1, Fob[0]);
    to_global_rev(T, gFh, Fob[1]);
    to_global_rev(T, gW0, Wob[0]);
    to_global_rev(T, gW1, Wob[1]);
}

// Part A, one lane per Gauss point (three per face, 21 faces per wavefront):
// the equilibrium part's reverse, stored per point as an EqAdj record.
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_eq_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? m.nf : m.nfi;
    const int f = f0 + xcd_block_a() * 84 + wave * 21 + slot;
    if (slot >= 21 || f >= f1) return;
    R T[3][3], wl[5], gl[3][5], wr[5], gr[3][5], off[2][3], Fob[2][5], Wob[2][5];
    gp_setup<R, MODE, WALL, true>(m, a, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
    PointFwd<R> P;
    point_forward<R, VISC>(p, R(dt_), wl, wr, P);
    EqAdj<R> E;
    eq_reverse<R, VISC, PRFIX>(p, P, gl, gr, Fob, Wob, E);
    const size_t ng = 3 * (size_t)m.nf, g = 3 * (size_t)f + k;
    double *o = a.EQ + g;
    int t = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) o[(t++) * ng] = double(E.gcb[d][q]);
    o[(t++) * ng] = double(E.gCb.rho);
    o[(t++) * ng] = double(E.gCb.U);
    o[(t++) * ng] = double(E.gCb.V);
    o[(t++) * ng] = double(E.gCb.W);
    o[(t++) * ng] = double(E.gCb.lam);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        o[(t++) * ng] = double(E.cF0b[j]);
        o[(t++) * ng] = double(E.cF1b[j]);
        o[(t++) * ng] = double(E.cWb[j]);
        o[(t++) * ng] = double(E.Ucb[j]);
    }
}

// Part B, one lane per (Gauss point, side) (six per face, 10 faces per
// wavefront): one kinetic side's reverse, stored as a SideAdj record.
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_side_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 6, k = (lane - 6 * slot) >> 1, side = lane & 1;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? m.nf : m.nfi;
    const int f = f0 + xcd_block_a() * 40 + wave * 10 + slot;
    if (slot >= 10 || f >= f1) return;
    R T[3][3], wl[5], gl[3][5], wr[5], gr[3][5], off[2][3], Fob[2][5], Wob[2][5];
    gp_setup<R, MODE, WALL, true>(m, a, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
    PointFwd<R> P;
    point_forward<R, VISC>(p, R(dt_), wl, wr, P);
    const size_t ng = 3 * (size_t)m.nf, g = 3 * (size_t)f + k;
    R gcb[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) gcb[d][q] = R(a.EQ[(size_t)(5 * d + q) * ng + g]);
    SideAdj<R> S;
    side_reverse<R, VISC, PRFIX>(p, P, side == 1, side ? gr : gl, gcb, Fob, Wob, S);
    double *o = a.SB + 2 * g + side;
    const size_t ns = 2 * ng;
    int t = 0;
    o[(t++) * ns] = double(S.gb.rho);
    o[(t++) * ns] = double(S.gb.U);
    o[(t++) * ns] = double(S.gb.V);
    o[(t++) * ns] = double(S.gb.W);
    o[(t++) * ns] = double(S.gb.lam);
    o[(t++) * ns] = double(S.m0b);
    o[(t++) * ns] = double(S.m1b);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) o[(t++) * ns] = double(S.grb[d][q]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        o[(t++) * ns] = double(S.cF0b[j]);
        o[(t++) * ns] = double(S.cF1b[j]);
        o[(t++) * ns] = double(S.cWb[j]);
        o[(t++) * ns] = double(S.Ucb[j]);
    }
    o[(t++) * ns] = double(S.taub);
}

template <typename R>
__device__ __forceinline__ void load_side(const double *SB, size_t ns, size_t idx, SideAdj<R> &S)
{
    const double *o = SB + idx;
    int t = 0;
    S.gb.rho = R(o[(t++) * ns]);
    S.gb.U = R(o[(t++) * ns]);
    S.gb.V = R(o[(t++) * ns]);
    S.gb.W = R(o[(t++) * ns]);
    S.gb.lam = R(o[(t++) * ns]);
    S.m0b = R(o[(t++) * ns]);
    S.m1b = R(o[(t++) * ns]);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) S.grb[d][q] = R(o[(t++) * ns]);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        S.cF0b[j] = R(o[(t++) * ns]);
        S.cF1b[j] = R(o[(t++) * ns]);
        S.cWb[j] = R(o[(t++) * ns]);
        S.Ucb[j] = R(o[(t++) * ns]);
    }
    S.taub = R(o[(t++) * ns]);
}

// Part C, one lane per Gauss point: the common reverse, then the rotation
// back and the polynomial evaluations reversed; the ten coefficient adjoints
// of each side and component are summed over the face's three Gauss points
// in order onto its first lane, which writes them.
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_common_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int nf = m.nf;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? nf : m.nfi;
    const int f = f0 + xcd_block_a() * 84 + wave * 21 + slot;
    const bool live = slot < 21 && f < f1;
    R Wb[2][5], Gb[2][5][3], off[2][3];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Wb[sd][q] = R(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) Gb[sd][q][d] = R(0);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) off[sd][d] = R(0);
    }
    if (live) {
        R T[3][3], wl[5], gl[3][5], wr[5], gr[3][5], Fob[2][5], Wob[2][5];
        gp_setup<R, MODE, WALL, false>(m, a, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
        PointFwd<R> P;
        point_forward<R, VISC>(p, R(dt_), wl, wr, P);
        const size_t ng = 3 * (size_t)nf, g = 3 * (size_t)f + k;
        EqAdj<R> E;
        const double *e = a.EQ + g;
        int t = 15;
        E.gCb.rho = R(e[(t++) * ng]);
        E.gCb.U = R(e[(t++) * ng]);
        E.gCb.V = R(e[(t++) * ng]);
        E.gCb.W = R(e[(t++) * ng]);
        E.gCb.lam = R(e[(t++) * ng]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            E.cF0b[j] = R(e[(t++) * ng]);
            E.cF1b[j] = R(e[(t++) * ng]);
            E.cWb[j] = R(e[(t++) * ng]);
            E.Ucb[j] = R(e[(t++) * ng]);
        }
        SideAdj<R> SL, SR;
        load_side(a.SB, 2 * ng, 2 * g, SL);
        load_side(a.SB, 2 * ng, 2 * g + 1, SR);
        R wlb[5], wrb[5];
        common_reverse<R, VISC>(p, R(dt_), wl, wr, P, E, SL, SR, wlb, wrb);
        if (WALL) {
            // the ghost is a linear function of the left state; its transpose is itself
            R wg[5], gg[3][5];
            slip_ghost(wrb, SR.grb, wg, gg);
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                wlb[q] += wg[q];
                wrb[q] = R(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    SL.grb[d][q] += gg[d][q];
                    SR.grb[d][q] = R(0);
                }
            }
        }
        point_adjoint_global(T, wlb, SL.grb, Wb[0], Gb[0]);
        point_adjoint_global(T, wrb, SR.grb, Wb[1], Gb[1]);
    }
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
            if (live && k == 0 && !(WALL && sd == 1)) {
#pragma unroll
                for (int t = 0; t < 10; ++t) a.CB[(size_t)(50 * sd + 10 * q + t) * nf + f] = double(cb[t]);
            }
        }
}

template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL>
void launch_flux_vjp_parts(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    const int nfaces = WALL ? m.nf - m.nfi : m.nfi;
    if (nfaces <= 0) return;
    const dim3 block(kFluxThreadsA);
    const dim3 g3((unsigned)((nfaces + 83) / 84)), g6((unsigned)((nfaces + 39) / 40));
    hipLaunchKernelGGL((flux_vjp_eq_kernel<R, MODE, VISC, PRFIX, WALL>), g3, block, 0, st, m, a, p, dt);
    hipLaunchKernelGGL((flux_vjp_side_kernel<R, MODE, VISC, PRFIX, WALL>), g6, block, 0, st, m, a, p, dt);
    hipLaunchKernelGGL((flux_vjp_common_kernel<R, MODE, VISC, PRFIX, WALL>), g3, block, 0, st, m, a, p, dt);
}

template <typename R, int MODE, bool WALL>
void launch_flux_vjp_part(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (visc && prfix)
        launch_flux_vjp_parts<R, MODE, true, true, WALL>(m, a, p, dt, st);
    else if (visc)
        launch_flux_vjp_parts<R, MODE, true, false, WALL>(m, a, p, dt, st);
    else if (prfix)
        launch_flux_vjp_parts<R, MODE, false, true, WALL>(m, a, p, dt, st);
    else
        launch_flux_vjp_parts<R, MODE, false, false, WALL>(m, a, p, dt, st);
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
template <typename R>
__global__ __launch_bounds__(kRecThreads) void recon_vjp_kernel(DevMesh m, AdjRecon a, Params p)
{
    __shared__ __align__(16) R sBuf[kM2Chunk * kRecCells];
    const int n = m.nc, nf = m.nf;
    const int q = threadIdx.x / kRecCells;  // component, uniform over the wavefront
    const int l = threadIdx.x % kRecCells;
    const int tb = xcd_block_a();
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
    const int i = xcd_block_a() * kBlock + (int)threadIdx.x;
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
