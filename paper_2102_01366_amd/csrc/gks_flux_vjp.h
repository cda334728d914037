// Kernels of the discrete adjoint of the flux stage: the reverse of the cell
// update and of the gas-kinetic flux (Sec. 2.2) as kernel B implements it.
// Face-to-cell accumulations are fixed-order gathers, so the adjoint is
// bitwise reproducible.  Adjoint arrays are FP64; the forward quantities are
// recomputed in the bulk type R.  Instantiated once per bulk type
// (gks_adjoint_flux_f64.hip, gks_adjoint_flux_f32.hip).
#pragma once

#include "gks_device.h"
#include "gks_flux_adj.h"
#include "gks_internal.h"

namespace gks {

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
// One wavefront per block, as in the forward flux kernel: these kernels hold
// one or two wavefronts per SIMD, and a SIMD then takes the next block as
// soon as its own wavefront ends.  Per wavefront: 21 faces x 3 Gauss points
// (eq, common), 10 faces x 3 Gauss points x 2 sides (side).
#ifndef GKS_FLUX_THREADS_ADJ
#define GKS_FLUX_THREADS_ADJ 64
#endif
constexpr int kFluxThreadsA = GKS_FLUX_THREADS_ADJ;
constexpr int kWavesA = kFluxThreadsA / 64;
constexpr int kFaces3A = 21 * kWavesA, kFaces6A = 10 * kWavesA;

// Per Gauss point k of face f: the face frame, both sides' point states in it
// (the slip ghost on a wall face) and the offsets of the polynomial
// evaluations; with ADJ also the adjoints Fob, Wob of the point outputs,
// formed from the cells' adjoints (the transpose of the cell update).  A
// quadratic face's point has its own normal and weight in both.
// the wall tag of wall face f and its wall velocity (global frame)
template <typename R>
__device__ __forceinline__ int wall_bc(const DevMesh &m, int f, R u[3])
{
    const int w = f - m.nfi, nw = m.nf - m.nfi;
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = static_cast<const R *>(m.wvel)[(size_t)d * nw + w];
    return m.wtag[w];
}

template <typename R, int MODE, bool WALL, bool ADJ>
__device__ __forceinline__ void gp_setup(const DevMesh &m, const AdjFlux &a, const Params &p, int f, int k, double dt_,
                                         R T[3][3],
                                         R wl[5], R gl[3][5], R wr[5], R gr[3][5], R off[2][3], R Fob[2][5],
                                         R Wob[2][5])
{
    const int nf = m.nf, n = m.nc;
    const int L = m.fcell[f], Rc = WALL ? L : m.fcell[nf + f];
    const R *fg = static_cast<const R *>(m.fgeo);
    // a face on the quadratic path: this Gauss point's own normal and weight
    const bool quad = f >= m.nfc;
    const int nq = nf - m.nfc, fq = f - m.nfc;
    const R *cg = static_cast<const R *>(m.cgeo);
    R nrm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        nrm[d] = quad ? cg[(size_t)(4 * k + d) * nq + fq] : fg[(size_t)(F_N + d) * nf + f];
        off[0][d] = fg[(size_t)(F_RL + 3 * k + d) * nf + f];
        off[1][d] = off[0][d] + fg[(size_t)(F_D + d) * nf + f];
    }
    rotation(nrm, T);
    const R *coef = static_cast<const R *>(a.coef);
    eval_local(CoefView<R>{coef, n, L}, off[0], T, wl, gl);
    if (WALL) {
        R u[3];
        const int tag = wall_bc(m, f, u);
        wall_ghost(p, tag, T, u, wl, gl, wr, gr);
    } else {
        eval_local(CoefView<R>{coef, n, Rc}, off[1], T, wr, gr);
    }
    if (!ADJ) return;
    const double iL = m.geoD[(size_t)G_INVVOL * n + L];
    const double iR = WALL ? 0.0 : m.geoD[(size_t)G_INVVOL * n + Rc];
    double nn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) nn[d] = quad ? m.cnrm[(size_t)(3 * k + d) * nq + fq] : m.fnrm[(size_t)d * nf + f];
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
    const R w = (quad ? cg[(size_t)(4 * k + 3) * nq + fq] : fg[(size_t)F_AREA * nf + f]) * R(1.0 / 3.0);
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
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL, bool SMOOTH>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_eq_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? m.nf : m.nfi;
    const int f = f0 + xcd_block() * kFaces3A + wave * 21 + slot;
    if (slot >= 21 || f >= f1) return;
    R T[3][3], wl[5], gl[3][5], wr[5], gr[3][5], off[2][3], Fob[2][5], Wob[2][5];
    gp_setup<R, MODE, WALL, true>(m, a, p, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
    PointFwd<R> P;
    point_forward<R, VISC, SMOOTH>(p, R(dt_), wl, wr, P);
    EqAdj<R> E;
    eq_reverse<R, VISC, PRFIX, SMOOTH>(p, P, gl, gr, Fob, Wob, E);
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
    o[(t++) * ng] = double(E.taub);
}

// Part B, one lane per (Gauss point, side) (six per face, 10 faces per
// wavefront): one kinetic side's reverse, stored as a SideAdj record.
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL, bool SMOOTH>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_side_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 6, k = (lane - 6 * slot) >> 1, side = lane & 1;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? m.nf : m.nfi;
    const int f = f0 + xcd_block() * kFaces6A + wave * 10 + slot;
    if (slot >= 10 || f >= f1) return;
    R T[3][3], wl[5], gl[3][5], wr[5], gr[3][5], off[2][3], Fob[2][5], Wob[2][5];
    gp_setup<R, MODE, WALL, true>(m, a, p, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
    PointFwd<R> P;
    point_forward<R, VISC, SMOOTH>(p, R(dt_), wl, wr, P);
    const size_t ng = 3 * (size_t)m.nf, g = 3 * (size_t)f + k;
    R gcb[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) gcb[d][q] = R(a.EQ[(size_t)(5 * d + q) * ng + g]);
    SideAdj<R> S;
    side_reverse<R, VISC, PRFIX, SMOOTH>(p, P, side == 1, side ? gr : gl, gcb, Fob, Wob, S);
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
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL, bool SMOOTH>
__global__ __launch_bounds__(kFluxThreadsA) void flux_vjp_common_kernel(DevMesh m, AdjFlux a, Params p, double dt_)
{
    const int nf = m.nf;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int f0 = WALL ? m.nfi : 0, f1 = WALL ? nf : m.nfi;
    const int f = f0 + xcd_block() * kFaces3A + wave * 21 + slot;
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
        gp_setup<R, MODE, WALL, false>(m, a, p, f, k, dt_, T, wl, gl, wr, gr, off, Fob, Wob);
        PointFwd<R> P;
        point_forward<R, VISC, SMOOTH>(p, R(dt_), wl, wr, P);
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
        E.taub = R(e[(t++) * ng]);
        SideAdj<R> SL, SR;
        load_side(a.SB, 2 * ng, 2 * g, SL);
        load_side(a.SB, 2 * ng, 2 * g + 1, SR);
        R wlb[5], wrb[5];
        common_reverse<R, VISC, SMOOTH>(p, R(dt_), wl, wr, P, E, SL, SR, wlb, wrb);
        if (WALL) {
            // the ghost is a function of the left state: its reverse
            R u[3];
            const int tag = wall_bc(m, f, u);
            wall_ghost_rev(p, tag, T, u, wl, gl, wrb, SR.grb, wlb, SL.grb);
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                wrb[q] = R(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) SR.grb[d][q] = R(0);
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

template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL, bool SMOOTH>
void launch_flux_vjp_parts(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    const int nfaces = WALL ? m.nf - m.nfi : m.nfi;
    if (nfaces <= 0) return;
    const dim3 block(kFluxThreadsA);
    const dim3 g3((unsigned)((nfaces + kFaces3A - 1) / kFaces3A)), g6((unsigned)((nfaces + kFaces6A - 1) / kFaces6A));
    hipLaunchKernelGGL((flux_vjp_eq_kernel<R, MODE, VISC, PRFIX, WALL, SMOOTH>), g3, block, 0, st, m, a, p, dt);
    hipLaunchKernelGGL((flux_vjp_side_kernel<R, MODE, VISC, PRFIX, WALL, SMOOTH>), g6, block, 0, st, m, a, p, dt);
    hipLaunchKernelGGL((flux_vjp_common_kernel<R, MODE, VISC, PRFIX, WALL, SMOOTH>), g3, block, 0, st, m, a, p, dt);
}

template <typename R, int MODE, bool WALL, bool SMOOTH>
void launch_flux_vjp_part(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (visc && prfix)
        launch_flux_vjp_parts<R, MODE, true, true, WALL, SMOOTH>(m, a, p, dt, st);
    else if (visc)
        launch_flux_vjp_parts<R, MODE, true, false, WALL, SMOOTH>(m, a, p, dt, st);
    else if (prfix)
        launch_flux_vjp_parts<R, MODE, false, true, WALL, SMOOTH>(m, a, p, dt, st);
    else
        launch_flux_vjp_parts<R, MODE, false, false, WALL, SMOOTH>(m, a, p, dt, st);
}

template <typename R, int MODE>
void launch_flux_vjp_mode(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, hipStream_t st)
{
    if (p.flux == FLUX_KIND_SMOOTH) {
        launch_flux_vjp_part<R, MODE, false, true>(m, a, p, dt, st);
        launch_flux_vjp_part<R, MODE, true, true>(m, a, p, dt, st);
    } else {
        launch_flux_vjp_part<R, MODE, false, false>(m, a, p, dt, st);
        launch_flux_vjp_part<R, MODE, true, false>(m, a, p, dt, st);
    }
}

template <typename R>
hipError_t launch_flux_vjp_t(const DevMesh &m, const AdjFlux &a, const Params &p, double dt, int mode,
                             hipStream_t st)
{
    if (mode == FLUX_ADJ_STAGE1)
        launch_flux_vjp_mode<R, FLUX_ADJ_STAGE1>(m, a, p, dt, st);
    else
        launch_flux_vjp_mode<R, FLUX_ADJ_STAGE2>(m, a, p, dt, st);
    return hipGetLastError();
}

}  // namespace gks
