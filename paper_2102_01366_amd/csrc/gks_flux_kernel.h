// Kernel B of libgks: the gas-kinetic flux (Sec. 2.2) at the three Gauss
// points of each face, for the full distribution of eq. 2nd-flux and its
// smooth-flow form (eq. 2nd-smooth-flux).  Instantiated once per bulk type
// (gks_flux_f64.hip, gks_flux_f32.hip).
#pragma once

#include "gks_device.h"
#include "gks_flux.h"
#include "gks_internal.h"

namespace gks {

template <typename R>
struct DevCoef {
    const R *coef;
    int n, cell;
    __device__ __forceinline__ R operator()(int q, int k) const
    {
        return coef[(size_t)(10 * q + k) * n + cell];
    }
};

// Three lanes per face, one per Gauss point: 21 faces per wavefront (lane 63
// idle).  The lanes of a face are summed in Gauss-point order by shuffles and
// the first lane writes the face.  The kernel holds one wavefront per SIMD
// (its registers), so a block is one wavefront: each SIMD takes the next
// block as soon as its own wavefront ends, instead of waiting for the
// slowest wavefront of a wider block.
#ifndef GKS_FLUX_THREADS
#define GKS_FLUX_THREADS 64
#endif
constexpr int kFluxThreads = GKS_FLUX_THREADS;
// Wavefronts per SIMD the compiler must fit (registers): the Euler flux
// (VISC false) two, at the cost of a 64-byte spill per lane in FP64 (9% faster
// than one wavefront on the walled blast); the Navier-Stokes form one
#ifndef GKS_FLUX_EULER_WAVES
#define GKS_FLUX_EULER_WAVES 2
#endif
template <bool VISC>
constexpr int flux_min_waves() { return VISC ? 1 : GKS_FLUX_EULER_WAVES; }
constexpr int kFacesPerWave = 21;
constexpr int kFacesPerBlock = kFacesPerWave * (kFluxThreads / 64);

// WALL: the launch over the wall faces [nfi, nf) (a ghost on the right, as
// the face's wall tag says), else over interior faces.  CURVED: faces on the
// quadratic path (eq. flux-para-coord-gauss), each Gauss point with its own
// normal and weight, which also write each point's weighted interface values
// for the cell gradients; interior faces [nfc, nfi) or, on a mesh with bent
// edges, the wall faces.  Without CURVED the interior launch covers [0,
// min(nfc, nfi)).  SMOOTH: eq. 2nd-smooth-flux.
// MODE FLUX_DEBUG_RAW (debug exports only) writes |Gamma| sum_k w_k F_k(dt)
// and F_k(dt/2) instead of the fitted flux and its time derivative; each
// mode is a kernel of its own, with one copy of the point routine.
template <typename R, int MODE, bool VISC, bool PRFIX, bool WALL, bool SMOOTH, bool CURVED>
__global__ __launch_bounds__(kFluxThreads, flux_min_waves<VISC>()) void flux_kernel(DevMesh m, DevState s, Params p, double dt_,
                                                                             const double *dtp)
{
    constexpr bool RAW = MODE == FLUX_DEBUG_RAW;
    const int nf = m.nf, n = m.nc;
    const R dt = R(dtp ? *dtp : dt_);
    const R *coef = static_cast<const R *>(s.coef);
    R *FF = static_cast<R *>(s.FF), *FT = static_cast<R *>(s.FT), *FW0 = static_cast<R *>(s.FW0),
      *FWs = static_cast<R *>(s.FWs);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / 3, k = lane - 3 * slot;
    const int nfc = m.nfc < m.nfi ? m.nfc : m.nfi;
    const int f0 = WALL ? m.nfi : (CURVED ? m.nfc : 0), f1 = WALL ? nf : (CURVED ? m.nfi : nfc);
    const int f = f0 + xcd_block() * kFacesPerBlock + wave * kFacesPerWave + slot;
    const bool live = slot < kFacesPerWave && f < f1;
    const int nq = nf - m.nfc, fq = f - m.nfc;  // CURVED: the face's column of cgeo, GC0, GCs
    R acc[4][5];
    if (live) {
        const int L = m.fcell[f], Rc = m.fcell[nf + f];
        const R *fg = static_cast<const R *>(m.fgeo);
        const R *cg = static_cast<const R *>(m.cgeo);
        R nrm[3], dv[3], r[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            nrm[d] = CURVED ? cg[(size_t)(4 * k + d) * nq + fq] : fg[(size_t)(F_N + d) * nf + f];
            dv[d] = fg[(size_t)(F_D + d) * nf + f];
            r[d] = fg[(size_t)(F_RL + 3 * k + d) * nf + f];
        }
        // the point's weight is a third of this area (its area scale on a quadratic face)
        const R area = CURVED ? cg[(size_t)(4 * k + 3) * nq + fq] : fg[(size_t)F_AREA * nf + f];
        WallBC<R> bc{WALL_SLIP, {R(0), R(0), R(0)}};
        if (WALL) {
            const int w = f - m.nfi, nw = nf - m.nfi;
            bc.tag = m.wtag[w];
#pragma unroll
            for (int d = 0; d < 3; ++d) bc.u[d] = static_cast<const R *>(m.wvel)[(size_t)d * nw + w];
        }
        gauss_point_terms<R, VISC, PRFIX, DevCoef<R>, DevCoef<R>, SMOOTH, RAW>(
            p, dt, nrm, area, r, dv, DevCoef<R>{coef, n, L}, DevCoef<R>{coef, n, WALL ? L : Rc}, acc, WALL, &bc);
    } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[a][q] = R(0);
    }
    if constexpr (CURVED) {
        // a quadratic face: each Gauss point's weighted interface values, as
        // FW0 and FWs but per point (row 3q + k), which the cell update
        // multiplies by the point's own normal (eq. gauss-formula)
        if (live) {
            R *GC0 = static_cast<R *>(s.GC0), *GCs = static_cast<R *>(s.GCs);
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                const size_t o = (size_t)(3 * q + k) * nq + fq;
                if (MODE == FLUX_STAGE1) {
                    GC0[o] = acc[2][q];
                    GCs[o] = R(0.5) * (acc[2][q] + acc[3][q]);
                } else if (MODE == FLUX_STAGE2) {
                    GCs[o] = acc[3][q] - acc[2][q];
                } else {
                    GC0[o] = acc[2][q];
                    GCs[o] = acc[3][q];
                }
            }
        }
    }
    // sum the three Gauss points of each face onto its first lane
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const R v1 = __shfl_down(acc[a][q], 1, 64);
            const R v2 = __shfl_down(acc[a][q], 2, 64);
            acc[a][q] = (acc[a][q] + v1) + v2;
        }
    if (!live || k != 0) return;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const size_t o = (size_t)q * nf + f;
        if (MODE == FLUX_STAGE1) {
            FF[o] = acc[0][q];
            FT[o] = acc[1][q];
            FW0[o] = acc[2][q];
            FWs[o] = R(0.5) * (acc[2][q] + acc[3][q]);
        } else if (MODE == FLUX_STAGE2) {
            FT[o] = acc[1][q];
            FWs[o] = acc[3][q] - acc[2][q];
        } else {
            FF[o] = acc[0][q];
            FT[o] = acc[1][q];
            FW0[o] = acc[2][q];
            FWs[o] = acc[3][q];
        }
    }
}

template <typename R, int MODE, bool WALL, bool SMOOTH, bool CURVED>
void launch_flux_part(const DevMesh &m, const DevState &s, const Params &p, double dt, const double *dtp,
                      hipStream_t st)
{
    const int nfc = m.nfc < m.nfi ? m.nfc : m.nfi;
    const int nfaces = WALL ? m.nf - m.nfi : (CURVED ? m.nfi - nfc : nfc);
    if (nfaces <= 0) return;
    const dim3 grid((unsigned)((nfaces + kFacesPerBlock - 1) / kFacesPerBlock)), block(kFluxThreads);
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (visc && prfix)
        hipLaunchKernelGGL((flux_kernel<R, MODE, true, true, WALL, SMOOTH, CURVED>), grid, block, 0, st, m, s, p, dt, dtp);
    else if (visc)
        hipLaunchKernelGGL((flux_kernel<R, MODE, true, false, WALL, SMOOTH, CURVED>), grid, block, 0, st, m, s, p, dt, dtp);
    else if (prfix)
        hipLaunchKernelGGL((flux_kernel<R, MODE, false, true, WALL, SMOOTH, CURVED>), grid, block, 0, st, m, s, p, dt, dtp);
    else
        hipLaunchKernelGGL((flux_kernel<R, MODE, false, false, WALL, SMOOTH, CURVED>), grid, block, 0, st, m, s, p, dt, dtp);
}

template <typename R, int MODE, bool SMOOTH>
void launch_flux_mode(const DevMesh &m, const DevState &s, const Params &p, double dt, const double *dtp,
                      hipStream_t st)
{
    launch_flux_part<R, MODE, false, SMOOTH, false>(m, s, p, dt, dtp, st);
    if (m.nfc < m.nf) {
        // a mesh with bent edges: its quadratic interior faces, then every wall face
        launch_flux_part<R, MODE, false, SMOOTH, true>(m, s, p, dt, dtp, st);
        launch_flux_part<R, MODE, true, SMOOTH, true>(m, s, p, dt, dtp, st);
    } else {
        launch_flux_part<R, MODE, true, SMOOTH, false>(m, s, p, dt, dtp, st);
    }
}

template <typename R, bool SMOOTH>
void launch_flux_kind(const DevMesh &m, const DevState &s, const Params &p, double dt, const double *dtp,
                      int mode, hipStream_t st)
{
    if (mode == FLUX_STAGE1)
        launch_flux_mode<R, FLUX_STAGE1, SMOOTH>(m, s, p, dt, dtp, st);
    else if (mode == FLUX_STAGE2)
        launch_flux_mode<R, FLUX_STAGE2, SMOOTH>(m, s, p, dt, dtp, st);
    else if (mode == FLUX_DEBUG_RAW)
        launch_flux_mode<R, FLUX_DEBUG_RAW, SMOOTH>(m, s, p, dt, dtp, st);
    else
        launch_flux_mode<R, FLUX_DEBUG, SMOOTH>(m, s, p, dt, dtp, st);
}

template <typename R>
hipError_t launch_flux_t(const DevMesh &m, const DevState &s, const Params &p, double dt, const double *dtp,
                         int mode, hipStream_t st)
{
    if (p.flux == FLUX_KIND_SMOOTH)
        launch_flux_kind<R, true>(m, s, p, dt, dtp, mode, st);
    else
        launch_flux_kind<R, false>(m, s, p, dt, dtp, mode, st);
    return hipGetLastError();
}

}  // namespace gks
