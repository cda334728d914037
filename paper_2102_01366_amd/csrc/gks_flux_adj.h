// Discrete adjoint of the gas-kinetic flux of gks_flux.h (Sec. 2.2 of Ji,
// Zhao, Shyy & Xu): hand-written reverse mode of every routine there, so that
// the vector-Jacobian product of one Gauss point costs a few forward
// evaluations.  Each *_rev routine takes the forward inputs (it recomputes
// what it needs) and the adjoints of the forward outputs, and ADDS the
// adjoints of the forward inputs into the arrays it is given.  Branches are
// differentiated as taken; d|x|/dx is taken as sign(x) with sign(0) = 0.
#pragma once

#include "gks_flux.h"

namespace gks {

#define GKS_HD __host__ __device__ __forceinline__

// A scheduling fence between the unrolled per-direction blocks of the reverse:
// keeps the scheduler from interleaving them, which would hold several
// directions' temporaries at once (the device pass only).
__host__ __device__ __forceinline__ void sched_fence()
{
#ifdef __HIP_DEVICE_COMPILE__
    __builtin_amdgcn_sched_barrier(0);
#endif
}

// adjoints of a Prim and of a moment table
template <typename R>
struct PrimB {
    R rho, U, V, W, lam;
};
template <typename R>
GKS_HD void zero(PrimB<R> &b)
{
    b.rho = b.U = b.V = b.W = b.lam = R(0);
}
template <typename R>
struct TabB {
    R u[7], v[6], w[6], xi2, xi4;
};
template <typename R>
GKS_HD void zero(TabB<R> &t)
{
#pragma unroll
    for (int k = 0; k < 7; ++k) t.u[k] = R(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) t.v[k] = t.w[k] = R(0);
    t.xi2 = t.xi4 = R(0);
}

template <typename R>
GKS_HD R sign_of(R x)
{
    return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

// rho = w0, U = w_{1..3} / w0, lam = (K+3) w0 / (4 D), D = w4 - |w_{1..3}|^2 / (2 w0)
template <typename R>
GKS_HD void primitive_rev(const R w[5], R K, const PrimB<R> &gb, R wb[5])
{
    const R ir = R(1) / w[0];
    const R U = w[1] * ir, V = w[2] * ir, W = w[3] * ir;
    const R q = U * U + V * V + W * W;
    const R D = w[4] - R(0.5) * w[0] * q;
    const R lam = (K + R(3)) * w[0] / (R(4) * D);
    const R lD = lam / D;
    wb[0] += gb.rho + gb.lam * (lam * ir - lD * R(0.5) * q) - (gb.U * U + gb.V * V + gb.W * W) * ir;
    wb[1] += gb.U * ir + gb.lam * lD * U;
    wb[2] += gb.V * ir + gb.lam * lD * V;
    wb[3] += gb.W * ir + gb.lam * lD * W;
    wb[4] -= gb.lam * lD;
}

// Reverse of m[k+2] = U m[k+1] + (k+1) h m[k], h = 1/(2 lam), k = N-3..0;
// leaves the adjoints of the seeds m[0], m[1] in mb[0], mb[1].
template <int N, typename R>
GKS_HD void recursion_rev(R U, R lam, const R *m, R *mb, R &Ub, R &lamb)
{
    const R h = R(0.5) / lam;
    R hb = R(0);
#pragma unroll
    for (int k = N - 3; k >= 0; --k) {
        const R t = mb[k + 2];
        Ub += t * m[k + 1];
        mb[k + 1] += t * U;
        hb += t * R(k + 1) * m[k];
        mb[k] += t * (R(k + 1) * h);
    }
    lamb -= hb * h / lam;
}

// full-line moments: m[0] = 1, m[1] = U
template <int N, typename R>
GKS_HD void gauss_moments_rev(R U, R lam, const R *m, R *mb, R &Ub, R &lamb)
{
    recursion_rev<N>(U, lam, m, mb, Ub, lamb);
    Ub += mb[1];
}

template <typename R>
GKS_HD void vw_tables_rev(const Prim<R> &g, R K, const Tab<R> &t, TabB<R> &tb, PrimB<R> &gb)
{
    R vb[6], wb[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        vb[k] = tb.v[k];
        wb[k] = tb.w[k];
    }
    gauss_moments_rev<6>(g.V, g.lam, t.v, vb, gb.V, gb.lam);
    gauss_moments_rev<6>(g.W, g.lam, t.w, wb, gb.W, gb.lam);
    // xi2 = K / (2 lam), xi4 = K (K+2) / (4 lam^2)
    gb.lam -= tb.xi2 * t.xi2 * g.ilam + tb.xi4 * R(2) * t.xi4 * g.ilam;
}

template <int A, int B, int C, typename R>
GKS_HD void psi_mom_rev(const Tab<R> &T, const R tb[5], TabB<R> &Tb)
{
    const R *u = T.u, *v = T.v, *w = T.w;
    const R s4 = R(0.5) * tb[4];
    const R mb = tb[0] + s4 * T.xi2;
    Tb.xi2 += s4 * (u[A] * v[B] * w[C]);
    Tb.u[A] += mb * v[B] * w[C];
    Tb.v[B] += mb * u[A] * w[C];
    Tb.w[C] += mb * u[A] * v[B];
    Tb.u[A + 1] += tb[1] * v[B] * w[C];
    Tb.v[B] += tb[1] * u[A + 1] * w[C];
    Tb.w[C] += tb[1] * u[A + 1] * v[B];
    Tb.u[A] += tb[2] * v[B + 1] * w[C];
    Tb.v[B + 1] += tb[2] * u[A] * w[C];
    Tb.w[C] += tb[2] * u[A] * v[B + 1];
    Tb.u[A] += tb[3] * v[B] * w[C + 1];
    Tb.v[B] += tb[3] * u[A] * w[C + 1];
    Tb.w[C + 1] += tb[3] * u[A] * v[B];
    Tb.u[A + 2] += s4 * v[B] * w[C];
    Tb.v[B] += s4 * u[A + 2] * w[C];
    Tb.w[C] += s4 * u[A + 2] * v[B];
    Tb.u[A] += s4 * v[B + 2] * w[C];
    Tb.v[B + 2] += s4 * u[A] * w[C];
    Tb.w[C] += s4 * u[A] * v[B + 2];
    Tb.u[A] += s4 * v[B] * w[C + 2];
    Tb.v[B] += s4 * u[A] * w[C + 2];
    Tb.w[C + 2] += s4 * u[A] * v[B];
}

// Reverse of contract<A,B,C>: out += s <u^A v^B w^C (a.psi) psi>.  Adds the
// adjoints of the table (Tb), of a (ab) and of s (sb).
template <int A, int B, int C, typename R>
GKS_HD void contract_rev_split(const Tab<R> &T, const R a[5], R s, const R outb[5], R *ub, TabB<R> &Tb,
                               R ab[5], R &sb);

template <int A, int B, int C, typename R>
GKS_HD void contract_rev(const Tab<R> &T, const R a[5], R s, const R outb[5], TabB<R> &Tb, R ab[5],
                         R &sb)
{
    contract_rev_split<A, B, C>(T, a, s, outb, Tb.u, Tb, ab, sb);
}

// The same with the adjoints of the u table in ub (so that a table sharing
// its v, w and xi entries with another can keep a u-adjoint of its own).
template <int A, int B, int C, typename R>
GKS_HD void contract_rev_split(const Tab<R> &T, const R a[5], R s, const R outb[5], R *ub, TabB<R> &Tb,
                               R ab[5], R &sb)
{
    const R *U = T.u, *V = T.v, *W = T.w;
    // forward values
    const R h = R(0.5) * a[4];
    const R c0 = a[0] + h * T.xi2;
    const R P0 = c0 * U[A] + a[1] * U[A + 1] + h * U[A + 2];
    const R P1 = c0 * U[A + 1] + a[1] * U[A + 2] + h * U[A + 3];
    const R P2 = c0 * U[A + 2] + a[1] * U[A + 3] + h * U[A + 4];
    // VW(i, j) = V[B+i] W[C+j]
    R VW[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j + i < 5; ++j) VW[i][j] = V[B + i] * W[C + j];
    const R X00 = a[2] * VW[1][0] + a[3] * VW[0][1] + h * (VW[2][0] + VW[0][2]);
    const R X10 = a[2] * VW[2][0] + a[3] * VW[1][1] + h * (VW[3][0] + VW[1][2]);
    const R X01 = a[2] * VW[1][1] + a[3] * VW[0][2] + h * (VW[2][1] + VW[0][3]);
    const R X20 = a[2] * VW[3][0] + a[3] * VW[2][1] + h * (VW[4][0] + VW[2][2]);
    const R X02 = a[2] * VW[1][2] + a[3] * VW[0][3] + h * (VW[2][2] + VW[0][4]);
    const R S000 = P0 * VW[0][0] + U[A] * X00;
    const R S100 = P1 * VW[0][0] + U[A + 1] * X00;
    const R S010 = P0 * VW[1][0] + U[A] * X10;
    const R S001 = P0 * VW[0][1] + U[A] * X01;
    const R S200 = P2 * VW[0][0] + U[A + 2] * X00;
    const R S020 = P0 * VW[2][0] + U[A] * X20;
    const R S002 = P0 * VW[0][2] + U[A] * X02;
    const R dx = T.xi4 - T.xi2 * T.xi2;
    const R Sxi = T.xi2 * S000 + h * dx * (U[A] * VW[0][0]);
    sb += outb[0] * S000 + outb[1] * S100 + outb[2] * S010 + outb[3] * S001 +
          R(0.5) * outb[4] * (S200 + S020 + S002 + Sxi);
    // adjoints of the S terms
    const R q = R(0.5) * s * outb[4];
    R S000b = s * outb[0];
    const R S100b = s * outb[1], S010b = s * outb[2], S001b = s * outb[3];
    const R S200b = q, S020b = q, S002b = q, Sxib = q;
    R VWb[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j + i < 5; ++j) VWb[i][j] = R(0);
    R Ub[5] = {R(0), R(0), R(0), R(0), R(0)};  // adjoints of U[A..A+4]
    R hb = R(0);
    // Sxi
    S000b += T.xi2 * Sxib;
    Tb.xi2 += Sxib * (S000 - R(2) * h * T.xi2 * (U[A] * VW[0][0]));
    Tb.xi4 += Sxib * h * (U[A] * VW[0][0]);
    hb += Sxib * dx * (U[A] * VW[0][0]);
    Ub[0] += Sxib * h * dx * VW[0][0];
    VWb[0][0] += Sxib * h * dx * U[A];
    // S terms: S = P VW + U X
    R P0b = S000b * VW[0][0] + S010b * VW[1][0] + S001b * VW[0][1] + S020b * VW[2][0] + S002b * VW[0][2];
    const R P1b = S100b * VW[0][0];
    const R P2b = S200b * VW[0][0];
    VWb[0][0] += S000b * P0 + S100b * P1 + S200b * P2;
    VWb[1][0] += S010b * P0;
    VWb[0][1] += S001b * P0;
    VWb[2][0] += S020b * P0;
    VWb[0][2] += S002b * P0;
    const R X00b = S000b * U[A] + S100b * U[A + 1] + S200b * U[A + 2];
    const R X10b = S010b * U[A], X01b = S001b * U[A], X20b = S020b * U[A], X02b = S002b * U[A];
    Ub[0] += S000b * X00 + S010b * X10 + S001b * X01 + S020b * X20 + S002b * X02;
    Ub[1] += S100b * X00;
    Ub[2] += S200b * X00;
    // X terms
    ab[2] += X00b * VW[1][0] + X10b * VW[2][0] + X01b * VW[1][1] + X20b * VW[3][0] + X02b * VW[1][2];
    ab[3] += X00b * VW[0][1] + X10b * VW[1][1] + X01b * VW[0][2] + X20b * VW[2][1] + X02b * VW[0][3];
    hb += X00b * (VW[2][0] + VW[0][2]) + X10b * (VW[3][0] + VW[1][2]) + X01b * (VW[2][1] + VW[0][3]) +
          X20b * (VW[4][0] + VW[2][2]) + X02b * (VW[2][2] + VW[0][4]);
    VWb[1][0] += X00b * a[2];
    VWb[0][1] += X00b * a[3];
    VWb[2][0] += X00b * h + X10b * a[2];
    VWb[0][2] += X00b * h + X01b * a[3];
    VWb[1][1] += X10b * a[3] + X01b * a[2];
    VWb[3][0] += X10b * h + X20b * a[2];
    VWb[1][2] += X10b * h + X02b * a[2];
    VWb[2][1] += X01b * h + X20b * a[3];
    VWb[0][3] += X01b * h + X02b * a[3];
    VWb[4][0] += X20b * h;
    VWb[2][2] += X20b * h + X02b * h;
    VWb[0][4] += X02b * h;
    // P terms: P_k = c0 U[A+k] + a1 U[A+k+1] + h U[A+k+2]
    const R c0b = P0b * U[A] + P1b * U[A + 1] + P2b * U[A + 2];
    ab[1] += P0b * U[A + 1] + P1b * U[A + 2] + P2b * U[A + 3];
    hb += P0b * U[A + 2] + P1b * U[A + 3] + P2b * U[A + 4];
    Ub[0] += P0b * c0;
    Ub[1] += P0b * a[1] + P1b * c0;
    Ub[2] += P0b * h + P1b * a[1] + P2b * c0;
    Ub[3] += P1b * h + P2b * a[1];
    Ub[4] += P2b * h;
    // c0 = a0 + h xi2, h = a4 / 2
    ab[0] += c0b;
    hb += c0b * T.xi2;
    Tb.xi2 += c0b * h;
    ab[4] += R(0.5) * hb;
#pragma unroll
    for (int k = 0; k < 5; ++k) ub[A + k] += Ub[k];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = 0; j + i < 5; ++j) {
            Tb.v[B + i] += VWb[i][j] * W[C + j];
            Tb.w[C + j] += VWb[i][j] * V[B + i];
        }
}

// Reverse of micro_slope: a = M(g) b.  Adds to gb and bb.
template <typename R>
GKS_HD void micro_slope_rev(const Prim<R> &g, R K, const R b[5], const R abar[5], PrimB<R> &gb, R bb[5])
{
    const R U = g.U, V = g.V, W = g.W, lam = g.lam;
    const R q2 = U * U + V * V + W * W + (K + R(3)) / (R(2) * lam);
    const R R1 = b[1] - U * b[0], R2 = b[2] - V * b[0], R3 = b[3] - W * b[0];
    const R R4 = R(2) * b[4] - q2 * b[0];
    const R c = R(4) * lam * lam / (K + R(3));
    const R X = R4 - R(2) * U * R1 - R(2) * V * R2 - R(2) * W * R3;
    const R a4 = c * X;
    const R a1 = R(2) * lam * R1 - U * a4;
    const R a2 = R(2) * lam * R2 - V * a4;
    const R a3 = R(2) * lam * R3 - W * a4;
    R a1b = abar[1], a2b = abar[2], a3b = abar[3], a4b = abar[4];
    const R a0b = abar[0];
    R Ub = R(0), Vb = R(0), Wb = R(0), lamb = R(0), q2b = R(0);
    // a0 = b0 - U a1 - V a2 - W a3 - a4 q2 / 2
    bb[0] += a0b;
    Ub -= a0b * a1;
    a1b -= a0b * U;
    Vb -= a0b * a2;
    a2b -= a0b * V;
    Wb -= a0b * a3;
    a3b -= a0b * W;
    a4b -= R(0.5) * a0b * q2;
    q2b -= R(0.5) * a0b * a4;
    // a_k = 2 lam R_k - U_k a4
    R R1b = R(2) * lam * a1b, R2b = R(2) * lam * a2b, R3b = R(2) * lam * a3b;
    lamb += R(2) * (a1b * R1 + a2b * R2 + a3b * R3);
    Ub -= a1b * a4;
    Vb -= a2b * a4;
    Wb -= a3b * a4;
    a4b -= a1b * U + a2b * V + a3b * W;
    // a4 = c X
    const R Xb = a4b * c;
    lamb += a4b * X * R(8) * lam / (K + R(3));
    const R R4b = Xb;
    Ub -= R(2) * Xb * R1;
    R1b -= R(2) * Xb * U;
    Vb -= R(2) * Xb * R2;
    R2b -= R(2) * Xb * V;
    Wb -= R(2) * Xb * R3;
    R3b -= R(2) * Xb * W;
    // R4 = 2 b4 - q2 b0; R_k = b_k - U_k b0
    bb[4] += R(2) * R4b;
    q2b -= R4b * b[0];
    bb[0] -= R4b * q2 + R1b * U + R2b * V + R3b * W;
    bb[1] += R1b;
    bb[2] += R2b;
    bb[3] += R3b;
    Ub -= R1b * b[0];
    Vb -= R2b * b[0];
    Wb -= R3b * b[0];
    // q2 = |U|^2 + (K+3) / (2 lam)
    Ub += R(2) * U * q2b;
    Vb += R(2) * V * q2b;
    Wb += R(2) * W * q2b;
    lamb -= q2b * (K + R(3)) / (R(2) * lam * lam);
    gb.U += Ub;
    gb.V += Vb;
    gb.W += Wb;
    gb.lam += lamb;
}

template <typename R>
GKS_HD void heat_moment_rev(const R Uc[3], const R F[5], const R V[5], R hb, R Ucb[3], R Fb[5], R Vb[5])
{
    const R U = Uc[0], Vv = Uc[1], W = Uc[2], U2 = U * U + Vv * Vv + W * W;
    Fb[4] += hb;
    Fb[1] -= hb * U;
    Fb[2] -= hb * Vv;
    Fb[3] -= hb * W;
    Fb[0] += hb * (R(0.5) * U2 + U * U);
    Vb[4] -= hb * U;
    Vb[2] += hb * U * Vv;
    Vb[3] += hb * U * W;
    Vb[0] -= hb * R(0.5) * U * U2;
    Ucb[0] += hb * (-F[1] + R(3) * U * F[0] - V[4] + Vv * V[2] + W * V[3] - R(0.5) * U2 * V[0] - U * U * V[0]);
    Ucb[1] += hb * (-F[2] + Vv * F[0] + U * V[2] - U * Vv * V[0]);
    Ucb[2] += hb * (-F[3] + W * F[0] + U * V[3] - U * W * V[0]);
}

// adjoint of a TimeCoef (tau included: the kinetic parts use it in cW0)
template <typename R>
struct TimeCoefB {
    R tau, cF[2][6], cW[6];
};
template <typename R>
GKS_HD void zero(TimeCoefB<R> &t)
{
    t.tau = R(0);
#pragma unroll
    for (int k = 0; k < 6; ++k) t.cF[0][k] = t.cF[1][k] = t.cW[k] = R(0);
}

template <typename R, bool VISC>
GKS_HD void time_coefficients_rev(R tau, R taun, R dt, const TimeCoefB<R> &tb, R &taub, R &taunb)
{
    taub += tb.tau;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const R del = k == 0 ? dt : R(0.5) * dt;
        const R e = exp(-del / taun);
        const R E1 = taun * (R(1) - e);
        const R *c = tb.cF[k];
        R E1b, E2b;
        if (VISC) {
            E1b = -c[0] + tau * c[1] + tau * c[2] + c[3] - tau * c[4] - tau * c[5];
            E2b = c[1] - c[4];
            taub += c[1] * (E1 - del) + c[2] * (E1 - del) - c[4] * E1 - c[5] * E1;
        } else {
            E1b = -c[0] + c[3];
            E2b = c[1] - c[4];
        }
        // E1 = taun (1 - e), E2 = taun^2 (1 - e) - taun del e, e = exp(-del / taun)
        taunb += E1b * (R(1) - e) + E2b * (R(2) * taun * (R(1) - e) - del * e);
        const R eb = -E1b * taun - E2b * (taun * taun + taun * del);
        taunb += eb * e * del / (taun * taun);
    }
    const R et = exp(-dt / taun);
    const R *c = tb.cW;
    R etb = -c[0] + c[3];
    if (VISC) {
        etb += c[1] * (dt + tau) + c[2] * tau - c[4] * (tau + dt) - c[5] * tau;
        taub += c[1] * (et - R(1)) + c[2] * (et - R(1)) - c[4] * et - c[5] * et;
    } else {
        etb += dt * c[1] - dt * c[4];
    }
    taunb += etb * et * dt / (taun * taun);
}

// Reverse of add_part.  cF0b .. cW1b, Fb, Vb, Ucb, rhob are added to.
template <typename R, bool PRFIX>
GKS_HD void add_part_rev(const Params &p, R rho, const R *cF0, const R *cF1, const R *cW0, const R *cW1,
                         const R F[3][5], const R V[3][5], const R Uc[3], const R Fob[2][5],
                         const R Wob[2][5], R &rhob, R *cF0b, R *cF1b, R *cW0b, R *cW1b, R Fb[3][5],
                         R Vb[3][5], R Ucb[3])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const R f0 = cF0[0] * F[0][q] + cF0[1] * F[1][q] + cF0[2] * F[2][q];
        const R f1 = cF1[0] * F[0][q] + cF1[1] * F[1][q] + cF1[2] * F[2][q];
        const R w0 = cW0[0] * V[0][q] + cW0[1] * V[1][q] + cW0[2] * V[2][q];
        const R w1 = cW1[0] * V[0][q] + cW1[1] * V[1][q] + cW1[2] * V[2][q];
        rhob += Fob[0][q] * f0 + Fob[1][q] * f1 + Wob[0][q] * w0 + Wob[1][q] * w1;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Fb[j][q] += rho * (Fob[0][q] * cF0[j] + Fob[1][q] * cF1[j]);
            Vb[j][q] += rho * (Wob[0][q] * cW0[j] + Wob[1][q] * cW1[j]);
            cF0b[j] += rho * Fob[0][q] * F[j][q];
            cF1b[j] += rho * Fob[1][q] * F[j][q];
            cW0b[j] += rho * Wob[0][q] * V[j][q];
            cW1b[j] += rho * Wob[1][q] * V[j][q];
        }
    }
    if (PRFIX) {
        const R fac = R(1.0 / p.prandtl - 1.0);
        R hv[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) hv[j] = heat_moment(Uc, F[j], V[j]);
        rhob += fac * (Fob[0][4] * (cF0[0] * hv[0] + cF0[1] * hv[1] + cF0[2] * hv[2]) +
                       Fob[1][4] * (cF1[0] * hv[0] + cF1[1] * hv[1] + cF1[2] * hv[2]));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cF0b[j] += fac * rho * Fob[0][4] * hv[j];
            cF1b[j] += fac * rho * Fob[1][4] * hv[j];
            const R hb = fac * rho * (Fob[0][4] * cF0[j] + Fob[1][4] * cF1[j]);
            heat_moment_rev(Uc, F[j], V[j], hb, Ucb, Fb[j], Vb[j]);
        }
    }
}

// Forward values of one side's kinetic part (the quantities side_terms forms),
// kept for its reverse.
template <typename R>
struct SideFwd {
    Tab<R> Th, Tf;
    R a[3][5], B[5], A[5], F[3][5], V[3][5];
};

// The direction-d contractions of side_terms: F[1] += <u u_d (a.psi) psi>,
// V[1] += <u_d (a.psi) psi>, B -= <u_d (a.psi) psi> over the full line.
// SMOOTH (eq. 2nd-smooth-flux): only the tables and the share of g^c_x.
template <typename R, bool VISC, bool SMOOTH = false>
GKS_HD void side_forward(const Params &p, const Prim<R> &g, R m0, R m1, const R gr[3][5], SideFwd<R> &S,
                         R gc[3][5])
{
    const R K = R(p.K);
    {
        const R h = R(0.5) * g.ilam;
        S.Th.u[0] = m0;
        S.Th.u[1] = m1;
#pragma unroll
        for (int k = 0; k + 2 < 7; ++k) S.Th.u[k + 2] = g.U * S.Th.u[k + 1] + R(k + 1) * h * S.Th.u[k];
    }
    vw_tables(g, K, S.Th);
    if constexpr (SMOOTH) {
        const R ir = g.ir;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R b[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
            micro_slope(g, K, b, S.a[d]);
            contract<0, 0, 0>(S.Th, S.a[d], g.rho, gc[d]);
        }
        return;
    }
    psi_mom<1, 0, 0>(S.Th, S.F[0]);
    psi_mom<0, 0, 0>(S.Th, S.V[0]);
#pragma unroll
    for (int q = 0; q < 5; ++q) S.F[1][q] = S.V[1][q] = S.F[2][q] = S.V[2][q] = S.B[q] = S.A[q] = R(0);
    if (VISC) {
        gauss_moments_h<7>(g.U, R(0.5) * g.ilam, S.Tf.u);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            S.Tf.v[k] = S.Th.v[k];
            S.Tf.w[k] = S.Th.w[k];
        }
        S.Tf.xi2 = S.Th.xi2;
        S.Tf.xi4 = S.Th.xi4;
    }
    const R ir = g.ir;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
        micro_slope(g, K, b, S.a[d]);
        contract<0, 0, 0>(S.Th, S.a[d], g.rho, gc[d]);
        if (d == 0) {
            contract<2, 0, 0>(S.Th, S.a[d], R(1), S.F[1]);
            contract<1, 0, 0>(S.Th, S.a[d], R(1), S.V[1]);
            if (VISC) contract<1, 0, 0>(S.Tf, S.a[d], R(-1), S.B);
        } else if (d == 1) {
            contract<1, 1, 0>(S.Th, S.a[d], R(1), S.F[1]);
            contract<0, 1, 0>(S.Th, S.a[d], R(1), S.V[1]);
            if (VISC) contract<0, 1, 0>(S.Tf, S.a[d], R(-1), S.B);
        } else {
            contract<1, 0, 1>(S.Th, S.a[d], R(1), S.F[1]);
            contract<0, 0, 1>(S.Th, S.a[d], R(1), S.V[1]);
            if (VISC) contract<0, 0, 1>(S.Tf, S.a[d], R(-1), S.B);
        }
        sched_fence();
    }
    if (VISC) {
        micro_slope(g, K, S.B, S.A);
        contract<1, 0, 0>(S.Th, S.A, R(1), S.F[2]);
        contract<0, 0, 0>(S.Th, S.A, R(1), S.V[2]);
    }
}

// Reverse of side_terms.  gcb: adjoint of the side's share of g^c_x (from the
// equilibrium part).  Adds to gb, m0b, m1b, grb, tcb, Ucb.  SMOOTH: the side
// enters only through that share.
template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void side_terms_rev(const Params &p, const Prim<R> &g, R m0, R m1, const R gr[3][5],
                           const TimeCoef<R> &tc, const R Uc[3], const R gcb[3][5], const R Fob[2][5],
                           const R Wob[2][5], PrimB<R> &gb, R &m0b, R &m1b, R grb[3][5],
                           TimeCoefB<R> &tcb, R Ucb[3])
{
    const R K = R(p.K);
    SideFwd<R> S;
    {
        R gcs[3][5];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 5; ++q) gcs[d][q] = R(0);
        side_forward<R, VISC, SMOOTH>(p, g, m0, m1, gr, S, gcs);
    }
    R Fb[3][5], Vb[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 5; ++q) Fb[j][q] = Vb[j][q] = R(0);
    R rhob = R(0);
    if constexpr (!SMOOTH) {
        R cW0b[3] = {R(0), R(0), R(0)};
        const R cW0[3] = {R(1), -tc.tau, -tc.tau};
        add_part_rev<R, PRFIX>(p, g.rho, tc.cF[0] + 3, tc.cF[1] + 3, cW0, tc.cW + 3, S.F, S.V, Uc, Fob, Wob,
                               rhob, tcb.cF[0] + 3, tcb.cF[1] + 3, cW0b, tcb.cW + 3, Fb, Vb, Ucb);
        tcb.tau -= cW0b[1] + cW0b[2];
    }
    sched_fence();
    TabB<R> Thb;
    zero(Thb);
    // the full-line table shares v, w and xi with the half-line one: only its
    // u entries need an adjoint of their own
    R Tfub[7] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    R dummy = R(0);
    if constexpr (!SMOOTH) {
        psi_mom_rev<0, 0, 0>(S.Th, Vb[0], Thb);
        psi_mom_rev<1, 0, 0>(S.Th, Fb[0], Thb);
    }
    constexpr bool KIN_VISC = VISC && !SMOOTH;
    R Bb[5] = {R(0), R(0), R(0), R(0), R(0)};
    if (KIN_VISC) {
        R Ab[5] = {R(0), R(0), R(0), R(0), R(0)};
        contract_rev<0, 0, 0>(S.Th, S.A, R(1), Vb[2], Thb, Ab, dummy);
        contract_rev<1, 0, 0>(S.Th, S.A, R(1), Fb[2], Thb, Ab, dummy);
        micro_slope_rev(g, K, S.B, Ab, gb, Bb);
    }
    sched_fence();
    const R ir = g.ir;
    R irb = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // the slopes a_d recomputed rather than kept
        R b[5], a[5], ab[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
        micro_slope(g, K, b, a);
        if constexpr (!SMOOTH) {
            if (d == 0) {
                if (KIN_VISC) contract_rev_split<1, 0, 0>(S.Tf, a, R(-1), Bb, Tfub, Thb, ab, dummy);
                contract_rev<2, 0, 0>(S.Th, a, R(1), Fb[1], Thb, ab, dummy);
                contract_rev<1, 0, 0>(S.Th, a, R(1), Vb[1], Thb, ab, dummy);
            } else if (d == 1) {
                if (KIN_VISC) contract_rev_split<0, 1, 0>(S.Tf, a, R(-1), Bb, Tfub, Thb, ab, dummy);
                contract_rev<1, 1, 0>(S.Th, a, R(1), Fb[1], Thb, ab, dummy);
                contract_rev<0, 1, 0>(S.Th, a, R(1), Vb[1], Thb, ab, dummy);
            } else {
                if (KIN_VISC) contract_rev_split<0, 0, 1>(S.Tf, a, R(-1), Bb, Tfub, Thb, ab, dummy);
                contract_rev<1, 0, 1>(S.Th, a, R(1), Fb[1], Thb, ab, dummy);
                contract_rev<0, 0, 1>(S.Th, a, R(1), Vb[1], Thb, ab, dummy);
            }
        }
        contract_rev<0, 0, 0>(S.Th, a, g.rho, gcb[d], Thb, ab, rhob);
        R bb[5] = {R(0), R(0), R(0), R(0), R(0)};
        micro_slope_rev(g, K, b, ab, gb, bb);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            grb[d][q] += bb[q] * ir;
            irb += bb[q] * gr[d][q];
        }
        sched_fence();
    }
    rhob -= irb * ir * ir;
    if (KIN_VISC) gauss_moments_rev<7>(g.U, g.lam, S.Tf.u, Tfub, gb.U, gb.lam);
    vw_tables_rev(g, K, S.Th, Thb, gb);
    recursion_rev<7>(g.U, g.lam, S.Th.u, Thb.u, gb.U, gb.lam);
    m0b += Thb.u[0];
    m1b += Thb.u[1];
    gb.rho += rhob;
}

// The reverse of gks_point in four parts, so that a kernel can hold one
// part's working set at a time:
//   point_forward      the forward quantities that depend on the two point
//                      states only (primitive variables, half-line seeds, W^c,
//                      collision times, time coefficients);
//   eq_reverse         the equilibrium part's reverse, which also yields the
//                      adjoint of g^c_x (the kinetic slopes' contribution);
//   side_reverse       one kinetic side's reverse;
//   common_reverse     the reverse of the point_forward quantities.
template <typename R>
struct PointFwd {
    Prim<R> gL, gR, gC;
    R l0, l1, r0, r1, el, er;
    R Wc[5], Uc[3];
    R pl, pr, pc, z, tau, taun;
    TimeCoef<R> tc;
};

template <typename R, bool VISC, bool SMOOTH = false>
GKS_HD void point_forward(const Params &p, R dt, const R wl[5], const R wr[5], PointFwd<R> &P)
{
    const R K = R(p.K);
    P.gL = primitive(wl, K);
    P.gR = primitive(wr, K);
    const Prim<R> &gL = P.gL, &gR = P.gR;
    const R sl = sqrt(gL.lam), sr = sqrt(gR.lam);
    P.el = exp(-gL.lam * gL.U * gL.U) * (sqrt(R(M_PI) * gL.lam) * gL.ilam) * R(0.5 / M_PI);
    P.er = exp(-gR.lam * gR.U * gR.U) * (sqrt(R(M_PI) * gR.lam) * gR.ilam) * R(0.5 / M_PI);
    P.l0 = R(0.5) * erfc(-sl * gL.U);
    P.l1 = gL.U * P.l0 + P.el;
    P.r0 = R(0.5) * erfc(sr * gR.U);
    P.r1 = gR.U * P.r0 - P.er;
    const R hl = R(0.5) * gL.ilam, hr = R(0.5) * gR.ilam;
    const R l2 = gL.U * P.l1 + hl * P.l0, r2 = gR.U * P.r1 + hr * P.r0;
    const R tl = gL.V * gL.V + gL.W * gL.W + (R(2) + K) * hl;
    const R tr = gR.V * gR.V + gR.W * gR.W + (R(2) + K) * hr;
    P.Wc[0] = gL.rho * P.l0 + gR.rho * P.r0;
    P.Wc[1] = gL.rho * P.l1 + gR.rho * P.r1;
    P.Wc[2] = gL.rho * (gL.V * P.l0) + gR.rho * (gR.V * P.r0);
    P.Wc[3] = gL.rho * (gL.W * P.l0) + gR.rho * (gR.W * P.r0);
    P.Wc[4] = gL.rho * (R(0.5) * (l2 + P.l0 * tl)) + gR.rho * (R(0.5) * (r2 + P.r0 * tr));
    P.gC = primitive(P.Wc, K);
    P.Uc[0] = P.gC.U;
    P.Uc[1] = P.gC.V;
    P.Uc[2] = P.gC.W;
    P.pl = gL.rho * R(0.5) * gL.ilam;
    P.pr = gR.rho * R(0.5) * gR.ilam;
    P.pc = P.gC.rho * R(0.5) / P.gC.lam;
    P.z = (P.pl - P.pr) / (P.pl + P.pr);
    if constexpr (SMOOTH) {
        P.tau = VISC ? R(p.mu) / P.pc : R(0);
        P.taun = R(0);  // not used by eq. 2nd-smooth-flux
        time_coefficients_smooth<R>(P.tau, dt, P.tc);
        return;
    }
    const R jump = R(p.c_tau) * fabs(P.z) * dt;
    if (VISC) {
        P.tau = R(p.mu) / P.pc;
        P.taun = P.tau + jump;
    } else {
        P.tau = R(0);
        P.taun = R(p.eps_tau) * dt + jump;
    }
    time_coefficients<R, VISC>(P.tau, P.taun, dt, P.tc);
}

// adjoints produced by the equilibrium part
template <typename R>
struct EqAdj {
    R gcb[3][5];            // g^c_x (from both sides' slopes)
    PrimB<R> gCb;           // primitive variables of W^c (partial)
    R cF0b[3], cF1b[3], cWb[3];  // equilibrium time coefficients
    R Ucb[3];
    R taub;                 // tau through the equilibrium part's W(0) (eq. 2nd-smooth-flux only)
};

// adjoints produced by one kinetic side
template <typename R>
struct SideAdj {
    PrimB<R> gb;            // the side's primitive variables (partial)
    R m0b, m1b;             // its half-line seeds
    R grb[3][5];            // its point gradient (face frame)
    R cF0b[3], cF1b[3], cWb[3], taub;  // kinetic time coefficients, tau (in W(0))
    R Ucb[3];
};

template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void eq_reverse(const Params &p, const PointFwd<R> &P, const R gl[3][5], const R gr[3][5],
                       const R Fob[2][5], const R Wob[2][5], EqAdj<R> &E)
{
    const R K = R(p.K);
    const Prim<R> &gC = P.gC;
    R gc[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) gc[d][q] = R(0);
    {
        SideFwd<R> S;
        side_forward<R, VISC, SMOOTH>(p, P.gL, P.l0, P.l1, gl, S, gc);
        side_forward<R, VISC, SMOOTH>(p, P.gR, P.r0, P.r1, gr, S, gc);
    }
    Tab<R> TC;
    gauss_moments<7>(gC.U, gC.lam, TC.u);
    vw_tables(gC, K, TC);
    const R irc = gC.ir;
    R ac[3][5], F[3][5], V[3][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) F[1][q] = V[1][q] = F[2][q] = V[2][q] = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gc[d][q] * irc;
        micro_slope(gC, K, b, ac[d]);
        if (d == 0) {
            contract<1, 0, 0>(TC, ac[d], R(1), V[1]);
            contract<2, 0, 0>(TC, ac[d], R(1), F[1]);
        } else if (d == 1) {
            contract<0, 1, 0>(TC, ac[d], R(1), V[1]);
            contract<1, 1, 0>(TC, ac[d], R(1), F[1]);
        } else {
            contract<0, 0, 1>(TC, ac[d], R(1), V[1]);
            contract<1, 0, 1>(TC, ac[d], R(1), F[1]);
        }
    }
    R nB[5], Ac[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) nB[q] = -V[1][q];
    micro_slope(gC, K, nB, Ac);
    contract<1, 0, 0>(TC, Ac, R(1), F[2]);
    contract<0, 0, 0>(TC, Ac, R(1), V[2]);
    psi_mom<1, 0, 0>(TC, F[0]);
    psi_mom<0, 0, 0>(TC, V[0]);

    zero(E.gCb);
#pragma unroll
    for (int k = 0; k < 3; ++k) E.cF0b[k] = E.cF1b[k] = E.cWb[k] = E.Ucb[k] = R(0);
    R Fb[3][5], Vb[3][5];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 5; ++q) Fb[j][q] = Vb[j][q] = R(0);
    {
        const R t0 = SMOOTH ? -P.tc.tau : R(0);
        const R cW0[3] = {SMOOTH ? R(1) : R(0), t0, t0};
        R cW0b[3] = {R(0), R(0), R(0)};
        add_part_rev<R, PRFIX>(p, gC.rho, P.tc.cF[0], P.tc.cF[1], cW0, P.tc.cW, F, V, P.Uc, Fob, Wob, E.gCb.rho,
                               E.cF0b, E.cF1b, cW0b, E.cWb, Fb, Vb, E.Ucb);
        E.taub = SMOOTH ? -(cW0b[1] + cW0b[2]) : R(0);
    }
    TabB<R> TCb;
    zero(TCb);
    R dummy = R(0);
    psi_mom_rev<0, 0, 0>(TC, Vb[0], TCb);
    psi_mom_rev<1, 0, 0>(TC, Fb[0], TCb);
    {
        R Acb[5] = {R(0), R(0), R(0), R(0), R(0)}, nBb[5] = {R(0), R(0), R(0), R(0), R(0)};
        contract_rev<0, 0, 0>(TC, Ac, R(1), Vb[2], TCb, Acb, dummy);
        contract_rev<1, 0, 0>(TC, Ac, R(1), Fb[2], TCb, Acb, dummy);
        micro_slope_rev(gC, K, nB, Acb, E.gCb, nBb);
#pragma unroll
        for (int q = 0; q < 5; ++q) Vb[1][q] -= nBb[q];
    }
    R ircb = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R ab[5] = {R(0), R(0), R(0), R(0), R(0)};
        if (d == 0) {
            contract_rev<1, 0, 0>(TC, ac[d], R(1), Vb[1], TCb, ab, dummy);
            contract_rev<2, 0, 0>(TC, ac[d], R(1), Fb[1], TCb, ab, dummy);
        } else if (d == 1) {
            contract_rev<0, 1, 0>(TC, ac[d], R(1), Vb[1], TCb, ab, dummy);
            contract_rev<1, 1, 0>(TC, ac[d], R(1), Fb[1], TCb, ab, dummy);
        } else {
            contract_rev<0, 0, 1>(TC, ac[d], R(1), Vb[1], TCb, ab, dummy);
            contract_rev<1, 0, 1>(TC, ac[d], R(1), Fb[1], TCb, ab, dummy);
        }
        R b[5], bb[5] = {R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gc[d][q] * irc;
        micro_slope_rev(gC, K, b, ab, E.gCb, bb);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            E.gcb[d][q] = bb[q] * irc;
            ircb += bb[q] * gc[d][q];
        }
        sched_fence();
    }
    E.gCb.rho -= ircb * irc * irc;
    vw_tables_rev(gC, K, TC, TCb, E.gCb);
    gauss_moments_rev<7>(gC.U, gC.lam, TC.u, TCb.u, E.gCb.U, E.gCb.lam);
}

template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void side_reverse(const Params &p, const PointFwd<R> &P, bool right, const R g[3][5], const R gcb[3][5],
                         const R Fob[2][5], const R Wob[2][5], SideAdj<R> &A)
{
    TimeCoefB<R> tcb;
    zero(tcb);
    zero(A.gb);
    A.m0b = A.m1b = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) A.grb[d][q] = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) A.Ucb[k] = R(0);
    side_terms_rev<R, VISC, PRFIX, SMOOTH>(p, right ? P.gR : P.gL, right ? P.r0 : P.l0, right ? P.r1 : P.l1, g, P.tc,
                                   P.Uc, gcb, Fob, Wob, A.gb, A.m0b, A.m1b, A.grb, tcb, A.Ucb);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        A.cF0b[k] = tcb.cF[0][3 + k];
        A.cF1b[k] = tcb.cF[1][3 + k];
        A.cWb[k] = tcb.cW[3 + k];
    }
    A.taub = tcb.tau;
}

// Completes the reverse: sets wlb, wrb (the adjoints of the point states).
template <typename R, bool VISC, bool SMOOTH = false>
GKS_HD void common_reverse(const Params &p, R dt, const R wl[5], const R wr[5], const PointFwd<R> &P,
                           const EqAdj<R> &E, const SideAdj<R> &SL, const SideAdj<R> &SR, R wlb[5], R wrb[5])
{
    const R K = R(p.K);
    const Prim<R> &gL = P.gL, &gR = P.gR, &gC = P.gC;
    TimeCoefB<R> tcb;
    zero(tcb);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        tcb.cF[0][k] = E.cF0b[k];
        tcb.cF[1][k] = E.cF1b[k];
        tcb.cW[k] = E.cWb[k];
        tcb.cF[0][3 + k] = SL.cF0b[k] + SR.cF0b[k];
        tcb.cF[1][3 + k] = SL.cF1b[k] + SR.cF1b[k];
        tcb.cW[3 + k] = SL.cWb[k] + SR.cWb[k];
    }
    tcb.tau = SL.taub + SR.taub;
    PrimB<R> gLb = SL.gb, gRb = SR.gb, gCb = E.gCb;
    R l0b = SL.m0b, l1b = SL.m1b, r0b = SR.m0b, r1b = SR.m1b;
    gCb.U += E.Ucb[0] + SL.Ucb[0] + SR.Ucb[0];
    gCb.V += E.Ucb[1] + SL.Ucb[1] + SR.Ucb[1];
    gCb.W += E.Ucb[2] + SL.Ucb[2] + SR.Ucb[2];
    // collision times
    R pcb = R(0);
    if constexpr (SMOOTH) {
        // the coefficients of eq. 2nd-smooth-flux are linear in tau
        R taub = E.taub;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const R del = k == 0 ? dt : R(0.5) * dt;
            taub -= del * (tcb.cF[k][1] + tcb.cF[k][2]);
        }
        taub -= tcb.cW[1] + tcb.cW[2];
        if (VISC) pcb -= taub * P.tau / P.pc;
    } else {
        R taub = R(0), taunb = R(0);
        time_coefficients_rev<R, VISC>(P.tau, P.taun, dt, tcb, taub, taunb);
        R jumpb;
        if (VISC) {
            taub += taunb;
            jumpb = taunb;
            pcb -= taub * P.tau / P.pc;
        } else {
            jumpb = taunb;
        }
        const R zb = jumpb * R(p.c_tau) * dt * sign_of(P.z);
        const R sp = P.pl + P.pr;
        const R plb = zb * R(2) * P.pr / (sp * sp), prb = -zb * R(2) * P.pl / (sp * sp);
        gLb.rho += plb * R(0.5) * gL.ilam;
        gLb.lam -= plb * P.pl * gL.ilam;
        gRb.rho += prb * R(0.5) * gR.ilam;
        gRb.lam -= prb * P.pr * gR.ilam;
    }
    gCb.rho += pcb * R(0.5) * gC.ilam;
    gCb.lam -= pcb * P.pc * gC.ilam;
    // gC = primitive(Wc)
    R Wcb[5] = {R(0), R(0), R(0), R(0), R(0)};
    primitive_rev(P.Wc, K, gCb, Wcb);
    // the kinetic weighting, one side at a time: rho, V, W, seeds m0, m1,
    // m2 = U m1 + h m0, t = V^2 + W^2 + (2+K) h
    const R s4 = R(0.5) * Wcb[4];
    {
        const R hl = R(0.5) * gL.ilam, l2 = gL.U * P.l1 + hl * P.l0;
        const R tl = gL.V * gL.V + gL.W * gL.W + (R(2) + K) * hl;
        gLb.rho += Wcb[0] * P.l0 + Wcb[1] * P.l1 + Wcb[2] * gL.V * P.l0 + Wcb[3] * gL.W * P.l0 + s4 * (l2 + P.l0 * tl);
        const R l2b = gL.rho * s4, tlb = gL.rho * s4 * P.l0;
        l0b += gL.rho * (Wcb[0] + Wcb[2] * gL.V + Wcb[3] * gL.W + s4 * tl);
        l1b += gL.rho * Wcb[1];
        gLb.V += gL.rho * Wcb[2] * P.l0 + R(2) * gL.V * tlb;
        gLb.W += gL.rho * Wcb[3] * P.l0 + R(2) * gL.W * tlb;
        gLb.U += l2b * P.l1;
        l1b += l2b * gL.U;
        l0b += l2b * hl;
        const R hlb = l2b * P.l0 + (R(2) + K) * tlb;
        gLb.lam -= hlb * hl * gL.ilam;
    }
    {
        const R hr = R(0.5) * gR.ilam, r2 = gR.U * P.r1 + hr * P.r0;
        const R tr = gR.V * gR.V + gR.W * gR.W + (R(2) + K) * hr;
        gRb.rho += Wcb[0] * P.r0 + Wcb[1] * P.r1 + Wcb[2] * gR.V * P.r0 + Wcb[3] * gR.W * P.r0 + s4 * (r2 + P.r0 * tr);
        const R r2b = gR.rho * s4, trb = gR.rho * s4 * P.r0;
        r0b += gR.rho * (Wcb[0] + Wcb[2] * gR.V + Wcb[3] * gR.W + s4 * tr);
        r1b += gR.rho * Wcb[1];
        gRb.V += gR.rho * Wcb[2] * P.r0 + R(2) * gR.V * trb;
        gRb.W += gR.rho * Wcb[3] * P.r0 + R(2) * gR.W * trb;
        gRb.U += r2b * P.r1;
        r1b += r2b * gR.U;
        r0b += r2b * hr;
        const R hrb = r2b * P.r0 + (R(2) + K) * trb;
        gRb.lam -= hrb * hr * gR.ilam;
    }
    // half-line seeds: d l0/dU = 2 lam e, d l0/dlam = U e, d l1/dU = l0,
    // d l1/dlam = -e/(2 lam); the right side with the signs of u < 0
    gLb.U += l0b * R(2) * gL.lam * P.el + l1b * P.l0;
    gLb.lam += l0b * gL.U * P.el - l1b * P.el / (R(2) * gL.lam);
    gRb.U += -r0b * R(2) * gR.lam * P.er + r1b * P.r0;
    gRb.lam += -r0b * gR.U * P.er + r1b * P.er / (R(2) * gR.lam);
#pragma unroll
    for (int q = 0; q < 5; ++q) wlb[q] = wrb[q] = R(0);
    primitive_rev(wl, K, gLb, wlb);
    primitive_rev(wr, K, gRb, wrb);
}

// Vector-Jacobian product of gks_point: given the adjoints Fob, Wob of its
// outputs, adds the adjoints of wl, gl, wr, gr (the four parts in sequence).
template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void gks_point_vjp(const Params &p, R dt, const R wl[5], const R gl[3][5], const R wr[5],
                          const R gr[3][5], const R Fob[2][5], const R Wob[2][5], R wlb[5], R glb[3][5],
                          R wrb[5], R grb[3][5])
{
    PointFwd<R> P;
    point_forward<R, VISC, SMOOTH>(p, dt, wl, wr, P);
    EqAdj<R> E;
    eq_reverse<R, VISC, PRFIX, SMOOTH>(p, P, gl, gr, Fob, Wob, E);
    SideAdj<R> SL, SR;
    side_reverse<R, VISC, PRFIX, SMOOTH>(p, P, true, gr, E.gcb, Fob, Wob, SR);
    side_reverse<R, VISC, PRFIX, SMOOTH>(p, P, false, gl, E.gcb, Fob, Wob, SL);
    R a[5], b[5];
    common_reverse<R, VISC, SMOOTH>(p, dt, wl, wr, P, E, SL, SR, a, b);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        wlb[q] += a[q];
        wrb[q] += b[q];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            glb[d][q] += SL.grb[d][q];
            grb[d][q] += SR.grb[d][q];
        }
    }
}

// Reverse of noslip_ghost (gks_flux.h): given the adjoints wgb, ggb of the
// ghost state and gradient, adds the adjoints of the interior point state w
// and gradient g.  The forward quantities are recomputed.
template <typename R>
GKS_HD void noslip_ghost_rev(bool iso, R gamma, R Tw, const R uw[3], const R w[5], const R g[3][5],
                             const R wgb[5], const R ggb[3][5], R wb[5], R gb[3][5])
{
    const R g1 = gamma - R(1), rho = w[0], ir = R(1) / rho;
    R U[3], Ug[3], Q = R(0), Qg = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        U[a] = w[1 + a] * ir;
        Ug[a] = R(2) * uw[a] - U[a];
        Q += R(0.5) * U[a] * U[a];
        Qg += R(0.5) * Ug[a] * Ug[a];
    }
    const R p = g1 * (w[4] - rho * Q), T = p * ir;
    const R Tg = iso ? R(2) * Tw - T : T, rhog = p / Tg;
    R rhob = R(0), irb = R(0), Ub[3] = {R(0), R(0), R(0)}, Ugb[3] = {R(0), R(0), R(0)};
    R Qb = R(0), Qgb = R(0), pb = R(0), Tb = R(0), Tgb = R(0), rhogb = R(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // forward of axis j
        const R dr = g[j][0];
        R dU[3], dQ = R(0), dQg = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dU[a] = (g[j][1 + a] - dr * U[a]) * ir;
            dQ += U[a] * dU[a];
            dQg += Ug[a] * dU[a];
        }
        const R dp = g1 * (g[j][4] - dr * Q - rho * dQ);
        const R dT = (dp - dr * T) * ir;
        const R dTg = iso ? dT : -dT;
        const R drg = (-dp - dTg * rhog) / Tg;
        // reverse: gg[j][0] = drg, gg[j][1+a] = drg Ug + rhog dU, gg[j][4] = drg Qg + rhog dQg - dp/g1
        R drgb = ggb[j][0] + ggb[j][4] * Qg;
        R dUb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            drgb += ggb[j][1 + a] * Ug[a];
            Ugb[a] += ggb[j][1 + a] * drg;
            rhogb += ggb[j][1 + a] * dU[a];
            dUb[a] = ggb[j][1 + a] * rhog;
        }
        Qgb += ggb[j][4] * drg;
        rhogb += ggb[j][4] * dQg;
        const R dQgb = ggb[j][4] * rhog;
        R dpb = -ggb[j][4] / g1;
        // drg = (-dp - dTg rhog) / Tg
        dpb -= drgb / Tg;
        const R dTgb = -drgb * rhog / Tg;
        rhogb -= drgb * dTg / Tg;
        Tgb -= drgb * drg / Tg;
        const R dTb = iso ? dTgb : -dTgb;
        // dT = (dp - dr T) ir
        dpb += dTb * ir;
        R drb = -dTb * T * ir;
        Tb -= dTb * dr * ir;
        irb += dTb * (dp - dr * T);
        // dp = g1 (g4 - dr Q - rho dQ)
        gb[j][4] += dpb * g1;
        drb -= dpb * g1 * Q;
        Qb -= dpb * g1 * dr;
        rhob -= dpb * g1 * dQ;
        const R dQb = -dpb * g1 * rho;
        // dQ = sum U dU, dQg = sum Ug dU, dU = (g - dr U) ir
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Ub[a] += dQb * dU[a];
            Ugb[a] += dQgb * dU[a];
            const R dUt = dUb[a] + dQb * U[a] + dQgb * Ug[a];
            gb[j][1 + a] += dUt * ir;
            drb -= dUt * U[a] * ir;
            Ub[a] -= dUt * dr * ir;
            irb += dUt * (g[j][1 + a] - dr * U[a]);
        }
        gb[j][0] += drb;
    }
    // wg = (rhog, rhog Ug, rhog Qg + p/g1)
    rhogb += wgb[0] + wgb[4] * Qg;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rhogb += wgb[1 + a] * Ug[a];
        Ugb[a] += wgb[1 + a] * rhog;
    }
    Qgb += wgb[4] * rhog;
    pb += wgb[4] / g1;
    // rhog = p / Tg, Tg = 2 Tw - T or T, T = p ir
    pb += rhogb / Tg;
    Tgb -= rhogb * rhog / Tg;
    Tb += iso ? -Tgb : Tgb;
    pb += Tb * ir;
    irb += Tb * p;
    // p = g1 (w4 - rho Q)
    wb[4] += pb * g1;
    rhob -= pb * g1 * Q;
    Qb -= pb * g1 * rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Ugb[a] += Qgb * Ug[a];
        Ub[a] += Qb * U[a] - Ugb[a];
        wb[1 + a] += Ub[a] * ir;
        irb += Ub[a] * w[1 + a];
    }
    rhob -= irb * ir * ir;
    wb[0] += rhob;
}

// Reverse of farfield_ghost (gks_flux.h): adds to wb the adjoint of the
// interior point state (the ghost has no gradients, so gb gets nothing).
// Differentiated as implemented: the branch taken, the free stream constant.
template <typename R>
GKS_HD void farfield_ghost_rev(R gamma, const R wf[5], const R w[5], const R wgb[5], R wb[5])
{
    const R g1 = gamma - R(1);
    const R ri = w[0], rf = wf[0];
    R Ui[3], Uf[3], ki = R(0), kf = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Ui[a] = w[1 + a] / ri;
        Uf[a] = wf[1 + a] / rf;
        ki += R(0.5) * Ui[a] * Ui[a];
        kf += R(0.5) * Uf[a] * Uf[a];
    }
    const R pi = g1 * (w[4] - ri * ki), pf = g1 * (wf[4] - rf * kf);
    const R ai = sqrt(gamma * pi / ri), af = sqrt(gamma * pf / rf);
    if (Ui[0] >= ai) {  // supersonic outflow: the ghost is the interior state
#pragma unroll
        for (int q = 0; q < 5; ++q) wb[q] += wgb[q];
        return;
    }
    if (Ui[0] <= -ai) return;  // supersonic inflow: the free stream
    const R Rp = Ui[0] + R(2) * ai / g1, Rm = Uf[0] - R(2) * af / g1;
    const R ub = R(0.5) * (Rp + Rm), ab = R(0.25) * g1 * (Rp - Rm);
    const bool out = ub > R(0);
    const R s = out ? pi / pow(ri, gamma) : pf / pow(rf, gamma);
    const R X = ab * ab / (gamma * s);
    const R rb = pow(X, R(1) / g1), pb = rb * ab * ab / gamma;
    const R ut1 = out ? Ui[1] : Uf[1], ut2 = out ? Ui[2] : Uf[2];
    // wg = (rb, rb ub, rb ut1, rb ut2, pb/g1 + rb (ub^2 + ut1^2 + ut2^2)/2)
    const R k2 = R(0.5) * (ub * ub + ut1 * ut1 + ut2 * ut2);
    R rbb = wgb[0] + wgb[1] * ub + wgb[2] * ut1 + wgb[3] * ut2 + wgb[4] * k2;
    R ubb = wgb[1] * rb + wgb[4] * rb * ub;
    const R ut1b = wgb[2] * rb + wgb[4] * rb * ut1, ut2b = wgb[3] * rb + wgb[4] * rb * ut2;
    const R pbb = wgb[4] / g1;
    // pb = rb ab^2 / gamma, rb = X^(1/g1), X = ab^2 / (gamma s)
    rbb += pbb * ab * ab / gamma;
    R abb = pbb * R(2) * rb * ab / gamma;
    const R Xb = rbb * rb / (g1 * X);
    abb += Xb * R(2) * ab / (gamma * s);
    const R sb = -Xb * X / s;
    // ab = g1 (Rp - Rm) / 4, ub = (Rp + Rm) / 2; Rm is the free stream's
    const R Rpb = R(0.25) * g1 * abb + R(0.5) * ubb;
    R Uib[3] = {Rpb, R(0), R(0)};
    R aib = R(2) * Rpb / g1, pib = R(0), rib = R(0);
    if (out) {
        // s = pi ri^-gamma, ut = Ui[1], Ui[2]
        const R rg = pow(ri, gamma);
        pib += sb / rg;
        rib -= gamma * sb * s / ri;
        Uib[1] += ut1b;
        Uib[2] += ut2b;
    }
    // ai = sqrt(gamma pi / ri)
    pib += aib * gamma / (R(2) * ai * ri);
    rib -= aib * ai / (R(2) * ri);
    // pi = g1 (w4 - ri ki), ki = |Ui|^2 / 2, Ui = w[1+a] / ri
    wb[4] += g1 * pib;
    rib -= g1 * pib * ki;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Uib[a] -= g1 * pib * ri * Ui[a];
        wb[1 + a] += Uib[a] / ri;
        rib -= Uib[a] * Ui[a] / ri;
    }
    wb[0] += rib;
}

// The wall ghost of a point and its reverse, as the flux uses them: the
// slip mirror (its own transpose), the far-field state or the no-slip
// reflection.
template <typename R>
GKS_HD void wall_ghost(const Params &p, int tag, const R T[3][3], const R u[3], const R wl[5], const R gl[3][5],
                       R wr[5], R gr[3][5])
{
    if (tag == WALL_SLIP) {
        slip_ghost(wl, gl, wr, gr);
        return;
    }
    if (tag == WALL_FARFIELD) {
        R wf[5];
        wf[0] = R(p.farfield[0]);
        wf[4] = R(p.farfield[4]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            wf[1 + a] = T[a][0] * R(p.farfield[1]) + T[a][1] * R(p.farfield[2]) + T[a][2] * R(p.farfield[3]);
        farfield_ghost(R(p.gamma), wf, wl, wr, gr);
        return;
    }
    R uw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) uw[a] = T[a][0] * u[0] + T[a][1] * u[1] + T[a][2] * u[2];
    noslip_ghost(tag == WALL_ISOTHERMAL, R(p.gamma), R(p.wall_T), uw, wl, gl, wr, gr);
}

// wrb, grb: adjoints of the ghost; adds to wlb, glb
template <typename R>
GKS_HD void wall_ghost_rev(const Params &p, int tag, const R T[3][3], const R u[3], const R wl[5],
                           const R gl[3][5], const R wrb[5], const R grb[3][5], R wlb[5], R glb[3][5])
{
    if (tag == WALL_SLIP) {
        R wg[5], gg[3][5];
        slip_ghost(wrb, grb, wg, gg);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            wlb[q] += wg[q];
#pragma unroll
            for (int d = 0; d < 3; ++d) glb[d][q] += gg[d][q];
        }
        return;
    }
    if (tag == WALL_FARFIELD) {
        R wf[5];
        wf[0] = R(p.farfield[0]);
        wf[4] = R(p.farfield[4]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            wf[1 + a] = T[a][0] * R(p.farfield[1]) + T[a][1] * R(p.farfield[2]) + T[a][2] * R(p.farfield[3]);
        farfield_ghost_rev(R(p.gamma), wf, wl, wrb, wlb);
        return;
    }
    R uw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) uw[a] = T[a][0] * u[0] + T[a][1] * u[1] + T[a][2] * u[2];
    noslip_ghost_rev(tag == WALL_ISOTHERMAL, R(p.gamma), R(p.wall_T), uw, wl, gl, wrb, grb, wlb, glb);
}

// Reverse of the rotation in eval_local: adjoints of the rotated point state
// w and gradient g (face frame) to the unrotated W[5] and G[5][3] (set).
template <typename R>
GKS_HD void point_adjoint_global(const R T[3][3], const R wb[5], const R gb[3][5], R Wb[5], R Gb[5][3])
{
    Wb[0] = wb[0];
    Wb[4] = wb[4];
#pragma unroll
    for (int b = 0; b < 3; ++b) Wb[1 + b] = T[0][b] * wb[1] + T[1][b] * wb[2] + T[2][b] * wb[3];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
        for (int d = 0; d < 3; ++d) Gb[q][d] = R(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        R dWb[5];
        dWb[0] = gb[j][0];
        dWb[4] = gb[j][4];
#pragma unroll
        for (int b = 0; b < 3; ++b) dWb[1 + b] = T[0][b] * gb[j][1] + T[1][b] * gb[j][2] + T[2][b] * gb[j][3];
#pragma unroll
        for (int q = 0; q < 5; ++q)
#pragma unroll
            for (int d = 0; d < 3; ++d) Gb[q][d] += T[j][d] * dWb[q];
    }
}

// Reverse of the polynomial evaluation at offset r for one component:
// adjoints of its value w and gradient G[3] to its ten coefficients (set).
template <typename R>
GKS_HD void coef_adjoint(const R r[3], R w, const R G[3], R cb[10])
{
    cb[0] = w;
    cb[1] = w * r[0] + G[0];
    cb[2] = w * r[1] + G[1];
    cb[3] = w * r[2] + G[2];
    cb[4] = R(0.5) * w * r[0] * r[0] + G[0] * r[0];
    cb[5] = R(0.5) * w * r[1] * r[1] + G[1] * r[1];
    cb[6] = R(0.5) * w * r[2] * r[2] + G[2] * r[2];
    cb[7] = w * r[0] * r[1] + G[0] * r[1] + G[1] * r[0];
    cb[8] = w * r[0] * r[2] + G[0] * r[2] + G[2] * r[0];
    cb[9] = w * r[1] * r[2] + G[1] * r[2] + G[2] * r[1];
}

// Reverse of eval_local: adjoints of the rotated point state w and gradient g
// to the cell's coefficients cb[5][10] (added).
template <typename R>
GKS_HD void eval_local_rev(const R r[3], const R T[3][3], const R wb[5], const R gb[3][5], R cb[5][10])
{
    R Wb[5], Gb[5][3];
    point_adjoint_global(T, wb, gb, Wb, Gb);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        R t[10];
        coef_adjoint(r, Wb[q], Gb[q], t);
#pragma unroll
        for (int k = 0; k < 10; ++k) cb[q][k] += t[k];
    }
}

// to_global sets gout[1+a] = sum_b T[b][a] l[1+b]; its transpose
template <typename R>
GKS_HD void to_global_rev(const R T[3][3], const R goutb[5], R lb[5])
{
    lb[0] = goutb[0];
    lb[4] = goutb[4];
#pragma unroll
    for (int b = 0; b < 3; ++b) lb[1 + b] = T[b][0] * goutb[1] + T[b][1] * goutb[2] + T[b][2] * goutb[3];
}

// Vector-Jacobian product of gauss_point_terms down to the unrotated point
// values: accb = adjoint of acc[4][5]; sets the adjoints of both sides' point
// state Wb[2][5] and gradient Gb[2][5][3] (global frame) and the two offsets
// r[2][3] at which the cells' polynomials are evaluated.
template <typename R, bool VISC, bool PRFIX, typename CoefL, typename CoefR, bool SMOOTH = false>
GKS_HD void gauss_point_vjp_point(const Params &p, R dt, const R nrm[3], R area, const R r[3], const R dv[3],
                                  const CoefL &cl, const CoefR &cr, const R accb[4][5], R Wb[2][5],
                                  R Gb[2][5][3], R off[2][3], bool wall = false)
{
    const R w = area * R(1.0 / 3.0);
    R T[3][3];
    rotation(nrm, T);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        off[0][d] = r[d];
        off[1][d] = r[d] + dv[d];
    }
    R wl[5], gl[3][5], wr[5], gr[3][5];
    eval_local(cl, off[0], T, wl, gl);
    if (wall)
        slip_ghost(wl, gl, wr, gr);
    else
        eval_local(cr, off[1], T, wr, gr);
    const R idt = R(1) / dt;
    // acc0 = w (4 Fh - F1)/dt, acc1 = 4 w (F1 - 2 Fh)/dt^2, acc2 = w W0, acc3 = w W1
    R gF1[5], gFh[5], gW0[5], gW1[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        gF1[q] = w * (-accb[0][q] * idt + R(4) * accb[1][q] * (idt * idt));
        gFh[q] = w * (R(4) * accb[0][q] * idt - R(8) * accb[1][q] * (idt * idt));
        gW0[q] = w * accb[2][q];
        gW1[q] = w * accb[3][q];
    }
    R Fob[2][5], Wob[2][5];
    to_global_rev(T, gF1, Fob[0]);
    to_global_rev(T, gFh, Fob[1]);
    to_global_rev(T, gW0, Wob[0]);
    to_global_rev(T, gW1, Wob[1]);
    R wlb[5], glb[3][5], wrb[5], grb[3][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        wlb[q] = wrb[q] = R(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) glb[d][q] = grb[d][q] = R(0);
    }
    gks_point_vjp<R, VISC, PRFIX, SMOOTH>(p, dt, wl, gl, wr, gr, Fob, Wob, wlb, glb, wrb, grb);
    if (wall) {
        // the ghost is a linear function of the left state; its transpose is itself
        R wg[5], gg[3][5];
        slip_ghost(wrb, grb, wg, gg);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            wlb[q] += wg[q];
            wrb[q] = R(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                glb[d][q] += gg[d][q];
                grb[d][q] = R(0);
            }
        }
    }
    point_adjoint_global(T, wlb, glb, Wb[0], Gb[0]);
    point_adjoint_global(T, wrb, grb, Wb[1], Gb[1]);
}

// Vector-Jacobian product of gauss_point_terms with respect to the two
// cells' coefficients: accb = adjoint of acc[4][5]; adds to cbl, cbr.
template <typename R, bool VISC, bool PRFIX, typename CoefL, typename CoefR, bool SMOOTH = false>
GKS_HD void gauss_point_terms_vjp(const Params &p, R dt, const R nrm[3], R area, const R r[3], const R dv[3],
                                  const CoefL &cl, const CoefR &cr, const R accb[4][5], R cbl[5][10],
                                  R cbr[5][10])
{
    R Wb[2][5], Gb[2][5][3], off[2][3];
    gauss_point_vjp_point<R, VISC, PRFIX, CoefL, CoefR, SMOOTH>(p, dt, nrm, area, r, dv, cl, cr, accb, Wb, Gb, off);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        R t[10];
        coef_adjoint(off[0], Wb[0][q], Gb[0][q], t);
#pragma unroll
        for (int k = 0; k < 10; ++k) cbl[q][k] += t[k];
        coef_adjoint(off[1], Wb[1][q], Gb[1][q], t);
#pragma unroll
        for (int k = 0; k < 10; ++k) cbr[q][k] += t[k];
    }
}

#undef GKS_HD

}  // namespace gks
