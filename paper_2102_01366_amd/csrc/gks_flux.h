// Gas-kinetic flux of the compact GKS (Sec. 2.2 of Ji, Zhao, Shyy & Xu) at
// the Gauss points of one face, written once for the device (R = double or
// float) and for host-side operation counting (R = a counting scalar).
//
// In the face frame (eq. rotate-matrix-3d) every moment of a Maxwellian
// factorises into 1-D moments of u (full or half line), v, w and xi^2.  The
// integrands of eq. 2nd-flux are contracted with the microscopic slopes in
// closed form (psi_mom / contract below); the slopes solve the 5x5 moment
// systems of eq. co in closed form (micro_slope).
#pragma once

#include "gks_internal.h"

#include <cmath>

namespace gks {

#define GKS_HD __host__ __device__ __forceinline__

// Maxwellian g = rho (lam/pi)^((K+3)/2) exp(-lam(|u-U|^2 + xi^2)) of a state;
// rho E = rho (|U|^2/2 + (K+3)/(4 lam)).
// ir = 1/rho and ilam = 1/lam are kept so that the many quotients by rho and
// lam below are products (FP64 division is a long instruction sequence).
template <typename R>
struct Prim {
    R rho, U, V, W, lam, ir, ilam;
};

template <typename R>
GKS_HD Prim<R> primitive(const R w[5], R K)
{
    Prim<R> g;
    g.rho = w[0];
    g.ir = R(1) / w[0];
    g.U = w[1] * g.ir;
    g.V = w[2] * g.ir;
    g.W = w[3] * g.ir;
    g.lam = (K + R(3)) * w[0] / (R(4) * (w[4] - R(0.5) * w[0] * (g.U * g.U + g.V * g.V + g.W * g.W)));
    g.ilam = R(1) / g.lam;
    return g;
}

// normalised moments <c^k>, k < N, of a Gaussian of mean U and variance h = 1/(2 lam)
template <int N, typename R>
GKS_HD void gauss_moments_h(R U, R h, R *m)
{
    m[0] = R(1);
    m[1] = U;
#pragma unroll
    for (int k = 0; k + 2 < N; ++k) m[k + 2] = U * m[k + 1] + R(k + 1) * h * m[k];
}
template <int N, typename R>
GKS_HD void gauss_moments(R U, R lam, R *m)
{
    const R h = R(0.5) / lam;
    m[0] = R(1);
    m[1] = U;
#pragma unroll
    for (int k = 0; k + 2 < N; ++k) m[k + 2] = U * m[k + 1] + R(k + 1) * h * m[k];
}

// the same over u > 0 (pos) or u < 0:
// <1>_{u>0} = erfc(-sqrt(lam) U)/2, <u>_{u>0} = U <1>_{u>0} + exp(-lam U^2) / (2 sqrt(pi lam))
template <int N, typename R>
GKS_HD void half_moments(R U, R lam, bool pos, R *m)
{
    const R h = R(0.5) / lam;
    const R sl = sqrt(lam);
    const R e = exp(-lam * U * U) / (R(2) * sqrt(R(M_PI) * lam));
    if (pos) {
        m[0] = R(0.5) * erfc(-sl * U);
        m[1] = U * m[0] + e;
    } else {
        m[0] = R(0.5) * erfc(sl * U);
        m[1] = U * m[0] - e;
    }
#pragma unroll
    for (int k = 0; k + 2 < N; ++k) m[k + 2] = U * m[k + 1] + R(k + 1) * h * m[k];
}

// Moment tables of one Maxwellian: u (full or half line) to order 6, v and w
// to order 5, <xi^2> and <xi^4>.
template <typename R>
struct Tab {
    R u[7], v[6], w[6], xi2, xi4;
};

template <typename R>
GKS_HD void vw_tables(const Prim<R> &g, R K, Tab<R> &t)
{
    const R h = R(0.5) * g.ilam;
    gauss_moments_h<6>(g.V, h, t.v);
    gauss_moments_h<6>(g.W, h, t.w);
    t.xi2 = K * h;
    t.xi4 = K * (K + R(2)) * (h * h);
}

// t[j] = <u^A v^B w^C psi_j>, psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2)
template <int A, int B, int C, typename R>
GKS_HD void psi_mom(const Tab<R> &T, R t[5])
{
    const R m = T.u[A] * T.v[B] * T.w[C];
    t[0] = m;
    t[1] = T.u[A + 1] * T.v[B] * T.w[C];
    t[2] = T.u[A] * T.v[B + 1] * T.w[C];
    t[3] = T.u[A] * T.v[B] * T.w[C + 1];
    t[4] = R(0.5) * (T.u[A + 2] * T.v[B] * T.w[C] + T.u[A] * T.v[B + 2] * T.w[C] +
                     T.u[A] * T.v[B] * T.w[C + 2] + T.xi2 * m);
}

// out += s <u^A v^B w^C (a.psi) psi>, factorised.  With h = a_4/2 and
// S(al,be,ga) = <u^al v^be w^ga (a.psi)> = P_al V_be W_ga + U_al X(be,ga), where
//   P_al = (a_0 + h <xi^2>) U_al + a_1 U_{al+1} + h U_{al+2},
//   X(be,ga) = a_2 V_{be+1} W_ga + a_3 V_be W_{ga+1} + h (V_{be+2} W_ga + V_be W_{ga+2}),
// the five components are S(A,B,C), S(A+1,B,C), S(A,B+1,C), S(A,B,C+1) and
// (S(A+2,B,C) + S(A,B+2,C) + S(A,B,C+2) + <xi^2 u^A v^B w^C (a.psi)>) / 2,
// using <xi^2 Y (a.psi)> = <xi^2> S + h (<xi^4> - <xi^2>^2) <Y>.
template <int A, int B, int C, typename R>
GKS_HD void contract(const Tab<R> &T, const R a[5], R s, R out[5])
{
    const R *U = T.u, *V = T.v, *W = T.w;
    const R h = R(0.5) * a[4];
    const R c0 = a[0] + h * T.xi2;
    const R P0 = c0 * U[A] + a[1] * U[A + 1] + h * U[A + 2];
    const R P1 = c0 * U[A + 1] + a[1] * U[A + 2] + h * U[A + 3];
    const R P2 = c0 * U[A + 2] + a[1] * U[A + 3] + h * U[A + 4];
    const R vw00 = V[B] * W[C], vw10 = V[B + 1] * W[C], vw01 = V[B] * W[C + 1];
    const R vw20 = V[B + 2] * W[C], vw02 = V[B] * W[C + 2];
    const R vw11 = V[B + 1] * W[C + 1];
    const R X00 = a[2] * vw10 + a[3] * vw01 + h * (vw20 + vw02);
    const R X10 = a[2] * vw20 + a[3] * vw11 + h * (V[B + 3] * W[C] + V[B + 1] * W[C + 2]);
    const R X01 = a[2] * vw11 + a[3] * vw02 + h * (V[B + 2] * W[C + 1] + V[B] * W[C + 3]);
    const R X20 = a[2] * (V[B + 3] * W[C]) + a[3] * (V[B + 2] * W[C + 1]) +
                  h * (V[B + 4] * W[C] + V[B + 2] * W[C + 2]);
    const R X02 = a[2] * (V[B + 1] * W[C + 2]) + a[3] * (V[B] * W[C + 3]) +
                  h * (V[B + 2] * W[C + 2] + V[B] * W[C + 4]);
    const R S000 = P0 * vw00 + U[A] * X00;
    const R S100 = P1 * vw00 + U[A + 1] * X00;
    const R S010 = P0 * vw10 + U[A] * X10;
    const R S001 = P0 * vw01 + U[A] * X01;
    const R S200 = P2 * vw00 + U[A + 2] * X00;
    const R S020 = P0 * vw20 + U[A] * X20;
    const R S002 = P0 * vw02 + U[A] * X02;
    const R Sxi = T.xi2 * S000 + h * (T.xi4 - T.xi2 * T.xi2) * (U[A] * vw00);
    out[0] += s * S000;
    out[1] += s * S100;
    out[2] += s * S010;
    out[3] += s * S001;
    out[4] += R(0.5) * s * (S200 + S020 + S002 + Sxi);
}

// Solve <psi psi^T> a = b for a Maxwellian (eq. co) in closed form.
template <typename R>
GKS_HD void micro_slope(const Prim<R> &g, R K, const R b[5], R a[5])
{
    const R U = g.U, V = g.V, W = g.W, lam = g.lam;
    const R q2 = U * U + V * V + W * W + (K + R(3)) * (R(0.5) * g.ilam);
    const R R1 = b[1] - U * b[0], R2 = b[2] - V * b[0], R3 = b[3] - W * b[0];
    const R R4 = R(2) * b[4] - q2 * b[0];
    // 4 / (K + 3) is the same quotient in every call
    a[4] = lam * lam * (R(4) / (K + R(3))) * (R4 - R(2) * U * R1 - R(2) * V * R2 - R(2) * W * R3);
    a[1] = R(2) * lam * R1 - U * a[4];
    a[2] = R(2) * lam * R2 - V * a[4];
    a[3] = R(2) * lam * R3 - W * a[4];
    a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - R(0.5) * a[4] * q2;
}

// Heat flux about U^c of a moment pair: with F = <u psi Y> and V = <psi Y>,
// <(u-U)((u-U)^2 + (v-V)^2 + (w-W)^2 + xi^2) Y>/2 =
//   F4 - U F1 - V F2 - W F3 + (|U|^2/2 + U^2) F0 - U V4 + U V V2 + U W V3 - U |U|^2/2 V0
template <typename R>
GKS_HD R heat_moment(const R Uc[3], const R F[5], const R V[5])
{
    const R U = Uc[0], Vv = Uc[1], W = Uc[2], U2 = U * U + Vv * Vv + W * W;
    return F[4] - U * F[1] - Vv * F[2] - W * F[3] + (R(0.5) * U2 + U * U) * F[0] - U * V[4] +
           U * Vv * V[2] + U * W * V[3] - R(0.5) * U * U2 * V[0];
}

// The interface-time coefficients of eq. 2nd-flux.  cF[k][0..5]: time
// integrals over [0, delta_k], delta = (dt, dt/2), of the six coefficients
// (equilibrium: 1 - e, (t + tau) e - tau, t - tau + tau e; kinetic: e,
// -(tau + t) e, -tau e, with e = exp(-t/tau_n)); cW[0..5]: the same
// coefficients at t = dt.  At t = 0 they are (0, 0, 0, 1, -tau, -tau).
template <typename R>
struct TimeCoef {
    R tau, cF[2][6], cW[6];
};

template <typename R, bool VISC>
GKS_HD void time_coefficients(R tau, R taun, R dt, TimeCoef<R> &tc)
{
    tc.tau = tau;
    const R itaun = R(1) / taun;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const R del = k == 0 ? dt : R(0.5) * dt;
        const R e = exp(-del * itaun);
        const R E1 = taun * (R(1) - e);
        const R E2 = taun * taun * (R(1) - e) - taun * del * e;
        if (VISC) {
            tc.cF[k][0] = del - E1;
            tc.cF[k][1] = E2 + tau * E1 - tau * del;
            tc.cF[k][2] = R(0.5) * del * del - tau * del + tau * E1;
            tc.cF[k][3] = E1;
            tc.cF[k][4] = -(tau * E1 + E2);
            tc.cF[k][5] = -tau * E1;
        } else {
            tc.cF[k][0] = del - E1;
            tc.cF[k][1] = E2;
            tc.cF[k][2] = R(0.5) * del * del;
            tc.cF[k][3] = E1;
            tc.cF[k][4] = -E2;
            tc.cF[k][5] = R(0);
        }
    }
    const R et = exp(-dt * itaun);
    tc.cW[0] = R(1) - et;
    tc.cW[3] = et;
    if (VISC) {
        tc.cW[1] = (dt + tau) * et - tau;
        tc.cW[2] = dt - tau + tau * et;
        tc.cW[4] = -(tau + dt) * et;
        tc.cW[5] = -tau * et;
    } else {
        tc.cW[1] = dt * et;
        tc.cW[2] = dt;
        tc.cW[4] = -dt * et;
        tc.cW[5] = R(0);
    }
}

// The coefficients of eq. 2nd-smooth-flux in the same slots: the
// equilibrium part 1, -tau, t - tau (the limit tau_n -> 0 of eq. 2nd-flux
// with tau kept) and no kinetic part.  At t = 0 the equilibrium part is
// (1, -tau, -tau).
template <typename R>
GKS_HD void time_coefficients_smooth(R tau, R dt, TimeCoef<R> &tc)
{
    tc.tau = tau;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const R del = k == 0 ? dt : R(0.5) * dt;
        tc.cF[k][0] = del;
        tc.cF[k][1] = -tau * del;
        tc.cF[k][2] = R(0.5) * del * del - tau * del;
        tc.cF[k][3] = tc.cF[k][4] = tc.cF[k][5] = R(0);
    }
    tc.cW[0] = R(1);
    tc.cW[1] = -tau;
    tc.cW[2] = dt - tau;
    tc.cW[3] = tc.cW[4] = tc.cW[5] = R(0);
}

// Adds the part a, b, c of eq. 2nd-flux with moment vectors F_j = <u psi Y_j>,
// V_j = <psi Y_j> (Y_0 = 1, Y_1 = slopes term, Y_2 = time-slope term) to the
// time integrals Fo, the point values Wo (t = 0, dt), and, with the Prandtl
// correction, the heat flux into the energy flux.
template <typename R, bool PRFIX>
GKS_HD void add_part(const Params &p, R rho, const R *cF0, const R *cF1, const R *cW0, const R *cW1,
                     const R F[3][5], const R V[3][5], const R Uc[3], R Fo[2][5], R Wo[2][5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        Fo[0][q] += rho * (cF0[0] * F[0][q] + cF0[1] * F[1][q] + cF0[2] * F[2][q]);
        Fo[1][q] += rho * (cF1[0] * F[0][q] + cF1[1] * F[1][q] + cF1[2] * F[2][q]);
        Wo[0][q] += rho * (cW0[0] * V[0][q] + cW0[1] * V[1][q] + cW0[2] * V[2][q]);
        Wo[1][q] += rho * (cW1[0] * V[0][q] + cW1[1] * V[1][q] + cW1[2] * V[2][q]);
    }
    if (PRFIX) {
        const R fac = R(1.0 / p.prandtl - 1.0);
        const R h0 = heat_moment(Uc, F[0], V[0]), h1 = heat_moment(Uc, F[1], V[1]),
                h2 = heat_moment(Uc, F[2], V[2]);
        Fo[0][4] += fac * rho * (cF0[0] * h0 + cF0[1] * h1 + cF0[2] * h2);
        Fo[1][4] += fac * rho * (cF1[0] * h0 + cF1[1] * h1 + cF1[2] * h2);
    }
}

// Kinetic part of one side (u > 0 for the left state, u < 0 for the right),
// given its half-line seeds <1>, <u>: the slopes' contribution to the
// interface gradients gc, and the side's terms of eq. 2nd-flux (none with
// the smooth-flow distribution, SMOOTH).
template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void side_terms(const Params &p, const Prim<R> &g, R m0, R m1, const R gr[3][5],
                       const TimeCoef<R> &tc, const R Uc[3], R gc[3][5], R Fo[2][5], R Wo[2][5])
{
    const R K = R(p.K);
    Tab<R> Th;
    {
        const R h = R(0.5) * g.ilam;
        Th.u[0] = m0;
        Th.u[1] = m1;
#pragma unroll
        for (int k = 0; k + 2 < 7; ++k) Th.u[k + 2] = g.U * Th.u[k + 1] + R(k + 1) * h * Th.u[k];
    }
    vw_tables(g, K, Th);
    if constexpr (SMOOTH) {
        const R ir = g.ir;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            R b[5], a[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
            micro_slope(g, K, b, a);
            contract<0, 0, 0>(Th, a, g.rho, gc[d]);
        }
        return;
    }
    R F[3][5], V[3][5];
    psi_mom<1, 0, 0>(Th, F[0]);
    psi_mom<0, 0, 0>(Th, V[0]);
#pragma unroll
    for (int q = 0; q < 5; ++q) F[1][q] = V[1][q] = F[2][q] = V[2][q] = R(0);
    R B[5] = {R(0), R(0), R(0), R(0), R(0)};
    Tab<R> Tf;
    if (VISC) {
        gauss_moments_h<7>(g.U, R(0.5) * g.ilam, Tf.u);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Tf.v[k] = Th.v[k];
            Tf.w[k] = Th.w[k];
        }
        Tf.xi2 = Th.xi2;
        Tf.xi4 = Th.xi4;
    }
    const R ir = g.ir;
    // one direction at a time: a_d, its share of g^c_{x_d}, of
    // sum_d <u u_d (a_d.psi) psi> and of sum_d <u_d (a_d.psi) psi>
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5], a[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
        micro_slope(g, K, b, a);
        contract<0, 0, 0>(Th, a, g.rho, gc[d]);
        if (d == 0) {
            contract<2, 0, 0>(Th, a, R(1), F[1]);
            contract<1, 0, 0>(Th, a, R(1), V[1]);
            if (VISC) contract<1, 0, 0>(Tf, a, R(-1), B);
        } else if (d == 1) {
            contract<1, 1, 0>(Th, a, R(1), F[1]);
            contract<0, 1, 0>(Th, a, R(1), V[1]);
            if (VISC) contract<0, 1, 0>(Tf, a, R(-1), B);
        } else {
            contract<1, 0, 1>(Th, a, R(1), F[1]);
            contract<0, 0, 1>(Th, a, R(1), V[1]);
            if (VISC) contract<0, 0, 1>(Tf, a, R(-1), B);
        }
    }
    if (VISC) {
        // A of this side from its full-space compatibility condition
        R A[5];
        micro_slope(g, K, B, A);
        contract<1, 0, 0>(Th, A, R(1), F[2]);
        contract<0, 0, 0>(Th, A, R(1), V[2]);
    }
    const R cW0[3] = {R(1), -tc.tau, -tc.tau};
    add_part<R, PRFIX>(p, g.rho, tc.cF[0] + 3, tc.cF[1] + 3, cW0, tc.cW + 3, F, V, Uc, Fo, Wo);
}

// Everything of one interface point that both kinetic sides and the
// equilibrium part need: the two sides' primitive states and half-line seeds
// <1>, <u>, the kinetically weighted equilibrium g^c (eq. new-equ-part) and
// the time coefficients of its collision times.
template <typename R>
struct PointSetup {
    Prim<R> gL, gR, gC;
    R l0, l1, r0, r1;
    TimeCoef<R> tc;
};

template <typename R, bool VISC, bool SMOOTH = false>
GKS_HD void point_setup(const Params &p, R dt, const R wl[5], const R wr[5], PointSetup<R> &S)
{
    const R K = R(p.K);
    const Prim<R> gL = primitive(wl, K), gR = primitive(wr, K);
    S.gL = gL;
    S.gR = gR;
    // half-line seeds <1> and <u> of both sides
    R l0, l1, r0, r1;
    {
        // exp(-lam U^2) / (2 sqrt(pi lam)) = exp(-lam U^2) sqrt(pi lam) / (2 pi lam)
        const R sl = sqrt(gL.lam),
                e = exp(-gL.lam * gL.U * gL.U) * (sqrt(R(M_PI) * gL.lam) * gL.ilam) * R(0.5 / M_PI);
        l0 = R(0.5) * erfc(-sl * gL.U);
        l1 = gL.U * l0 + e;
        const R sr = sqrt(gR.lam),
                f = exp(-gR.lam * gR.U * gR.U) * (sqrt(R(M_PI) * gR.lam) * gR.ilam) * R(0.5 / M_PI);
        r0 = R(0.5) * erfc(sr * gR.U);
        r1 = gR.U * r0 - f;
    }
    S.l0 = l0;
    S.l1 = l1;
    S.r0 = r0;
    S.r1 = r1;
    // eq. new-equ-part: W^c = rho_l <psi>_{u>0} + rho_r <psi>_{u<0}
    R Wc[5];
    {
        const R hl = R(0.5) * gL.ilam, hr = R(0.5) * gR.ilam;
        const R l2 = gL.U * l1 + hl * l0, r2 = gR.U * r1 + hr * r0;
        const R tl = gL.V * gL.V + gL.W * gL.W + (R(2) + K) * hl;
        const R tr = gR.V * gR.V + gR.W * gR.W + (R(2) + K) * hr;
        Wc[0] = gL.rho * l0 + gR.rho * r0;
        Wc[1] = gL.rho * l1 + gR.rho * r1;
        Wc[2] = gL.rho * (gL.V * l0) + gR.rho * (gR.V * r0);
        Wc[3] = gL.rho * (gL.W * l0) + gR.rho * (gR.W * r0);
        Wc[4] = gL.rho * (R(0.5) * (l2 + l0 * tl)) + gR.rho * (R(0.5) * (r2 + r0 * tr));
    }
    const Prim<R> gC = primitive(Wc, K);
    S.gC = gC;
    // collision times (Sec. 2.2)
    const R pl = gL.rho * R(0.5) * gL.ilam, pr = gR.rho * R(0.5) * gR.ilam, pc = gC.rho * R(0.5) * gC.ilam;
    if constexpr (SMOOTH) {
        time_coefficients_smooth<R>(VISC ? R(p.mu) / pc : R(0), dt, S.tc);
    } else {
        const R jump = R(p.c_tau) * fabs((pl - pr) / (pl + pr)) * dt;
        R tau, taun;
        if (VISC) {
            tau = R(p.mu) / pc;
            taun = tau + jump;
        } else {
            tau = R(0);
            taun = R(p.eps_tau) * dt + jump;
        }
        time_coefficients<R, VISC>(tau, taun, dt, S.tc);
    }
}

// The equilibrium part of eq. 2nd-flux: g^c with slopes a^c (from g^c_x,
// gc) and A^c, added to Fo and Wo.
template <typename R, bool PRFIX, bool SMOOTH = false>
GKS_HD void equilibrium_terms(const Params &p, const Prim<R> &gC, const TimeCoef<R> &tc, const R gc[3][5],
                              R Fo[2][5], R Wo[2][5])
{
    const R K = R(p.K);
    const R Uc[3] = {gC.U, gC.V, gC.W};
    Tab<R> TC;
    gauss_moments_h<7>(gC.U, R(0.5) * gC.ilam, TC.u);
    vw_tables(gC, K, TC);
    R F[3][5], V[3][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) F[1][q] = V[1][q] = F[2][q] = V[2][q] = R(0);
    const R irc = gC.ir;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5], a[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gc[d][q] * irc;
        micro_slope(gC, K, b, a);
        if (d == 0) {
            contract<1, 0, 0>(TC, a, R(1), V[1]);
            contract<2, 0, 0>(TC, a, R(1), F[1]);
        } else if (d == 1) {
            contract<0, 1, 0>(TC, a, R(1), V[1]);
            contract<1, 1, 0>(TC, a, R(1), F[1]);
        } else {
            contract<0, 0, 1>(TC, a, R(1), V[1]);
            contract<1, 0, 1>(TC, a, R(1), F[1]);
        }
    }
    {
        R nB[5], Ac[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) nB[q] = -V[1][q];
        micro_slope(gC, K, nB, Ac);
        contract<1, 0, 0>(TC, Ac, R(1), F[2]);
        contract<0, 0, 0>(TC, Ac, R(1), V[2]);
    }
    psi_mom<1, 0, 0>(TC, F[0]);
    psi_mom<0, 0, 0>(TC, V[0]);
    const R cW0[3] = {SMOOTH ? R(1) : R(0), SMOOTH ? -tc.tau : R(0), SMOOTH ? -tc.tau : R(0)};
    add_part<R, PRFIX>(p, gC.rho, tc.cF[0], tc.cF[1], cW0, tc.cW, F, V, Uc, Fo, Wo);
}

// Time-dependent distribution of eq. 2nd-flux (SMOOTH: of eq.
// 2nd-smooth-flux) at one interface point, face frame.  Outputs: Fo[0] =
// F(dt), Fo[1] = F(dt/2) (time integrals of the flux), Wo[0] = W(0), Wo[1] =
// W(dt).
template <typename R, bool VISC, bool PRFIX, bool SMOOTH = false>
GKS_HD void gks_point(const Params &p, R dt, const R wl[5], const R gl[3][5], const R wr[5],
                      const R gr[3][5], R Fo[2][5], R Wo[2][5])
{
    PointSetup<R> S;
    point_setup<R, VISC, SMOOTH>(p, dt, wl, wr, S);
    const R Uc[3] = {S.gC.U, S.gC.V, S.gC.W};
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) Fo[k][q] = Wo[k][q] = R(0);
    R gc[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 5; ++q) gc[d][q] = R(0);
    side_terms<R, VISC, PRFIX, SMOOTH>(p, S.gL, S.l0, S.l1, gl, S.tc, Uc, gc, Fo, Wo);
    side_terms<R, VISC, PRFIX, SMOOTH>(p, S.gR, S.r0, S.r1, gr, S.tc, Uc, gc, Fo, Wo);
    equilibrium_terms<R, PRFIX, SMOOTH>(p, S.gC, S.tc, gc, Fo, Wo);
}

// Whether the face frame uses the cancellation-free form of 1/(1 + n1).
template <typename R>
struct RobustFrame {
    static constexpr bool value = false;
};
template <>
struct RobustFrame<float> {
    static constexpr bool value = true;
};

// rotation of eq. rotate-matrix-3d (Lambda when n1 = -1).  For a unit normal
// 1/(1 + n1) = (1 - n1)/(n2^2 + n3^2); in FP32 the right-hand side is used
// when n1 < 0, where 1 + n1 would cancel (normals close to -e1 are common on
// jittered meshes).  FP64 keeps the printed form.
template <typename R>
GKS_HD void rotation(const R n[3], R T[3][3])
{
    if (n[0] == R(-1)) {
        T[0][0] = R(-1); T[0][1] = R(0); T[0][2] = R(0);
        T[1][0] = R(0); T[1][1] = R(-1); T[1][2] = R(0);
        T[2][0] = R(0); T[2][1] = R(0); T[2][2] = R(1);
        return;
    }
    const R n1 = n[0], n2 = n[1], n3 = n[2];
    R ip;
    if (RobustFrame<R>::value && n1 < R(0))
        ip = (R(1) - n1) / (n2 * n2 + n3 * n3);
    else
        ip = R(1) / (R(1) + n1);
    T[0][0] = n1; T[0][1] = n2; T[0][2] = n3;
    T[1][0] = -n2; T[1][1] = n1 + n3 * n3 * ip; T[1][2] = -n2 * n3 * ip;
    T[2][0] = -n3; T[2][1] = -n2 * n3 * ip; T[2][2] = R(1) - n3 * n3 * ip;
}

// Reconstructed state and gradient of one cell at offset r from its centroid
// (coefficient k of component q from cf(q, k)), rotated into the face frame.
template <typename R, typename Coef>
GKS_HD void eval_local(const Coef &cf, const R r[3], const R T[3][3], R w[5], R g[3][5])
{
    R W[5], G[5][3];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        R c[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) c[k] = cf(q, k);
        W[q] = c[0] + c[1] * r[0] + c[2] * r[1] + c[3] * r[2] +
               R(0.5) * (c[4] * r[0] * r[0] + c[5] * r[1] * r[1] + c[6] * r[2] * r[2]) +
               c[7] * r[0] * r[1] + c[8] * r[0] * r[2] + c[9] * r[1] * r[2];
        G[q][0] = c[1] + c[4] * r[0] + c[7] * r[1] + c[8] * r[2];
        G[q][1] = c[2] + c[7] * r[0] + c[5] * r[1] + c[9] * r[2];
        G[q][2] = c[3] + c[8] * r[0] + c[9] * r[1] + c[6] * r[2];
    }
    w[0] = W[0];
    w[4] = W[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) w[1 + a] = T[a][0] * W[1] + T[a][1] * W[2] + T[a][2] * W[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        R dW[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) dW[q] = T[j][0] * G[q][0] + T[j][1] * G[q][1] + T[j][2] * G[q][2];
        g[j][0] = dW[0];
        g[j][4] = dW[4];
#pragma unroll
        for (int a = 0; a < 3; ++a) g[j][1 + a] = T[a][0] * dW[1] + T[a][1] * dW[2] + T[a][2] * dW[3];
    }
}

template <typename R>
GKS_HD void to_global(const R T[3][3], const R l[5], R gout[5])
{
    gout[0] = l[0];
    gout[4] = l[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) gout[1 + a] = T[0][a] * l[1] + T[1][a] * l[2] + T[2][a] * l[3];
}

// Ghost state of a slip wall in the face frame (Sec. 4.4): the normal
// momentum is reversed; the normal derivatives are reversed except that of
// the normal momentum; of the tangential derivatives only the normal
// momentum's are reversed.  The map is its own inverse and its own transpose.
template <typename R>
GKS_HD void slip_ghost(const R w[5], const R g[3][5], R wg[5], R gg[3][5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        wg[q] = q == 1 ? -w[q] : w[q];
        gg[0][q] = q == 1 ? g[0][q] : -g[0][q];
        gg[1][q] = q == 1 ? -g[1][q] : g[1][q];
        gg[2][q] = q == 1 ? -g[2][q] : g[2][q];
    }
}

// Ghost state of a no-slip wall in the face frame (Sec. 4.4): the interior
// point state reflected through the wall point in primitive variables (T =
// p / rho): velocity 2 U_wall - U with unchanged derivatives, the same
// pressure with reversed derivatives, temperature T with reversed
// derivatives (adiabatic) or 2 T_wall - T with unchanged ones (isothermal);
// derivatives converted with the paper's chain rule.  uw is the wall
// velocity in the face frame; g[j][q] the derivative along axis j.
template <typename R>
GKS_HD void noslip_ghost(bool iso, R gamma, R Tw, const R uw[3], const R w[5], const R g[3][5], R wg[5],
                         R gg[3][5])
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
    wg[0] = rhog;
#pragma unroll
    for (int a = 0; a < 3; ++a) wg[1 + a] = rhog * Ug[a];
    wg[4] = rhog * Qg + p / g1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
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
        gg[j][0] = drg;
#pragma unroll
        for (int a = 0; a < 3; ++a) gg[j][1 + a] = drg * Ug[a] + rhog * dU[a];
        gg[j][4] = drg * Qg + rhog * dQg - dp / g1;
    }
}

// Far field in the face frame (normal e1, out of the domain): the locally
// one-dimensional characteristic state against the free stream wf (face
// frame).  Supersonic outflow: the interior state; supersonic inflow: the
// free stream; otherwise the outgoing invariant u_n + 2a/(gamma-1) from the
// interior, the incoming u_n - 2a/(gamma-1) from the free stream, entropy
// p/rho^gamma and tangential velocity from the upwind side.  Zero gradients.
template <typename R>
GKS_HD void farfield_ghost(R gamma, const R wf[5], const R w[5], R wg[5], R gg[3][5])
{
    const R g1 = gamma - R(1);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < 5; ++q) gg[j][q] = R(0);
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
    if (Ui[0] >= ai || Ui[0] <= -ai) {
        const R *src = Ui[0] >= ai ? w : wf;
#pragma unroll
        for (int q = 0; q < 5; ++q) wg[q] = src[q];
        return;
    }
    const R Rp = Ui[0] + R(2) * ai / g1, Rm = Uf[0] - R(2) * af / g1;
    const R ub = R(0.5) * (Rp + Rm), ab = R(0.25) * g1 * (Rp - Rm);
    const bool out = ub > R(0);
    const R s = out ? pi / pow(ri, gamma) : pf / pow(rf, gamma);
    const R rb = pow(ab * ab / (gamma * s), R(1) / g1), pb = rb * ab * ab / gamma;
    const R ut1 = out ? Ui[1] : Uf[1], ut2 = out ? Ui[2] : Uf[2];
    wg[0] = rb;
    wg[1] = rb * ub;
    wg[2] = rb * ut1;
    wg[3] = rb * ut2;
    wg[4] = pb / g1 + R(0.5) * rb * (ub * ub + ut1 * ut1 + ut2 * ut2);
}

// Boundary data of a wall face for the flux: its WallTag (2 slip, 3 no-slip
// adiabatic, 4 no-slip isothermal, 5 far field) and, on a no-slip wall, its
// velocity in the global frame.
template <typename R>
struct WallBC {
    int tag;
    R u[3];
};

// Terms of one Gauss point k of a face, weighted by w_k |Gamma| = |Gamma|/3:
// acc[0] = F_k, acc[1] = dF_k/dt (eq. linear-system), acc[2] = W_k(0),
// acc[3] = W_k(dt), all in the global frame.  r: the Gauss point relative to
// the owner centroid; dv: owner centroid minus the neighbour's (translated).
// On a wall face (no neighbour; cr is not evaluated) the right state is the
// ghost of the left one: the slip-wall mirror, or the no-slip reflection
// when bc says so.
// RAW: write |Gamma| w_k F_k(dt), F_k(dt/2) in place of the fitted flux and
// its time derivative (debug exports only)
template <typename R, bool VISC, bool PRFIX, typename CoefL, typename CoefR, bool SMOOTH = false, bool RAW = false>
GKS_HD void gauss_point_terms(const Params &p, R dt, const R nrm[3], R area, const R r[3], const R dv[3],
                              const CoefL &cl, const CoefR &cr, R acc[4][5], bool wall = false,
                              const WallBC<R> *bc = nullptr)
{
    const R w = area * R(1.0 / 3.0);
    R T[3][3];
    rotation(nrm, T);
    R rr[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) rr[d] = r[d] + dv[d];
    R wl[5], gl[3][5], wr[5], gr[3][5];
    eval_local(cl, r, T, wl, gl);
    R Fo[2][5], Wo[2][5];
    if (wall && bc && bc->tag == WALL_FARFIELD) {
        R wf[5];
        wf[0] = R(p.farfield[0]);
        wf[4] = R(p.farfield[4]);
#pragma unroll
        for (int a = 0; a < 3; ++a)
            wf[1 + a] = T[a][0] * R(p.farfield[1]) + T[a][1] * R(p.farfield[2]) + T[a][2] * R(p.farfield[3]);
        farfield_ghost(R(p.gamma), wf, wl, wr, gr);
    } else if (wall && bc && bc->tag != WALL_SLIP) {
        R uw[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) uw[a] = T[a][0] * bc->u[0] + T[a][1] * bc->u[1] + T[a][2] * bc->u[2];
        noslip_ghost(bc->tag == WALL_ISOTHERMAL, R(p.gamma), R(p.wall_T), uw, wl, gl, wr, gr);
    } else if (wall) {
        slip_ghost(wl, gl, wr, gr);
    } else {
        eval_local(cr, rr, T, wr, gr);
    }
    gks_point<R, VISC, PRFIX, SMOOTH>(p, dt, wl, gl, wr, gr, Fo, Wo);
    R F1[5], Fh[5], W0[5], W1[5];
    to_global(T, Fo[0], F1);
    to_global(T, Fo[1], Fh);
    to_global(T, Wo[0], W0);
    to_global(T, Wo[1], W1);
    const R idt = R(1) / dt;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (RAW) {  // the time integrals F(dt), F(dt/2) themselves, before the fit
            acc[0][q] = w * F1[q];
            acc[1][q] = w * Fh[q];
        } else {
            acc[0][q] = w * (R(4) * Fh[q] - F1[q]) * idt;
            acc[1][q] = w * R(4) * (F1[q] - R(2) * Fh[q]) * (idt * idt);
        }
        acc[2][q] = w * W0[q];
        acc[3][q] = w * W1[q];
    }
}

// All terms of one face: the sum over its three Gauss points, in order.
template <typename R, bool VISC, bool PRFIX, typename CoefL, typename CoefR, bool SMOOTH = false>
GKS_HD void face_terms(const Params &p, R dt, const R nrm[3], R area, const R rl[3][3], const R dv[3],
                       const CoefL &cl, const CoefR &cr, R acc[4][5], bool wall = false)
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[a][q] = R(0);
    for (int k = 0; k < 3; ++k) {
        R t[4][5];
        gauss_point_terms<R, VISC, PRFIX, CoefL, CoefR, SMOOTH>(p, dt, nrm, area, rl[k], dv, cl, cr, t, wall);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int q = 0; q < 5; ++q) acc[a][q] += t[a][q];
    }
}

#undef GKS_HD

}  // namespace gks
