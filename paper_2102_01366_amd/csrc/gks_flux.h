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
template <typename R>
struct Prim {
    R rho, U, V, W, lam;
};

template <typename R>
GKS_HD Prim<R> primitive(const R w[5], R K)
{
    Prim<R> g;
    g.rho = w[0];
    const R ir = R(1) / w[0];
    g.U = w[1] * ir;
    g.V = w[2] * ir;
    g.W = w[3] * ir;
    g.lam = (K + R(3)) * w[0] / (R(4) * (w[4] - R(0.5) * w[0] * (g.U * g.U + g.V * g.V + g.W * g.W)));
    return g;
}

// normalised moments <c^k>, k < N, of a Gaussian of mean U and variance 1/(2 lam)
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
    gauss_moments<6>(g.V, g.lam, t.v);
    gauss_moments<6>(g.W, g.lam, t.w);
    t.xi2 = K * R(0.5) / g.lam;
    t.xi4 = K * (K + R(2)) * R(0.25) / (g.lam * g.lam);
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
    const R q2 = U * U + V * V + W * W + (K + R(3)) / (R(2) * lam);
    const R R1 = b[1] - U * b[0], R2 = b[2] - V * b[0], R3 = b[3] - W * b[0];
    const R R4 = R(2) * b[4] - q2 * b[0];
    a[4] = R(4) * lam * lam / (K + R(3)) * (R4 - R(2) * U * R1 - R(2) * V * R2 - R(2) * W * R3);
    a[1] = R(2) * lam * R1 - U * a[4];
    a[2] = R(2) * lam * R2 - V * a[4];
    a[3] = R(2) * lam * R3 - W * a[4];
    a[0] = b[0] - U * a[1] - V * a[2] - W * a[3] - R(0.5) * a[4] * q2;
}

// Kinetic part of one side (u > 0 for the left state, u < 0 for the right):
// adds the slopes' contribution to the interface gradients gc, and the
// side's terms of eq. 2nd-flux to the time integrals Fo, point values Wo and
// time-integrated point values Io.
template <typename R>
GKS_HD void side_terms(const Params &p, const Prim<R> &g, const Tab<R> &Th, const R gr[3][5], R tau,
                       const R cF[2][3], const R cW[2][3], R gc[3][5], R Fo[2][5], R Wo[2][5],
                       R Io[2][5])
{
    const R K = R(p.K);
    R a[3][5];
    const R ir = R(1) / g.rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gr[d][q] * ir;
        micro_slope(g, K, b, a[d]);
        contract<0, 0, 0>(Th, a[d], g.rho, gc[d]);
    }
    // <u psi>, sum_d <u u_d (a_d.psi) psi>, and their point-value analogues
    R F0[5], F1[5] = {R(0), R(0), R(0), R(0), R(0)}, V0[5], V1[5] = {R(0), R(0), R(0), R(0), R(0)};
    psi_mom<1, 0, 0>(Th, F0);
    psi_mom<0, 0, 0>(Th, V0);
    contract<2, 0, 0>(Th, a[0], R(1), F1);
    contract<1, 1, 0>(Th, a[1], R(1), F1);
    contract<1, 0, 1>(Th, a[2], R(1), F1);
    contract<1, 0, 0>(Th, a[0], R(1), V1);
    contract<0, 1, 0>(Th, a[1], R(1), V1);
    contract<0, 0, 1>(Th, a[2], R(1), V1);
    R F2[5] = {R(0), R(0), R(0), R(0), R(0)}, V2[5] = {R(0), R(0), R(0), R(0), R(0)};
    if (tau > R(0)) {
        // A of this side from its full-space compatibility condition
        Tab<R> Tf;
        gauss_moments<7>(g.U, g.lam, Tf.u);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            Tf.v[k] = Th.v[k];
            Tf.w[k] = Th.w[k];
        }
        Tf.xi2 = Th.xi2;
        Tf.xi4 = Th.xi4;
        R B[5] = {R(0), R(0), R(0), R(0), R(0)}, A[5];
        contract<1, 0, 0>(Tf, a[0], R(-1), B);
        contract<0, 1, 0>(Tf, a[1], R(-1), B);
        contract<0, 0, 1>(Tf, a[2], R(-1), B);
        micro_slope(g, K, B, A);
        contract<1, 0, 0>(Th, A, R(1), F2);
        contract<0, 0, 0>(Th, A, R(1), V2);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Fo[k][q] += g.rho * (cF[k][0] * F0[q] + cF[k][1] * F1[q] + cF[k][2] * F2[q]);
            Wo[k][q] += g.rho * (cW[k][0] * V0[q] + cW[k][1] * V1[q] + cW[k][2] * V2[q]);
            Io[k][q] += g.rho * (cF[k][0] * V0[q] + cF[k][1] * V1[q] + cF[k][2] * V2[q]);
        }
}

// Time-dependent distribution of eq. 2nd-flux at one interface point, face
// frame.  Outputs: Fo[0] = F(dt), Fo[1] = F(dt/2) (time integrals of the
// flux), Wo[0] = W(0), Wo[1] = W(dt).
template <typename R>
GKS_HD void gks_point(const Params &p, R dt, const R wl[5], const R gl[3][5], const R wr[5],
                      const R gr[3][5], R Fo[2][5], R Wo[2][5])
{
    const R K = R(p.K);
    const Prim<R> gL = primitive(wl, K), gR = primitive(wr, K);
    Tab<R> TL, TR;
    half_moments<7>(gL.U, gL.lam, true, TL.u);
    vw_tables(gL, K, TL);
    half_moments<7>(gR.U, gR.lam, false, TR.u);
    vw_tables(gR, K, TR);
    // eq. new-equ-part: W^c from the two half Maxwellians
    R Wc[5], t[5];
    psi_mom<0, 0, 0>(TL, Wc);
    psi_mom<0, 0, 0>(TR, t);
#pragma unroll
    for (int q = 0; q < 5; ++q) Wc[q] = gL.rho * Wc[q] + gR.rho * t[q];
    const Prim<R> gC = primitive(Wc, K);
    // collision times (Sec. 2.2)
    const R pl = gL.rho * R(0.5) / gL.lam, pr = gR.rho * R(0.5) / gR.lam, pc = gC.rho * R(0.5) / gC.lam;
    const R jump = R(p.c_tau) * fabs((pl - pr) / (pl + pr)) * dt;
    R tau, taun;
    if (p.viscous) {
        tau = R(p.mu) / pc;
        taun = R(p.mu) / pc + jump;
    } else {
        tau = R(0);
        taun = R(p.eps_tau) * dt + jump;
    }
    // time integrals over [0, delta] of the coefficients of eq. 2nd-flux (tau_n
    // in the exponentials, tau elsewhere) for delta = dt, dt/2, and the point
    // coefficients at t = 0, dt
    R cF[2][6], cW[2][6];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const R del = k == 0 ? dt : R(0.5) * dt;
        const R e = exp(-del / taun);
        const R E1 = taun * (R(1) - e);
        const R E2 = taun * taun * (R(1) - e) - taun * del * e;
        cF[k][0] = del - E1;
        cF[k][1] = E2 + tau * E1 - tau * del;
        cF[k][2] = R(0.5) * del * del - tau * del + tau * E1;
        cF[k][3] = E1;
        cF[k][4] = -(tau * E1 + E2);
        cF[k][5] = -tau * E1;
        const R tt = k == 0 ? R(0) : dt;
        const R et = k == 0 ? R(1) : exp(-tt / taun);
        cW[k][0] = R(1) - et;
        cW[k][1] = (tt + tau) * et - tau;
        cW[k][2] = tt - tau + tau * et;
        cW[k][3] = et;
        cW[k][4] = -(tau + tt) * et;
        cW[k][5] = -tau * et;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Fo[k][q] = R(0);
            Wo[k][q] = R(0);
        }
    R Io[2][5]; // time integrals of W(t), for the Prandtl correction
    R gc[3][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        Io[0][q] = Io[1][q] = R(0);
        gc[0][q] = gc[1][q] = gc[2][q] = R(0);
    }
    {
        const R cFk[2][3] = {{cF[0][3], cF[0][4], cF[0][5]}, {cF[1][3], cF[1][4], cF[1][5]}};
        const R cWk[2][3] = {{cW[0][3], cW[0][4], cW[0][5]}, {cW[1][3], cW[1][4], cW[1][5]}};
        side_terms(p, gL, TL, gl, tau, cFk, cWk, gc, Fo, Wo, Io);
        side_terms(p, gR, TR, gr, tau, cFk, cWk, gc, Fo, Wo, Io);
    }
    // equilibrium part: g^c, its slopes a^c and A^c
    Tab<R> TC;
    gauss_moments<7>(gC.U, gC.lam, TC.u);
    vw_tables(gC, K, TC);
    R ac[3][5];
    const R irc = R(1) / gC.rho;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R b[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) b[q] = gc[d][q] * irc;
        micro_slope(gC, K, b, ac[d]);
    }
    R Bc[5] = {R(0), R(0), R(0), R(0), R(0)}, nB[5], Ac[5];
    contract<1, 0, 0>(TC, ac[0], R(1), Bc);
    contract<0, 1, 0>(TC, ac[1], R(1), Bc);
    contract<0, 0, 1>(TC, ac[2], R(1), Bc);
#pragma unroll
    for (int q = 0; q < 5; ++q) nB[q] = -Bc[q];
    micro_slope(gC, K, nB, Ac);
    R F0[5], F1[5] = {R(0), R(0), R(0), R(0), R(0)}, F2[5] = {R(0), R(0), R(0), R(0), R(0)}, V0[5],
             V2[5] = {R(0), R(0), R(0), R(0), R(0)};
    psi_mom<1, 0, 0>(TC, F0);
    psi_mom<0, 0, 0>(TC, V0);
    contract<2, 0, 0>(TC, ac[0], R(1), F1);
    contract<1, 1, 0>(TC, ac[1], R(1), F1);
    contract<1, 0, 1>(TC, ac[2], R(1), F1);
    contract<1, 0, 0>(TC, Ac, R(1), F2);
    contract<0, 0, 0>(TC, Ac, R(1), V2);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Fo[k][q] += gC.rho * (cF[k][0] * F0[q] + cF[k][1] * F1[q] + cF[k][2] * F2[q]);
            Wo[k][q] += gC.rho * (cW[k][0] * V0[q] + cW[k][1] * Bc[q] + cW[k][2] * V2[q]);
            Io[k][q] += gC.rho * (cF[k][0] * V0[q] + cF[k][1] * Bc[q] + cF[k][2] * V2[q]);
        }
    if (p.prandtl != 1.0) {
        // heat flux about U^c of the time-integrated distribution, from the
        // integrated flux and state: (u-U)((u-U)^2 + (v-V)^2 + (w-W)^2 + xi^2)/2
        const R U = gC.U, V = gC.V, W = gC.W, U2 = U * U + V * V + W * W;
        const R fac = R(1.0 / p.prandtl - 1.0);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const R *F = Fo[k], *I = Io[k];
            const R q = F[4] - U * F[1] - V * F[2] - W * F[3] + (R(0.5) * U2 + U * U) * F[0] -
                        U * I[4] + U * V * I[2] + U * W * I[3] - R(0.5) * U * U2 * I[0];
            Fo[k][4] += fac * q;
        }
    }
}

// rotation of eq. rotate-matrix-3d (Lambda when n1 = -1)
template <typename R>
GKS_HD void rotation(const R n[3], R T[3][3])
{
    if (n[0] == R(-1)) {
        T[0][0] = R(-1); T[0][1] = R(0); T[0][2] = R(0);
        T[1][0] = R(0); T[1][1] = R(-1); T[1][2] = R(0);
        T[2][0] = R(0); T[2][1] = R(0); T[2][2] = R(1);
        return;
    }
    const R n1 = n[0], n2 = n[1], n3 = n[2], ip = R(1) / (R(1) + n1);
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

// All terms of one face: acc[0] = |Gamma| sum_k w_k F_k, acc[1] the same for
// dF/dt (eq. linear-system), acc[2] / acc[3] the same for W_k(0) / W_k(dt).
// rl[k]: Gauss point k relative to the owner centroid; dv: owner centroid
// minus the neighbour's (translated) centroid.
template <typename R, typename CoefL, typename CoefR>
GKS_HD void face_terms(const Params &p, R dt, const R nrm[3], R area, const R rl[3][3], const R dv[3],
                       const CoefL &cl, const CoefR &cr, R acc[4][5])
{
    const R w = area * R(1.0 / 3.0);
    R T[3][3];
    rotation(nrm, T);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[a][q] = R(0);
    const R idt = R(1) / dt;
    for (int k = 0; k < 3; ++k) {
        R rr[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) rr[d] = rl[k][d] + dv[d];
        R wl[5], gl[3][5], wr[5], gr[3][5];
        eval_local(cl, rl[k], T, wl, gl);
        eval_local(cr, rr, T, wr, gr);
        R Fo[2][5], Wo[2][5];
        gks_point(p, dt, wl, gl, wr, gr, Fo, Wo);
        R F1[5], Fh[5], W0[5], W1[5];
        to_global(T, Fo[0], F1);
        to_global(T, Fo[1], Fh);
        to_global(T, Wo[0], W0);
        to_global(T, Wo[1], W1);
        // eq. linear-system
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            acc[0][q] += w * (R(4) * Fh[q] - F1[q]) * idt;
            acc[1][q] += w * R(4) * (F1[q] - R(2) * Fh[q]) * (idt * idt);
            acc[2][q] += w * W0[q];
            acc[3][q] += w * W1[q];
        }
    }
}

#undef GKS_HD

}  // namespace gks
