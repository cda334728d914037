// The nonlinear combination of reconstruction step 2 (Secs. 4.2-4.3) for one
// cell and component, and its hand-written reverse.  Given the constrained
// least-squares fit c = (g, H) of P^2 about the centroid, the cell's own
// step-1 slopes b and its neighbours' slopes sn, it forms the indicators
// beta_0 (two-step, eq. p0-non-linear-weight), beta_1, beta_2 (eq.
// smooth-indicator in closed form), sigma, the nonlinear weights (eq.
// non-linear-weight) and R = Q0 + alpha (P^2 - Q0) + lin (P^1 - Q0) as ten
// coefficients (c0, G, H).  The reverse differentiates them as implemented:
// |x| -> sign(x) with sign(0) = 0, x^(4/3) -> (4/3) x^(1/3).
#pragma once

#include "gks_internal.h"

#include <cmath>

namespace gks {

#define GKS_HD __host__ __device__ __forceinline__

template <typename R>
GKS_HD R sign_r(R x)
{
    return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0));
}

// Intermediate values of the combination, shared by the forward and reverse.
template <typename R>
struct WenoFwd {
    R corr, beta0, beta1, beta2, b0[4], S, sig1, w0v[4], ws0, X, sig, r0, r1, r2, ws, w1n, w2n, alpha, lin;
    R HC[3][3], CH[3][3];
    int np, nn;
};

template <typename R>
GKS_HD void weno_forward(const Params &p, R Q0, const R c[9], const R C[6], R vol23, R vol43, const R b[3],
                         const R sn[4][3], const bool has[4], WenoFwd<R> &f, R Rq[10])
{
    const R eps = R(p.eps_weno), g22 = R(p.g22), g12 = R(p.g12), g02 = R(p.g02), g11 = R(p.g11);
    f.corr = -(R(0.5) * (c[3] * C[0] + c[4] * C[1] + c[5] * C[2]) + (c[6] * C[3] + c[7] * C[4] + c[8] * C[5]));
    if (!p.nonlinear) {
        Rq[0] = Q0 + f.corr;
#pragma unroll
        for (int k = 0; k < 9; ++k) Rq[1 + k] = c[k];
        return;
    }
    f.beta1 = vol23 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    const R Hm[3][3] = {{c[3], c[6], c[7]}, {c[6], c[4], c[8]}, {c[7], c[8], c[5]}};
    const R Cm[3][3] = {{C[0], C[3], C[4]}, {C[3], C[1], C[5]}, {C[4], C[5], C[2]}};
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            R t1 = R(0), t2 = R(0);
#pragma unroll
            for (int z = 0; z < 3; ++z) {
                t1 += Hm[x][z] * Cm[z][y];
                t2 += Cm[x][z] * Hm[z][y];
            }
            f.HC[x][y] = t1;
            f.CH[x][y] = t2;
        }
    R trHCH = R(0);
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) trHCH += f.HC[x][y] * Hm[y][x];
    R h2 = R(0);
#pragma unroll
    for (int k = 3; k < 9; ++k) h2 += c[k] * c[k];
    f.beta2 = vol23 * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2] + trHCH) + vol43 * h2;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        f.b0[s] = has[s] ? vol23 * (sn[s][0] * sn[s][0] + sn[s][1] * sn[s][1] + sn[s][2] * sn[s][2]) : R(0);
    f.S = R(0);
    f.np = 0;
    f.nn = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f.nn += has[j] ? 1 : 0;
#pragma unroll
        for (int k = 0; k < j; ++k)
            if (has[j] && has[k]) {
                f.S += fabs(f.b0[j] - f.b0[k]);
                ++f.np;
            }
    }
    f.sig1 = R(0);
    f.ws0 = R(0);
    f.beta0 = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) f.w0v[j] = R(0);
    if (f.nn > 0) {
        f.sig1 = f.np ? R(pow(f.S / R(f.np), R(4.0 / 3.0))) : R(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f.w0v[j] = has[j] ? R(1) + f.sig1 / (eps + f.b0[j]) : R(0);
            if (has[j]) f.ws0 += f.w0v[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (has[j]) f.beta0 += (f.w0v[j] / f.ws0) * f.b0[j];
    }
    f.X = R(0.5) * (fabs(f.beta2 - f.beta1) + fabs(f.beta2 - f.beta0));
    f.sig = R(pow(f.X, R(4.0 / 3.0)));
    f.r2 = f.sig / (eps + f.beta2);
    f.r1 = f.sig / (eps + f.beta1);
    f.r0 = f.sig / (eps + f.beta0);
    const R w2 = g22 * (R(1) + f.r2 * f.r2), w1 = g12 * (R(1) + f.r1 * f.r1), w0 = g02 * (R(1) + f.r0 * f.r0);
    f.ws = w0 + w1 + w2;
    f.w2n = w2 / f.ws;
    f.w1n = w1 / f.ws;
    f.alpha = f.w2n / g22;
    f.lin = f.w1n / g11 - f.w2n * g12 / (g22 * g11);
    Rq[0] = Q0 + f.alpha * f.corr;
#pragma unroll
    for (int d = 0; d < 3; ++d) Rq[1 + d] = f.alpha * c[d] + f.lin * b[d];
#pragma unroll
    for (int k = 3; k < 9; ++k) Rq[1 + k] = f.alpha * c[k];
}

template <typename R>
GKS_HD R cbrt_pos(R x)
{
    return x > R(0) ? R(pow(x, R(1.0 / 3.0))) : R(0);
}

// Reverse: given Rqb (adjoint of Rq), sets Q0b, cb[9], bb[3], snb[4][3].
template <typename R>
GKS_HD void weno_reverse(const Params &p, const R c[9], const R C[6], R vol23, R vol43, const R b[3],
                         const R sn[4][3], const bool has[4], const WenoFwd<R> &f, const R Rqb[10], R &Q0b,
                         R cb[9], R bb[3], R snb[4][3])
{
    const R eps = R(p.eps_weno), g22 = R(p.g22), g12 = R(p.g12), g02 = R(p.g02), g11 = R(p.g11);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) snb[s][d] = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) bb[d] = R(0);
    R corrb;
    Q0b = Rqb[0];
    if (!p.nonlinear) {
        corrb = Rqb[0];
#pragma unroll
        for (int k = 0; k < 9; ++k) cb[k] = Rqb[1 + k];
    } else {
        corrb = Rqb[0] * f.alpha;
        R alphab = Rqb[0] * f.corr, linb = R(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            alphab += Rqb[1 + d] * c[d];
            linb += Rqb[1 + d] * b[d];
            cb[d] = f.alpha * Rqb[1 + d];
            bb[d] = f.lin * Rqb[1 + d];
        }
#pragma unroll
        for (int k = 3; k < 9; ++k) {
            alphab += Rqb[1 + k] * c[k];
            cb[k] = f.alpha * Rqb[1 + k];
        }
        const R w2nb = alphab / g22 - linb * g12 / (g22 * g11);
        const R w1nb = linb / g11;
        const R wsb = -(w2nb * f.w2n + w1nb * f.w1n) / f.ws;
        const R w2b = w2nb / f.ws + wsb, w1b = w1nb / f.ws + wsb, w0b = wsb;
        const R r2b = w2b * g22 * R(2) * f.r2, r1b = w1b * g12 * R(2) * f.r1, r0b = w0b * g02 * R(2) * f.r0;
        const R sigb = r2b / (eps + f.beta2) + r1b / (eps + f.beta1) + r0b / (eps + f.beta0);
        R beta2b = -r2b * f.r2 / (eps + f.beta2);
        R beta1b = -r1b * f.r1 / (eps + f.beta1);
        R beta0b = -r0b * f.r0 / (eps + f.beta0);
        const R Xb = sigb * R(4.0 / 3.0) * cbrt_pos(f.X);
        const R s21 = sign_r(f.beta2 - f.beta1), s20 = sign_r(f.beta2 - f.beta0);
        beta2b += R(0.5) * Xb * (s21 + s20);
        beta1b -= R(0.5) * Xb * s21;
        beta0b -= R(0.5) * Xb * s20;
#pragma unroll
        for (int d = 0; d < 3; ++d) bb[d] += R(2) * vol23 * b[d] * beta1b;
#pragma unroll
        for (int d = 0; d < 3; ++d) cb[d] += R(2) * vol23 * c[d] * beta2b;
#pragma unroll
        for (int k = 3; k < 9; ++k) cb[k] += R(2) * vol43 * c[k] * beta2b;
        // d tr(HCH)/dH = HC + CH; the off-diagonal entries of H appear twice
        const R tb = vol23 * beta2b;
        cb[3] += tb * (f.HC[0][0] + f.CH[0][0]);
        cb[4] += tb * (f.HC[1][1] + f.CH[1][1]);
        cb[5] += tb * (f.HC[2][2] + f.CH[2][2]);
        cb[6] += tb * (f.HC[0][1] + f.CH[0][1] + f.HC[1][0] + f.CH[1][0]);
        cb[7] += tb * (f.HC[0][2] + f.CH[0][2] + f.HC[2][0] + f.CH[2][0]);
        cb[8] += tb * (f.HC[1][2] + f.CH[1][2] + f.HC[2][1] + f.CH[2][1]);
        // beta_0 = sum_j (w_j / ws) b0_j, w_j = 1 + sig1 / (eps + b0_j)
        R b0b[4] = {R(0), R(0), R(0), R(0)};
        if (f.nn > 0) {
            const R ws0b = -beta0b * f.beta0 / f.ws0;
            R sig1b = R(0);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (has[j]) {
                    b0b[j] += beta0b * f.w0v[j] / f.ws0;
                    const R wjb = beta0b * f.b0[j] / f.ws0 + ws0b;
                    const R e = eps + f.b0[j];
                    sig1b += wjb / e;
                    b0b[j] -= wjb * f.sig1 / (e * e);
                }
            if (f.np > 0) {
                const R Sb = sig1b * R(4.0 / 3.0) * cbrt_pos(f.S / R(f.np)) / R(f.np);
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int k = 0; k < j; ++k)
                        if (has[j] && has[k]) {
                            const R sj = sign_r(f.b0[j] - f.b0[k]);
                            b0b[j] += Sb * sj;
                            b0b[k] -= Sb * sj;
                        }
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (has[s])
#pragma unroll
                for (int d = 0; d < 3; ++d) snb[s][d] = R(2) * vol23 * sn[s][d] * b0b[s];
    }
    // corr = -(0.5 (c3 C0 + c4 C1 + c5 C2) + c6 C3 + c7 C4 + c8 C5)
    cb[3] -= R(0.5) * C[0] * corrb;
    cb[4] -= R(0.5) * C[1] * corrb;
    cb[5] -= R(0.5) * C[2] * corrb;
    cb[6] -= C[3] * corrb;
    cb[7] -= C[4] * corrb;
    cb[8] -= C[5] * corrb;
}


// ---------------------------------------------------------------------------
// Second-order scheme (eq. final_weno_expression-2nd): R = w11 p1 + w01 p0,
// p1 = (P^1 - g01 P^0) / g11, p0 = P^0, with sigma = |beta1 - beta0|^(4/3) and
// beta0 the two-step indicator.  Both polynomials have the cell mean Q0, so
// R = Q0 + alpha (P^1 - Q0) with alpha = w11 / g11: ten coefficients
// (Q0, alpha b, 0 ... 0).
template <typename R>
struct Weno2Fwd {
    R beta0, beta1, b0[4], S, sig1, w0v[4], ws0, X, r0, r1, ws, w1n, alpha;
    int np, nn;
};

template <typename R>
GKS_HD void weno2_forward(const Params &p, R Q0, R vol23, const R b[3], const R sn[4][3], const bool has[4],
                          Weno2Fwd<R> &f, R Rq[10])
{
    const R eps = R(p.eps_weno), g11 = R(p.g11), g01 = R(p.g01);
#pragma unroll
    for (int k = 4; k < 10; ++k) Rq[k] = R(0);
    Rq[0] = Q0;
    if (!p.nonlinear) {
        f.alpha = R(1);
#pragma unroll
        for (int d = 0; d < 3; ++d) Rq[1 + d] = b[d];
        return;
    }
    f.beta1 = vol23 * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
#pragma unroll
    for (int s = 0; s < 4; ++s)
        f.b0[s] = has[s] ? vol23 * (sn[s][0] * sn[s][0] + sn[s][1] * sn[s][1] + sn[s][2] * sn[s][2]) : R(0);
    f.S = R(0);
    f.np = 0;
    f.nn = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f.nn += has[j] ? 1 : 0;
#pragma unroll
        for (int k = 0; k < j; ++k)
            if (has[j] && has[k]) {
                f.S += fabs(f.b0[j] - f.b0[k]);
                ++f.np;
            }
    }
    f.sig1 = R(0);
    f.ws0 = R(0);
    f.beta0 = R(0);
#pragma unroll
    for (int j = 0; j < 4; ++j) f.w0v[j] = R(0);
    if (f.nn > 0) {
        f.sig1 = f.np ? R(pow(f.S / R(f.np), R(4.0 / 3.0))) : R(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f.w0v[j] = has[j] ? R(1) + f.sig1 / (eps + f.b0[j]) : R(0);
            if (has[j]) f.ws0 += f.w0v[j];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (has[j]) f.beta0 += (f.w0v[j] / f.ws0) * f.b0[j];
    }
    f.X = fabs(f.beta1 - f.beta0);
    const R sig = R(pow(f.X, R(4.0 / 3.0)));
    f.r1 = sig / (eps + f.beta1);
    f.r0 = sig / (eps + f.beta0);
    const R w1 = g11 * (R(1) + f.r1 * f.r1), w0 = g01 * (R(1) + f.r0 * f.r0);
    f.ws = w0 + w1;
    f.w1n = w1 / f.ws;
    f.alpha = f.w1n / g11;
#pragma unroll
    for (int d = 0; d < 3; ++d) Rq[1 + d] = f.alpha * b[d];
}

template <typename R>
GKS_HD void weno2_reverse(const Params &p, R vol23, const R b[3], const R sn[4][3], const bool has[4],
                          const Weno2Fwd<R> &f, const R Rqb[10], R &Q0b, R bb[3], R snb[4][3])
{
    const R eps = R(p.eps_weno), g11 = R(p.g11), g01 = R(p.g01);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int d = 0; d < 3; ++d) snb[s][d] = R(0);
    Q0b = Rqb[0];
    R alphab = R(0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bb[d] = f.alpha * Rqb[1 + d];
        alphab += Rqb[1 + d] * b[d];
    }
    if (!p.nonlinear) return;
    const R w1nb = alphab / g11;
    const R wsb = -w1nb * f.w1n / f.ws;
    const R w1b = w1nb / f.ws + wsb, w0b = wsb;
    const R r1b = w1b * g11 * R(2) * f.r1, r0b = w0b * g01 * R(2) * f.r0;
    const R sigb = r1b / (eps + f.beta1) + r0b / (eps + f.beta0);
    R beta1b = -r1b * f.r1 / (eps + f.beta1);
    R beta0b = -r0b * f.r0 / (eps + f.beta0);
    const R Xb = sigb * R(4.0 / 3.0) * cbrt_pos(f.X);
    const R s10 = sign_r(f.beta1 - f.beta0);
    beta1b += Xb * s10;
    beta0b -= Xb * s10;
#pragma unroll
    for (int d = 0; d < 3; ++d) bb[d] += R(2) * vol23 * b[d] * beta1b;
    R b0b[4] = {R(0), R(0), R(0), R(0)};
    if (f.nn > 0) {
        const R ws0b = -beta0b * f.beta0 / f.ws0;
        R sig1b = R(0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (has[j]) {
                b0b[j] += beta0b * f.w0v[j] / f.ws0;
                const R wjb = beta0b * f.b0[j] / f.ws0 + ws0b;
                const R e = eps + f.b0[j];
                sig1b += wjb / e;
                b0b[j] -= wjb * f.sig1 / (e * e);
            }
        if (f.np > 0) {
            const R Sb = sig1b * R(4.0 / 3.0) * cbrt_pos(f.S / R(f.np)) / R(f.np);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int k = 0; k < j; ++k)
                    if (has[j] && has[k]) {
                        const R sj = sign_r(f.b0[j] - f.b0[k]);
                        b0b[j] += Sb * sj;
                        b0b[k] -= Sb * sj;
                    }
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (has[s])
#pragma unroll
            for (int d = 0; d < 3; ++d) snb[s][d] = R(2) * vol23 * sn[s][d] * b0b[s];
}

#undef GKS_HD

}  // namespace gks
