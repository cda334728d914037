// Host-side derivative checks of the flux routines.  The templated flux of
// gks_flux.h is evaluated with a forward-mode dual number (an exact
// Jacobian-vector product), beside the hand-written reverse of
// gks_flux_adj.h (a vector-Jacobian product), on the same inputs; a test
// compares <J v, ybar> with <v, J^T ybar> and J v with finite differences.
#include "../../include/gks.h"
#include "gks_flux_adj.h"
#include "gks_params.h"
#include "gks_recon_adj.h"

#include <cmath>
#include <type_traits>

namespace {

// value and one directional derivative
struct Dual {
    double v, d;
    Dual() : v(0.0), d(0.0) {}
    Dual(double x) : v(x), d(0.0) {}
    Dual(double x, double y) : v(x), d(y) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual &operator+=(Dual &a, Dual b) { a = a + b; return a; }
inline Dual &operator-=(Dual &a, Dual b) { a = a - b; return a; }
inline Dual &operator*=(Dual &a, Dual b) { a = a * b; return a; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }
inline bool operator!=(Dual a, Dual b) { return a.v != b.v; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline Dual exp(Dual a) { const double e = std::exp(a.v); return Dual(e, a.d * e); }
inline Dual sqrt(Dual a) { const double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
// d erfc(x)/dx = -2/sqrt(pi) exp(-x^2)
inline Dual erfc(Dual a) { return Dual(std::erfc(a.v), -a.d * 1.1283791670955126 * std::exp(-a.v * a.v)); }
// sign(0) = 0, as in the reverse
inline Dual fabs(Dual a) { return a.v > 0.0 ? a : (a.v < 0.0 ? -a : Dual(0.0, 0.0)); }
// x^e for a constant exponent e
inline Dual pow(Dual a, Dual e)
{
    const double v = std::pow(a.v, e.v);
    return Dual(v, a.v > 0.0 ? e.v * std::pow(a.v, e.v - 1.0) * a.d : 0.0);
}

template <typename R>
struct ArrCoef {
    const R *c;  // [5][10]
    R operator()(int q, int k) const { return c[10 * q + k]; }
};

template <bool VISC, bool PRFIX, bool SMOOTH>
void point_check(const gks::Params &p, double dt, const double x[40], const double v[40], const double yb[20],
                 double y[20], double jv[20], double xb[40])
{
    Dual wl[5], gl[3][5], wr[5], gr[3][5];
    for (int q = 0; q < 5; ++q) {
        wl[q] = Dual(x[q], v[q]);
        wr[q] = Dual(x[20 + q], v[20 + q]);
        for (int d = 0; d < 3; ++d) {
            gl[d][q] = Dual(x[5 + 5 * d + q], v[5 + 5 * d + q]);
            gr[d][q] = Dual(x[25 + 5 * d + q], v[25 + 5 * d + q]);
        }
    }
    Dual Fo[2][5], Wo[2][5];
    gks::gks_point<Dual, VISC, PRFIX, SMOOTH>(p, Dual(dt), wl, gl, wr, gr, Fo, Wo);
    for (int k = 0; k < 2; ++k)
        for (int q = 0; q < 5; ++q) {
            y[5 * k + q] = Fo[k][q].v;
            jv[5 * k + q] = Fo[k][q].d;
            y[10 + 5 * k + q] = Wo[k][q].v;
            jv[10 + 5 * k + q] = Wo[k][q].d;
        }
    double dwl[5], dgl[3][5], dwr[5], dgr[3][5], Fob[2][5], Wob[2][5];
    for (int q = 0; q < 5; ++q) {
        dwl[q] = x[q];
        dwr[q] = x[20 + q];
        for (int d = 0; d < 3; ++d) {
            dgl[d][q] = x[5 + 5 * d + q];
            dgr[d][q] = x[25 + 5 * d + q];
        }
        for (int k = 0; k < 2; ++k) {
            Fob[k][q] = yb[5 * k + q];
            Wob[k][q] = yb[10 + 5 * k + q];
        }
    }
    double wlb[5] = {0}, glb[3][5] = {{0}}, wrb[5] = {0}, grb[3][5] = {{0}};
    gks::gks_point_vjp<double, VISC, PRFIX, SMOOTH>(p, dt, dwl, dgl, dwr, dgr, Fob, Wob, wlb, glb, wrb, grb);
    for (int q = 0; q < 5; ++q) {
        xb[q] = wlb[q];
        xb[20 + q] = wrb[q];
        for (int d = 0; d < 3; ++d) {
            xb[5 + 5 * d + q] = glb[d][q];
            xb[25 + 5 * d + q] = grb[d][q];
        }
    }
}

template <bool VISC, bool PRFIX, bool SMOOTH>
void face_check(const gks::Params &p, double dt, const double geo[10], const double coef[100],
                const double v[100], const double ab[20], double acc[20], double jv[20], double cb[100])
{
    Dual nrm[3], r[3], dv[3], cd[100];
    for (int d = 0; d < 3; ++d) {
        nrm[d] = Dual(geo[d]);
        r[d] = Dual(geo[4 + d]);
        dv[d] = Dual(geo[7 + d]);
    }
    for (int k = 0; k < 100; ++k) cd[k] = Dual(coef[k], v[k]);
    Dual t[4][5];
    gks::gauss_point_terms<Dual, VISC, PRFIX, ArrCoef<Dual>, ArrCoef<Dual>, SMOOTH>(
        p, Dual(dt), nrm, Dual(geo[3]), r, dv, ArrCoef<Dual>{cd}, ArrCoef<Dual>{cd + 50}, t);
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 5; ++q) {
            acc[5 * a + q] = t[a][q].v;
            jv[5 * a + q] = t[a][q].d;
        }
    double nn[3], rr[3], dd[3], accb[4][5], cbl[5][10] = {{0}}, cbr[5][10] = {{0}};
    for (int d = 0; d < 3; ++d) {
        nn[d] = geo[d];
        rr[d] = geo[4 + d];
        dd[d] = geo[7 + d];
    }
    for (int a = 0; a < 4; ++a)
        for (int q = 0; q < 5; ++q) accb[a][q] = ab[5 * a + q];
    gks::gauss_point_terms_vjp<double, VISC, PRFIX, ArrCoef<double>, ArrCoef<double>, SMOOTH>(
        p, dt, nn, geo[3], rr, dd, ArrCoef<double>{coef}, ArrCoef<double>{coef + 50}, accb, cbl, cbr);
    for (int q = 0; q < 5; ++q)
        for (int k = 0; k < 10; ++k) {
            cb[10 * q + k] = cbl[q][k];
            cb[50 + 10 * q + k] = cbr[q][k];
        }
}

// calls f(VISC, PRFIX, SMOOTH) with the flags as std::integral_constant values
template <bool SMOOTH, typename F>
void dispatch_visc_prfix(bool visc, bool prfix, F &&f)
{
    using T = std::true_type;
    using N = std::false_type;
    using S = std::integral_constant<bool, SMOOTH>;
    if (visc && prfix) f(T{}, T{}, S{});
    else if (visc) f(T{}, N{}, S{});
    else if (prfix) f(N{}, T{}, S{});
    else f(N{}, N{}, S{});
}

}  // namespace

extern "C" gks_status gks_flux_point_check(const gks_config *cfg, double dt, const double x[40],
                                           const double v[40], const double ybar[20], double y[20],
                                           double jv[20], double xbar[40])
{
    if (!cfg || !x || !v || !ybar || !y || !jv || !xbar || !(dt > 0.0)) return GKS_E_INVAL;
    const gks::Params p = gks::params_from_config(cfg);
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    if (p.flux == gks::FLUX_KIND_SMOOTH)
        dispatch_visc_prfix<true>(visc, prfix, [&](auto v_, auto f_, auto s_) {
            point_check<decltype(v_)::value, decltype(f_)::value, decltype(s_)::value>(p, dt, x, v, ybar, y, jv, xbar);
        });
    else
        dispatch_visc_prfix<false>(visc, prfix, [&](auto v_, auto f_, auto s_) {
            point_check<decltype(v_)::value, decltype(f_)::value, decltype(s_)::value>(p, dt, x, v, ybar, y, jv, xbar);
        });
    return GKS_OK;
}

extern "C" gks_status gks_flux_face_check(const gks_config *cfg, double dt, const double geo[10],
                                          const double coef[100], const double v[100],
                                          const double accbar[20], double acc[20], double jv[20],
                                          double coefbar[100])
{
    if (!cfg || !geo || !coef || !v || !accbar || !acc || !jv || !coefbar || !(dt > 0.0)) return GKS_E_INVAL;
    const gks::Params p = gks::params_from_config(cfg);
    const bool visc = p.viscous != 0, prfix = p.prandtl != 1.0;
    auto run = [&](auto v_, auto f_, auto s_) {
        face_check<decltype(v_)::value, decltype(f_)::value, decltype(s_)::value>(p, dt, geo, coef, v, accbar, acc,
                                                                                  jv, coefbar);
    };
    if (p.flux == gks::FLUX_KIND_SMOOTH)
        dispatch_visc_prfix<true>(visc, prfix, run);
    else
        dispatch_visc_prfix<false>(visc, prfix, run);
    return GKS_OK;
}

extern "C" gks_status gks_wall_ghost_check(const gks_config *cfg, int32_t tag, const double uw[3],
                                           const double x[20], const double v[20], const double ybar[20],
                                           double y[20], double jv[20], double xbar[20])
{
    if (!cfg || !uw || !x || !v || !ybar || !y || !jv || !xbar) return GKS_E_INVAL;
    if (tag != GKS_FACE_NOSLIP_ADIABATIC && tag != GKS_FACE_NOSLIP_ISOTHERMAL && tag != GKS_FACE_FARFIELD)
        return GKS_E_INVAL;
    const gks::Params p = gks::params_from_config(cfg);
    const bool iso = tag == GKS_FACE_NOSLIP_ISOTHERMAL, far = tag == GKS_FACE_FARFIELD;
    Dual w[5], g[3][5], wg[5], gg[3][5], u[3], wf[5];
    for (int q = 0; q < 5; ++q) {
        w[q] = Dual(x[q], v[q]);
        wf[q] = Dual(p.farfield[q]);
        for (int j = 0; j < 3; ++j) g[j][q] = Dual(x[5 + 5 * j + q], v[5 + 5 * j + q]);
    }
    for (int a = 0; a < 3; ++a) u[a] = Dual(uw[a]);
    if (far)
        gks::farfield_ghost<Dual>(Dual(p.gamma), wf, w, wg, gg);
    else
        gks::noslip_ghost<Dual>(iso, Dual(p.gamma), Dual(p.wall_T), u, w, g, wg, gg);
    for (int q = 0; q < 5; ++q) {
        y[q] = wg[q].v;
        jv[q] = wg[q].d;
        for (int j = 0; j < 3; ++j) {
            y[5 + 5 * j + q] = gg[j][q].v;
            jv[5 + 5 * j + q] = gg[j][q].d;
        }
    }
    double wd[5], gd[3][5], wgb[5], ggb[3][5], wb[5] = {0}, gbb[3][5] = {{0}};
    for (int q = 0; q < 5; ++q) {
        wd[q] = x[q];
        wgb[q] = ybar[q];
        for (int j = 0; j < 3; ++j) {
            gd[j][q] = x[5 + 5 * j + q];
            ggb[j][q] = ybar[5 + 5 * j + q];
        }
    }
    if (far)
        gks::farfield_ghost_rev<double>(p.gamma, p.farfield, wd, wgb, wb);
    else
        gks::noslip_ghost_rev<double>(iso, p.gamma, p.wall_T, uw, wd, gd, wgb, ggb, wb, gbb);
    for (int q = 0; q < 5; ++q) {
        xbar[q] = wb[q];
        for (int j = 0; j < 3; ++j) xbar[5 + 5 * j + q] = gbb[j][q];
    }
    return GKS_OK;
}

extern "C" gks_status gks_weno_check(const gks_config *cfg, const double geo[8], int32_t has_mask,
                                     const double x[25], const double v[25], const double rbar[10],
                                     double r[10], double jv[10], double xbar[25])
{
    if (!cfg || !geo || !x || !v || !rbar || !r || !jv || !xbar) return GKS_E_INVAL;
    const gks::Params p = gks::params_from_config(cfg);
    bool has[4];
    for (int s = 0; s < 4; ++s) has[s] = (has_mask >> s) & 1;
    // forward with duals
    Dual Q0(x[0], v[0]), c[9], C[6], b[3], sn[4][3];
    for (int k = 0; k < 9; ++k) c[k] = Dual(x[1 + k], v[1 + k]);
    for (int d = 0; d < 3; ++d) b[d] = Dual(x[10 + d], v[10 + d]);
    for (int s = 0; s < 4; ++s)
        for (int d = 0; d < 3; ++d) sn[s][d] = Dual(x[13 + 3 * s + d], v[13 + 3 * s + d]);
    for (int k = 0; k < 6; ++k) C[k] = Dual(geo[k]);
    Dual Rq[10];
    if (p.order == 2) {
        // the second-order combination: x[1..9] (the fit) does not enter
        gks::Weno2Fwd<Dual> f2;
        gks::weno2_forward<Dual>(p, Q0, Dual(geo[6]), b, sn, has, f2, Rq);
        double bq[3], snq[4][3], Rd[10];
        for (int d = 0; d < 3; ++d) bq[d] = x[10 + d];
        for (int s = 0; s < 4; ++s)
            for (int d = 0; d < 3; ++d) snq[s][d] = x[13 + 3 * s + d];
        gks::Weno2Fwd<double> f;
        gks::weno2_forward<double>(p, x[0], geo[6], bq, snq, has, f, Rd);
        double Q0b, bb[3], snb[4][3];
        gks::weno2_reverse<double>(p, geo[6], bq, snq, has, f, rbar, Q0b, bb, snb);
        for (int k = 0; k < 10; ++k) {
            r[k] = Rq[k].v;
            jv[k] = Rq[k].d;
        }
        xbar[0] = Q0b;
        for (int k = 0; k < 9; ++k) xbar[1 + k] = 0.0;
        for (int d = 0; d < 3; ++d) xbar[10 + d] = bb[d];
        for (int s = 0; s < 4; ++s)
            for (int d = 0; d < 3; ++d) xbar[13 + 3 * s + d] = snb[s][d];
        return GKS_OK;
    }
    gks::WenoFwd<Dual> fd;
    gks::weno_forward<Dual>(p, Q0, c, C, Dual(geo[6]), Dual(geo[7]), b, sn, has, fd, Rq);
    for (int k = 0; k < 10; ++k) {
        r[k] = Rq[k].v;
        jv[k] = Rq[k].d;
    }
    // reverse in double
    double cq[9], Cq[6], bq[3], snq[4][3], Rd[10];
    for (int k = 0; k < 9; ++k) cq[k] = x[1 + k];
    for (int d = 0; d < 3; ++d) bq[d] = x[10 + d];
    for (int s = 0; s < 4; ++s)
        for (int d = 0; d < 3; ++d) snq[s][d] = x[13 + 3 * s + d];
    for (int k = 0; k < 6; ++k) Cq[k] = geo[k];
    gks::WenoFwd<double> f;
    gks::weno_forward<double>(p, x[0], cq, Cq, geo[6], geo[7], bq, snq, has, f, Rd);
    double Q0b, cb[9], bb[3], snb[4][3];
    gks::weno_reverse<double>(p, cq, Cq, geo[6], geo[7], bq, snq, has, f, rbar, Q0b, cb, bb, snb);
    xbar[0] = Q0b;
    for (int k = 0; k < 9; ++k) xbar[1 + k] = cb[k];
    for (int d = 0; d < 3; ++d) xbar[10 + d] = bb[d];
    for (int s = 0; s < 4; ++s)
        for (int d = 0; d < 3; ++d) xbar[13 + 3 * s + d] = snb[s][d];
    return GKS_OK;
}
