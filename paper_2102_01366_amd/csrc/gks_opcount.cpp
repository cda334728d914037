// Algorithmic operation count of the flux kernel: the face routine of
// gks_flux.h is run on the host with a scalar that counts every add/subtract,
// multiply, divide and special function (exp, erfc, sqrt) it performs.
// Negation, fabs and comparisons are not counted.  The count depends only on
// the branches the configuration selects (viscous slopes, Prandtl number).
#include "../../include/gks.h"
#include "gks_flux.h"
#include "gks_params.h"

#include <cmath>
#include <cstdint>

namespace {

struct Tally {
    uint64_t add = 0, mul = 0, div = 0, special = 0;
};
thread_local Tally tally;

struct Cnt {
    double v;
    Cnt() : v(0.0) {}
    Cnt(double x) : v(x) {}
};

inline Cnt operator+(Cnt a, Cnt b) { ++tally.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++tally.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++tally.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++tally.div; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt &operator+=(Cnt &a, Cnt b) { a = a + b; return a; }
inline Cnt &operator-=(Cnt &a, Cnt b) { a = a - b; return a; }
inline Cnt &operator*=(Cnt &a, Cnt b) { a = a * b; return a; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline Cnt pow(Cnt a, Cnt b) { ++tally.special; return Cnt(std::pow(a.v, b.v)); }
inline Cnt exp(Cnt a) { ++tally.special; return Cnt(std::exp(a.v)); }
inline Cnt erfc(Cnt a) { ++tally.special; return Cnt(std::erfc(a.v)); }
inline Cnt sqrt(Cnt a) { ++tally.special; return Cnt(std::sqrt(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }

struct HostCoef {
    const double *c;  // [5][10]
    Cnt operator()(int q, int k) const { return Cnt(c[10 * q + k]); }
};

}  // namespace

extern "C" gks_status gks_flux_op_count(const gks_config *cfg, double counts[4])
{
    if (!cfg || !counts) return GKS_E_INVAL;
    const gks::Params p = gks::params_from_config(cfg);
    // a generic face: unit normal away from the coordinate axes, two
    // different physical states with gradients
    double cl[50], cr[50];
    const double base[5] = {1.1, 0.2, -0.1, 0.15, 2.9};
    for (int q = 0; q < 5; ++q)
        for (int k = 0; k < 10; ++k) {
            cl[10 * q + k] = k == 0 ? base[q] : 0.01 * (1 + q + k);
            cr[10 * q + k] = k == 0 ? base[q] * 1.05 : -0.012 * (1 + q + k);
        }
    const double nn[3] = {0.48, -0.6, 0.64};
    Cnt nrm[3] = {Cnt(nn[0]), Cnt(nn[1]), Cnt(nn[2])};
    Cnt rl[3][3], dv[3];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) rl[k][d] = Cnt(0.01 * (k + 1) - 0.003 * d);
    for (int d = 0; d < 3; ++d) dv[d] = Cnt(0.02 + 0.001 * d);
    Cnt acc[4][5];
    tally = Tally{};
    const HostCoef L{cl}, R{cr};
    const bool sm = p.flux == gks::FLUX_KIND_SMOOTH;
    if (p.viscous && p.prandtl != 1.0)
        sm ? gks::face_terms<Cnt, true, true, HostCoef, HostCoef, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc)
           : gks::face_terms<Cnt, true, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc);
    else if (p.viscous)
        sm ? gks::face_terms<Cnt, true, false, HostCoef, HostCoef, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc)
           : gks::face_terms<Cnt, true, false>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc);
    else if (p.prandtl != 1.0)
        sm ? gks::face_terms<Cnt, false, true, HostCoef, HostCoef, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc)
           : gks::face_terms<Cnt, false, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc);
    else
        sm ? gks::face_terms<Cnt, false, false, HostCoef, HostCoef, true>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc)
           : gks::face_terms<Cnt, false, false>(p, Cnt(1e-3), nrm, Cnt(0.01), rl, dv, L, R, acc);
    counts[0] = (double)tally.add;
    counts[1] = (double)tally.mul;
    counts[2] = (double)tally.div;
    counts[3] = (double)tally.special;
    return GKS_OK;
}
