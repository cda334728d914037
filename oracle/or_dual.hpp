/*
 * or_dual.hpp -- test infrastructure, not part of the product.
 *
 * Forward-mode dual numbers for the tangent build of the oracle
 * (gks_oracle.c compiled as C++ with OR_TANGENT): a value and OR_NDIR
 * directional derivatives carried through every operation by the chain rule,
 * so that one run of the oracle yields the exact Jacobian-vector products of
 * its step map along OR_NDIR directions at once.
 *
 * Derivative conventions at the points where the map is not differentiable
 * (the same ones the library's discrete adjoint takes): d|x| = sign(x) dx
 * with sign(0) = 0; d(x^p) = p x^(p-1) dx, which is 0 at x = 0 for p > 1;
 * comparisons and branches look at the value only.
 *
 * A dual converts implicitly from double and int, never back: every place
 * where a value that depends on the state would flow into a plain double is
 * a compile error, so the tangent build cannot silently drop a derivative.
 */
#ifndef OR_DUAL_HPP
#define OR_DUAL_HPP

#include <cmath>

#ifndef OR_NDIR
#define OR_NDIR 16
#endif

struct or_dual {
    double v;
    double d[OR_NDIR];
    /* uninitialised like a plain double (the oracle declares large arrays of
     * polynomial terms and fills only what it uses) */
    or_dual() = default;
    or_dual(double x) : v(x)
    {
        for (int k = 0; k < OR_NDIR; ++k) d[k] = 0.0;
    }
    or_dual(int x) : or_dual((double)x) {}
    or_dual &operator+=(const or_dual &b)
    {
        v += b.v;
        for (int k = 0; k < OR_NDIR; ++k) d[k] += b.d[k];
        return *this;
    }
    or_dual &operator-=(const or_dual &b)
    {
        v -= b.v;
        for (int k = 0; k < OR_NDIR; ++k) d[k] -= b.d[k];
        return *this;
    }
    or_dual &operator*=(const or_dual &b)
    {
        for (int k = 0; k < OR_NDIR; ++k) d[k] = d[k] * b.v + v * b.d[k];
        v *= b.v;
        return *this;
    }
    or_dual &operator/=(const or_dual &b)
    {
        double q = v / b.v;
        for (int k = 0; k < OR_NDIR; ++k) d[k] = (d[k] - q * b.d[k]) / b.v;
        v = q;
        return *this;
    }
};

/* scale and shift: y = a x + c with the derivative a dx */
static inline or_dual or_affine(const or_dual &x, double a, double c)
{
    or_dual r;
    r.v = a * x.v + c;
    for (int k = 0; k < OR_NDIR; ++k) r.d[k] = a * x.d[k];
    return r;
}
/* a function of one variable: value f, derivative fp at x */
static inline or_dual or_chain(const or_dual &x, double f, double fp)
{
    or_dual r;
    r.v = f;
    for (int k = 0; k < OR_NDIR; ++k) r.d[k] = fp * x.d[k];
    return r;
}

static inline or_dual operator+(or_dual a, const or_dual &b) { return a += b; }
static inline or_dual operator-(or_dual a, const or_dual &b) { return a -= b; }
static inline or_dual operator*(or_dual a, const or_dual &b) { return a *= b; }
static inline or_dual operator/(or_dual a, const or_dual &b) { return a /= b; }
static inline or_dual operator+(const or_dual &a, double b) { return or_affine(a, 1.0, b); }
static inline or_dual operator+(double a, const or_dual &b) { return or_affine(b, 1.0, a); }
static inline or_dual operator-(const or_dual &a, double b) { return or_affine(a, 1.0, -b); }
static inline or_dual operator-(double a, const or_dual &b) { return or_affine(b, -1.0, a); }
static inline or_dual operator*(const or_dual &a, double b) { return or_affine(a, b, 0.0); }
static inline or_dual operator*(double a, const or_dual &b) { return or_affine(b, a, 0.0); }
static inline or_dual operator/(const or_dual &a, double b)
{
    or_dual r;
    r.v = a.v / b;
    for (int k = 0; k < OR_NDIR; ++k) r.d[k] = a.d[k] / b;
    return r;
}
static inline or_dual operator/(double a, const or_dual &b) { return or_chain(b, a / b.v, -a / (b.v * b.v)); }
static inline or_dual operator-(const or_dual &a) { return or_affine(a, -1.0, 0.0); }
static inline or_dual operator+(const or_dual &a) { return a; }

static inline bool operator<(const or_dual &a, const or_dual &b) { return a.v < b.v; }
static inline bool operator>(const or_dual &a, const or_dual &b) { return a.v > b.v; }
static inline bool operator<=(const or_dual &a, const or_dual &b) { return a.v <= b.v; }
static inline bool operator>=(const or_dual &a, const or_dual &b) { return a.v >= b.v; }
static inline bool operator==(const or_dual &a, const or_dual &b) { return a.v == b.v; }
static inline bool operator!=(const or_dual &a, const or_dual &b) { return a.v != b.v; }

static inline or_dual sqrt(const or_dual &x)
{
    double s = std::sqrt(x.v);
    return or_chain(x, s, 0.5 / s);
}
static inline or_dual exp(const or_dual &x)
{
    double e = std::exp(x.v);
    return or_chain(x, e, e);
}
/* erfc'(x) = -(2 / sqrt(pi)) exp(-x^2) */
static inline or_dual erfc(const or_dual &x)
{
    return or_chain(x, std::erfc(x.v), -2.0 / std::sqrt(M_PI) * std::exp(-x.v * x.v));
}
static inline or_dual fabs(const or_dual &x)
{
    double s = x.v > 0.0 ? 1.0 : (x.v < 0.0 ? -1.0 : 0.0);
    return or_chain(x, std::fabs(x.v), s);
}
static inline or_dual pow(const or_dual &x, double p)
{
    double f = std::pow(x.v, p);
    double fp = p == 0.0 ? 0.0 : p * std::pow(x.v, p - 1.0);
    return or_chain(x, f, fp);
}

#endif
