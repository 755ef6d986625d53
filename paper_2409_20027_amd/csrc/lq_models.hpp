// lq_models.hpp -- right-hand sides f(x, u) of the Newton models and their
// derivatives by forward-mode differentiation.
//
// The pendulum and cart-pole of Sec. V are written once, generic in the
// scalar type.  Evaluated on a second-order jet (value, gradient and Hessian
// over z = (x, u)) they give the Jacobians of the linearisation and, for
// S = sum_i lambda_i f_i, the co-state contractions of the second
// derivatives that enter P, M and R of the expansion.
#pragma once
#include <hip/hip_runtime.h>

#include "lq_desc.hpp"

namespace lqk {

// Second-order jet over NZ variables: value, gradient and (symmetric, stored
// full) Hessian, in arithmetic type RT.
template <int NZ, typename RT>
struct Jet {
    RT v;
    RT g[NZ];
    RT H[NZ][NZ];
};

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jvar(RT v, int i)
{
    Jet<NZ, RT> a;
    a.v = v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        a.g[p] = (p == i) ? (RT)1 : (RT)0;
#pragma unroll
        for (int q = 0; q < NZ; ++q) a.H[p][q] = (RT)0;
    }
    return a;
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jconst(RT v)
{
    return jvar<NZ, RT>(v, -1);
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> operator+(const Jet<NZ, RT> &a, const Jet<NZ, RT> &b)
{
    Jet<NZ, RT> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        r.g[p] = a.g[p] + b.g[p];
#pragma unroll
        for (int q = 0; q < NZ; ++q) r.H[p][q] = a.H[p][q] + b.H[p][q];
    }
    return r;
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> operator-(const Jet<NZ, RT> &a, const Jet<NZ, RT> &b)
{
    Jet<NZ, RT> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        r.g[p] = a.g[p] - b.g[p];
#pragma unroll
        for (int q = 0; q < NZ; ++q) r.H[p][q] = a.H[p][q] - b.H[p][q];
    }
    return r;
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> operator*(RT c, const Jet<NZ, RT> &a)
{
    Jet<NZ, RT> r;
    r.v = c * a.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        r.g[p] = c * a.g[p];
#pragma unroll
        for (int q = 0; q < NZ; ++q) r.H[p][q] = c * a.H[p][q];
    }
    return r;
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> operator+(RT c, const Jet<NZ, RT> &a)
{
    Jet<NZ, RT> r = a;
    r.v = c + a.v;
    return r;
}

// Product rule: (ab)'' = a b'' + b a'' + a' b'^T + b' a'^T.
template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> operator*(const Jet<NZ, RT> &a, const Jet<NZ, RT> &b)
{
    Jet<NZ, RT> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        r.g[p] = a.v * b.g[p] + b.v * a.g[p];
#pragma unroll
        for (int q = 0; q < NZ; ++q) r.H[p][q] = a.v * b.H[p][q] + b.v * a.H[p][q] + a.g[p] * b.g[q] + b.g[p] * a.g[q];
    }
    return r;
}

// phi(a) for a scalar function with derivatives d1 = phi'(a.v), d2 = phi''(a.v):
// gradient d1 a', Hessian d1 a'' + d2 a' a'^T.
template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jchain(const Jet<NZ, RT> &a, RT v, RT d1, RT d2)
{
    Jet<NZ, RT> r;
    r.v = v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) {
        r.g[p] = d1 * a.g[p];
#pragma unroll
        for (int q = 0; q < NZ; ++q) r.H[p][q] = d1 * a.H[p][q] + d2 * a.g[p] * a.g[q];
    }
    return r;
}

// sin x and cos x in FP64: Cody-Waite reduction x = k pi/2 + r with pi/2
// split into three doubles (each k * part subtracted by one fused
// multiply-add), then the Taylor series of sin and cos on |r| <= pi/4 with
// terms to r^17 and r^16 (truncation below 1e-18 relative), and the quadrant
// k mod 4.  Accurate to about one ulp for |x| up to ~1e5; about a third of
// the dependent operations of the general library routine.
LQK_DEV void sincos_cw(double x, double &s, double &c)
{
    constexpr double P1 = 0x1.921fb54442d18p+0, P2 = 0x1.1a62633145c07p-54, P3 = -0x1.f1976b7ed8fbcp-110;
    constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
    const double k = rint(x * TWO_OVER_PI);
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    r = fma(-k, P3, r);
    const double r2 = r * r;
    // 1/n! as compile-time quotients
    constexpr double f2 = 1.0 / 2, f3 = f2 / 3, f4 = f3 / 4, f5 = f4 / 5, f6 = f5 / 6, f7 = f6 / 7, f8 = f7 / 8;
    constexpr double f9 = f8 / 9, f10 = f9 / 10, f11 = f10 / 11, f12 = f11 / 12, f13 = f12 / 13, f14 = f13 / 14;
    constexpr double f15 = f14 / 15, f16 = f15 / 16, f17 = f16 / 17;
    double ps = fma(r2, f17, -f15);
    ps = fma(r2, ps, f13);
    ps = fma(r2, ps, -f11);
    ps = fma(r2, ps, f9);
    ps = fma(r2, ps, -f7);
    ps = fma(r2, ps, f5);
    ps = fma(r2, ps, -f3);
    const double S = fma(r * r2, ps, r);
    double pc = fma(r2, f16, -f14);
    pc = fma(r2, pc, f12);
    pc = fma(r2, pc, -f10);
    pc = fma(r2, pc, f8);
    pc = fma(r2, pc, -f6);
    pc = fma(r2, pc, f4);
    pc = fma(r2, pc, -f2);
    const double C = fma(r2, pc, 1.0);
    const int q = (int)(((int64_t)k) & 3);
    s = (q == 0) ? S : (q == 1) ? C : (q == 2) ? -S : -C;
    c = (q == 0) ? C : (q == 1) ? -S : (q == 2) ? -C : S;
}

// tanh z in FP64 as e / (e + 2) with e = expm1(2|z|), sign restored at the
// end: the quotient has no cancellation for any z.  expm1 by Cody-Waite
// reduction 2|z| = k ln2 + r, |r| <= ln2 / 2 (ln2 split into two doubles),
// the Taylor series of expm1(r) to r^13 (truncation below 2e-17 relative) and
// expm1(2|z|) = 2^k expm1(r) + (2^k - 1), exact scaling by 2^k.  Within 2.5
// ulp of tanh (libm's own is about 2); |z| > 20 gives +-1, which is tanh
// rounded to FP64 there.  About a fifth of the dependent operations of the
// library routine's double-double evaluation, which matters in the
// sequential rollout of the tanh model.
LQK_DEV double tanh_em1(double z)
{
    constexpr double L1 = 0x1.62e42feep-1, L2 = 0x1.a39ef35793c76p-33;   // ln2 = L1 + L2
    constexpr double INV_LN2 = 0x1.71547652b82fep+0;
    constexpr double f2 = 1.0 / 2, f3 = f2 / 3, f4 = f3 / 4, f5 = f4 / 5, f6 = f5 / 6, f7 = f6 / 7, f8 = f7 / 8;
    constexpr double f9 = f8 / 9, f10 = f9 / 10, f11 = f10 / 11, f12 = f11 / 12, f13 = f12 / 13;
    const double a = fabs(z);
    const double y = a + a;
    const double k = rint(y * INV_LN2);
    double r = fma(-k, L1, y);
    r = fma(-k, L2, r);
    double p = fma(r, f13, f12);
    p = fma(r, p, f11);
    p = fma(r, p, f10);
    p = fma(r, p, f9);
    p = fma(r, p, f8);
    p = fma(r, p, f7);
    p = fma(r, p, f6);
    p = fma(r, p, f5);
    p = fma(r, p, f4);
    p = fma(r, p, f3);
    p = fma(r, p, f2);
    const double q = fma(r * r, p, r);
    const double s = ldexp(1.0, (int)fmin(k, 64.0));
    const double e = fma(s, q, s - 1.0);
    const double t = e / (e + 2.0);
    return copysign(a > 20.0 ? 1.0 : t, z);
}

LQK_DEV void sincos_rt(double x, double &s, double &c) { sincos_cw(x, s, c); }
LQK_DEV void sincos_rt(float x, float &s, float &c)
{
    s = sinf(x);
    c = cosf(x);
}

// sin and cos of a jet (one reduction for both).
template <int NZ, typename RT>
LQK_DEV void jsincos(const Jet<NZ, RT> &a, Jet<NZ, RT> &js, Jet<NZ, RT> &jc)
{
    RT s, c;
    sincos_rt(a.v, s, c);
    js = jchain(a, s, c, -s);
    jc = jchain(a, c, -s, -c);
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jsin(const Jet<NZ, RT> &a)
{
    RT s, c;
    sincos_rt(a.v, s, c);
    return jchain(a, s, c, -s);
}

// 1 / a: derivatives -1/a^2 and 2/a^3.
template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jrecip(const Jet<NZ, RT> &a)
{
    const RT r = (RT)1 / a.v;
    return jchain(a, r, -r * r, (RT)2 * r * r * r);
}

// Scalar overloads, so that the models below read the same for RT and jets.
LQK_DEV double jsin(double a)
{
    double s, c;
    sincos_cw(a, s, c);
    return s;
}
LQK_DEV float jsin(float a) { return sinf(a); }
LQK_DEV void jsincos(double a, double &s, double &c) { sincos_cw(a, s, c); }
LQK_DEV void jsincos(float a, float &s, float &c) { sincos_rt(a, s, c); }
LQK_DEV double jrecip(double a) { return 1.0 / a; }
LQK_DEV float jrecip(float a) { return 1.0f / a; }

// First-order forward-mode number over NZ variables (value and gradient):
// the Jacobians of the parallel rollout need no second derivatives.
template <int NZ>
struct Dual {
    double v;
    double g[NZ];
};
template <int NZ>
LQK_DEV Dual<NZ> dvar(double v, int i)
{
    Dual<NZ> a;
    a.v = v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) a.g[p] = (p == i) ? 1.0 : 0.0;
    return a;
}
template <int NZ>
LQK_DEV Dual<NZ> operator+(const Dual<NZ> &a, const Dual<NZ> &b)
{
    Dual<NZ> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) r.g[p] = a.g[p] + b.g[p];
    return r;
}
template <int NZ>
LQK_DEV Dual<NZ> operator-(const Dual<NZ> &a, const Dual<NZ> &b)
{
    Dual<NZ> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) r.g[p] = a.g[p] - b.g[p];
    return r;
}
template <int NZ>
LQK_DEV Dual<NZ> operator*(double c, const Dual<NZ> &a)
{
    Dual<NZ> r;
    r.v = c * a.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) r.g[p] = c * a.g[p];
    return r;
}
template <int NZ>
LQK_DEV Dual<NZ> operator+(double c, const Dual<NZ> &a)
{
    Dual<NZ> r = a;
    r.v = c + a.v;
    return r;
}
template <int NZ>
LQK_DEV Dual<NZ> operator*(const Dual<NZ> &a, const Dual<NZ> &b)
{
    Dual<NZ> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) r.g[p] = a.v * b.g[p] + b.v * a.g[p];
    return r;
}
template <int NZ>
LQK_DEV Dual<NZ> dchain(const Dual<NZ> &a, double v, double d1)
{
    Dual<NZ> r;
    r.v = v;
#pragma unroll
    for (int p = 0; p < NZ; ++p) r.g[p] = d1 * a.g[p];
    return r;
}
template <int NZ>
LQK_DEV void jsincos(const Dual<NZ> &a, Dual<NZ> &js, Dual<NZ> &jc)
{
    double s, c;
    sincos_cw(a.v, s, c);
    js = dchain(a, s, c);
    jc = dchain(a, c, -s);
}
template <int NZ>
LQK_DEV Dual<NZ> jsin(const Dual<NZ> &a)
{
    double s, c;
    sincos_cw(a.v, s, c);
    return dchain(a, s, c);
}
template <int NZ>
LQK_DEV Dual<NZ> jrecip(const Dual<NZ> &a)
{
    const double r = 1.0 / a.v;
    return dchain(a, r, -r * r);
}

// Pendulum (Sec. V): z = (theta, omega, tau), prm = (g, l, m, b);
// f = (omega, -(g/l) sin theta + (tau - b omega) / (m l^2)).
template <typename S, typename RT>
LQK_DEV void pendulum_f(const RT *prm, const S *z, S *f)
{
    const RT g = prm[0], l = prm[1], m = prm[2], b = prm[3];
    const RT inv_ml2 = (RT)1 / (m * l * l);
    f[0] = z[1];
    f[1] = (-g / l) * jsin(z[0]) + inv_ml2 * (z[2] - b * z[1]);
}

// Cart-pole (Sec. V, textbook form): z = (p, theta, v, omega, F),
// prm = (g, l, m_c, m_p); with s = sin theta, c = cos theta, D = m_c + m_p s^2:
//   p''     = (F + m_p s (l omega^2 + g c)) / D,
//   theta'' = (-F c - m_p l omega^2 c s - (m_c + m_p) g s) / (l D).
template <typename S, typename RT>
LQK_DEV void cartpole_f(const RT *prm, const S *z, S *f)
{
    const RT g = prm[0], l = prm[1], mc = prm[2], mp = prm[3];
    S s, c;
    jsincos(z[1], s, c);
    const S w2 = z[3] * z[3];
    const S Dinv = jrecip(mc + mp * (s * s));
    f[0] = z[2];
    f[1] = z[3];
    f[2] = (z[4] + mp * (s * (l * w2 + g * c))) * Dinv;
    f[3] = ((RT)1 / l) * (((RT)-1 * (z[4] * c) - (mp * l) * (w2 * (c * s)) - ((mc + mp) * g) * s) * Dinv);
}

}  // namespace lqk
