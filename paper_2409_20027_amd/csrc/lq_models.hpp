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

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jsin(const Jet<NZ, RT> &a)
{
    const RT s = sin(a.v), c = cos(a.v);
    return jchain(a, s, c, -s);
}

template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jcos(const Jet<NZ, RT> &a)
{
    const RT s = sin(a.v), c = cos(a.v);
    return jchain(a, c, -s, -c);
}

// 1 / a: derivatives -1/a^2 and 2/a^3.
template <int NZ, typename RT>
LQK_DEV Jet<NZ, RT> jrecip(const Jet<NZ, RT> &a)
{
    const RT r = (RT)1 / a.v;
    return jchain(a, r, -r * r, (RT)2 * r * r * r);
}

// Scalar overloads, so that the models below read the same for RT and jets.
LQK_DEV double jsin(double a) { return sin(a); }
LQK_DEV double jcos(double a) { return cos(a); }
LQK_DEV double jrecip(double a) { return 1.0 / a; }
LQK_DEV float jsin(float a) { return sinf(a); }
LQK_DEV float jcos(float a) { return cosf(a); }
LQK_DEV float jrecip(float a) { return 1.0f / a; }

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
    const S s = jsin(z[1]), c = jcos(z[1]);
    const S w2 = z[3] * z[3];
    const S Dinv = jrecip(mc + mp * (s * s));
    f[0] = z[2];
    f[1] = z[3];
    f[2] = (z[4] + mp * (s * (l * w2 + g * c))) * Dinv;
    f[3] = ((RT)1 / l) * (((RT)-1 * (z[4] * c) - (mp * l) * (w2 * (c * s)) - ((mc + mp) * g) * s) * Dinv);
}

}  // namespace lqk
