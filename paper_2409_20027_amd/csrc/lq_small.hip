// lq_small.hip -- the LQ solve for small state dimensions (n <= 4) on gfx950:
// one lane per segment (the sweeps) or per scan entry (the scan levels), every
// matrix of an element in registers, sizes N = n and M = m fixed at compile
// time.
//
// At n <= 4 a value element (A, b, C, eta, J) of eq:value-fun-elements is at
// most 4 x 4, and the 16 x 16 matrix-core tiles of the general path would be
// mostly padding, with one wave's dependent instruction chain per stage.  Here a
// wave carries 64 segments (or scan entries) side by side, each lane running the
// same recursions in plain FP64 vector arithmetic:
//   k_small_value_fold     fold of a segment right to left (fused element build
//                          of eq:value-fun-elem-init, rank-m Woodbury form of
//                          eq:value-fun-param with the stage element on the left)
//   k_small_value_ks       one Kogge-Stone level of the suffix scan (the general
//                          operator eq:value-fun-param, n x n Gauss-Jordan)
//   k_small_value_riccati  Bellman steps from the segment's carry with the
//                          control law of eq:value-fun-feedback, and the
//                          composition of the segment's closed-loop maps (the
//                          elements of Alg. 3)
//   k_small_affine_ks      one level of an affine-map scan (eq:state-prop-comb-rule)
//   k_small_roll_apply     states, controls and co-states inside a segment
//   k_small_costate_fold,  the Newton step's co-state pass (segment fold of the
//   k_small_costate_apply  maps [[A', g], [0, 1]], then co-states from the scan)
// Scan entries are stored in the general path's layout (an (n+1) x (n+1)
// homogeneous block, row-major, at the start of a 256-double slot: A~ =
// [[A, b], [0, 1]], C~ = [[C, 0], [0, 0]], J~ = [[J, -eta], [-eta', c0]], affine
// maps [[F, e], [0, 1]]), so kernels of either path can follow one another on
// the same buffers.  The constant c0 of J~ never feeds S or s and is stored as 0.
// Every lane reports its own instance's failures (status word as in the general
// path: the failure at the largest stage is kept).
#include <math.h>
#include <cstdlib>

#include "lq_kernels.hpp"

namespace lqk {
namespace {

constexpr int SERR_NOT_PD = -2;
constexpr int SERR_SINGULAR = -3;
constexpr int SERR_NONFINITE = -4;

LQK_DEV void note1(bool ok, int err, int k, int &code, int &fk)
{
    const bool first = !ok && code == 0;
    code = first ? err : code;
    fk = first ? k : fk;
}

LQK_DEV void report1(int32_t *status, int inst, int code, int k)
{
    if (status) atomicMax(&status[inst], (int32_t)((-code) | (k << 8)));
}

LQK_DEV int gid() { return (int)blockIdx.x * 64 + (int)threadIdx.x; }

// ---- loads and stores of row-major blocks (nullable sources read as 0) ----

template <int R, int C>
LQK_DEV void ldm(const double *p, double (&X)[R][C])
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) X[i][j] = p ? p[i * C + j] : 0.0;
}
template <int R>
LQK_DEV void ldv(const double *p, double (&x)[R])
{
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = p ? p[i] : 0.0;
}
template <int R, int C>
LQK_DEV void stm(double *p, const double (&X)[R][C])
{
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < C; ++j) p[i * C + j] = X[i][j];
}
template <int R>
LQK_DEV void stv(double *p, const double (&x)[R])
{
#pragma unroll
    for (int i = 0; i < R; ++i) p[i] = x[i];
}

// ---- homogeneous entries (compact (N+1) x (N+1) blocks) ----

// A~ = [[A, b], [0, 1]]
template <int N>
LQK_DEV void load_map(const double *p, double (&F)[N][N], double (&e)[N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) F[i][j] = p[i * N1 + j];
        e[i] = p[i * N1 + N];
    }
}
template <int N>
LQK_DEV void store_map(double *p, const double (&F)[N][N], const double (&e)[N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) p[i * N1 + j] = F[i][j];
        p[i * N1 + N] = e[i];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) p[N * N1 + j] = 0.0;
    p[N * N1 + N] = 1.0;
}
// C~ = [[C, 0], [0, 0]]
template <int N>
LQK_DEV void load_c(const double *p, double (&C)[N][N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) C[i][j] = p[i * N1 + j];
}
template <int N>
LQK_DEV void store_c(double *p, const double (&C)[N][N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N1; ++i)
#pragma unroll
        for (int j = 0; j < N1; ++j) p[i * N1 + j] = (i < N && j < N) ? C[i][j] : 0.0;
}
// J~ = [[J, v], [v', 0]] with v = -eta (value functions: S~ = [[S, s], [s', 0]])
template <int N>
LQK_DEV void load_jv(const double *p, double (&J)[N][N], double (&v)[N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) J[i][j] = p[i * N1 + j];
        v[i] = p[i * N1 + N];
    }
}
template <int N>
LQK_DEV void store_jv(double *p, const double (&J)[N][N], const double (&v)[N])
{
    constexpr int N1 = N + 1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) p[i * N1 + j] = J[i][j];
        p[i * N1 + N] = v[i];
        p[N * N1 + i] = v[i];
    }
    p[N * N1 + N] = 0.0;
}

template <int N>
LQK_DEV void sym(double (&S)[N][N])
{
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            const double a = 0.5 * (S[i][j] + S[j][i]);
            S[i][j] = a;
            S[j][i] = a;
        }
}

// ---- small inverses ----

// Inverse of an R x R matrix by Gauss-Jordan elimination on [X | I] with
// partial pivoting (rows exchanged by selects); false for a zero or
// non-finite pivot.
template <int R>
LQK_DEV bool inv_gj(const double (&X)[R][R], double (&Y)[R][R])
{
    double a[R][2 * R];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            a[i][j] = X[i][j];
            a[i][R + j] = (i == j) ? 1.0 : 0.0;
        }
    bool ok = true;
#pragma unroll
    for (int p = 0; p < R; ++p) {
#pragma unroll
        for (int i = p + 1; i < R; ++i) {
            const bool sw = fabs(a[i][p]) > fabs(a[p][p]);
#pragma unroll
            for (int j = p; j < 2 * R; ++j) {
                const double t = a[p][j];
                a[p][j] = sw ? a[i][j] : t;
                a[i][j] = sw ? t : a[i][j];
            }
        }
        const double piv = a[p][p];
        ok = ok && (piv != 0.0) && isfinite(piv);
        const double r = 1.0 / piv;
#pragma unroll
        for (int j = p; j < 2 * R; ++j) a[p][j] *= r;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i == p) continue;
            const double f = a[i][p];
#pragma unroll
            for (int j = p; j < 2 * R; ++j) a[i][j] -= f * a[p][j];
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) Y[i][j] = a[i][R + j];
    return ok;
}

// Inverse of a symmetric R x R matrix through its Cholesky factor X = L L';
// false unless X is positive definite (a non-positive or NaN pivot).  A
// non-positive pivot is replaced by 1 so that the result stays finite; a NaN
// one is kept, so that a NaN in X reaches the inverse (and the value function
// downstream, where it is reported as non-finite at its stage).
template <int R>
LQK_DEV bool inv_spd(const double (&X)[R][R], double (&Y)[R][R])
{
    double L[R][R], id[R];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        double sj = X[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) sj -= L[j][k] * L[j][k];
        ok = ok && (sj > 0.0);
        const double dj = sqrt((sj > 0.0 || isnan(sj)) ? sj : 1.0);
        id[j] = 1.0 / dj;
        L[j][j] = dj;
#pragma unroll
        for (int i = j + 1; i < R; ++i) {
            double t = X[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t * id[j];
        }
    }
    // W = L^{-1} (lower triangular), then Y = W'W
    double W[R][R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i < j) {
                W[i][j] = 0.0;
                continue;
            }
            double t = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int k = j; k < i; ++k) t -= L[i][k] * W[k][j];
            W[i][j] = t * id[i];
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
        for (int j = 0; j < R; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < R; ++k) t += W[k][i] * W[k][j];
            Y[i][j] = t;
        }
    return ok;
}

// ---- stage data ----

template <int N, int M>
struct Stage {
    double A[N][N], B[N][M], c[N], Q[N][N], R[M][M], q[N];
    double Mx[N][M], r[M];   // cross terms (zero when absent)
};

template <int N, int M>
LQK_DEV void load_stage(const ProbPtrs &P, const InstDesc &d, int k, Stage<N, M> &w)
{
    ldm(P.A + d.oA + (int64_t)k * N * N, w.A);
    ldm(P.B + d.oB + (int64_t)k * N * M, w.B);
    ldv(P.c ? P.c + d.oc + (int64_t)k * N : nullptr, w.c);
    ldm(P.Q + d.oA + (int64_t)k * N * N, w.Q);
    ldm(P.R + d.oR + (int64_t)k * M * M, w.R);
    ldv(P.q ? P.q + d.oc + (int64_t)k * N : nullptr, w.q);
    ldm(P.M ? P.M + d.oB + (int64_t)k * N * M : nullptr, w.Mx);
    ldv(P.r ? P.r + d.og + (int64_t)k * M : nullptr, w.r);
}

// Stages per chunk of the sweeps: a lane streams its own segment, and a
// stage of an n <= 2 array fills a fraction of a cache line, so the sweeps
// issue the loads of CH stages together, while the line is still cached,
// instead of fetching it again for each stage.
template <int N>
constexpr int sweep_chunk() { return N <= 2 ? 4 : 1; }

// The stage element of eq:value-fun-elem-init in place, for cross terms M, r:
// A - B K_M, c - B K_r, Q - M K_M, q - M K_r with [K_M, K_r] = R^{-1}[M', r]
// (C = B R^{-1} B' stays implicit: the fold uses B and R).  False if R is not
// positive definite.
template <int N, int M>
LQK_DEV bool schur_cross(Stage<N, M> &w)
{
    const auto &Mk = w.Mx;
    const auto &rk = w.r;
    double Ri[M][M];
    const bool ok = inv_spd<M>(w.R, Ri);
    double KM[M][N], Kr[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < M; ++b) t += Ri[a][b] * Mk[j][b];
            KM[a][j] = t;
        }
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < M; ++b) t += Ri[a][b] * rk[b];
        Kr[a] = t;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double ta = w.A[i][j], tq = w.Q[i][j];
#pragma unroll
            for (int a = 0; a < M; ++a) {
                ta -= w.B[i][a] * KM[a][j];
                tq -= Mk[i][a] * KM[a][j];
            }
            w.A[i][j] = ta;
            w.Q[i][j] = tq;
        }
        double tc = w.c[i], tqv = w.q[i];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            tc -= w.B[i][a] * Kr[a];
            tqv -= Mk[i][a] * Kr[a];
        }
        w.c[i] = tc;
        w.q[i] = tqv;
    }
    return ok;
}

// ---- the element of an aggregate suffix ----

template <int N>
struct Elem {
    double A[N][N], b[N], C[N][N], e[N], J[N][N];   // e = eta
};

// E <- e_k (x) E for the stage element e_k = (A, c, B R^{-1} B', -q, Q) of w
// (eq:value-fun-param with the stage on the left, in the rank-m form):
//   W = R + B'J B,  P = B'J A,  v = eta - J c,  p = B'v,  H = A^ B,
//   A^ <- A^ A - H W^{-1} P,        b^ <- A^ c + b^ + H W^{-1} p,
//   C^ <- C^ + H W^{-1} H',         eta^ <- A'v - P'W^{-1} p - q,
//   J^ <- Q + A'J A - P'W^{-1} P    (then symmetrised).
// False if W is singular.
template <int N, int M>
LQK_DEV bool fold_stage(const Stage<N, M> &w, Elem<N> &E)
{
    double JB[N][M], JA[N][N], v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) t += E.J[i][k] * w.B[k][a];
            JB[i][a] = t;
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) t += E.J[i][k] * w.A[k][j];
            JA[i][j] = t;
        }
        double t = E.e[i];
#pragma unroll
        for (int k = 0; k < N; ++k) t -= E.J[i][k] * w.c[k];
        v[i] = t;
    }
    double W[M][M], Pm[M][N], pb[M], H[N][M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
        for (int b2 = 0; b2 < M; ++b2) {
            double t = w.R[a][b2];
#pragma unroll
            for (int k = 0; k < N; ++k) t += w.B[k][a] * JB[k][b2];
            W[a][b2] = t;
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) t += JB[k][a] * w.A[k][j];
            Pm[a][j] = t;
        }
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) t += w.B[k][a] * v[k];
        pb[a] = t;
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int a = 0; a < M; ++a) {
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) t += E.A[i][k] * w.B[k][a];
            H[i][a] = t;
        }
    double Wi[M][M];
    const bool ok = inv_gj<M>(W, Wi);
    double WP[M][N], Wp[M], WH[M][N];
#pragma unroll
    for (int a = 0; a < M; ++a) {
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double t = 0.0, u = 0.0;
#pragma unroll
            for (int b2 = 0; b2 < M; ++b2) {
                t += Wi[a][b2] * Pm[b2][j];
                u += Wi[a][b2] * H[j][b2];
            }
            WP[a][j] = t;
            WH[a][j] = u;
        }
        double t = 0.0;
#pragma unroll
        for (int b2 = 0; b2 < M; ++b2) t += Wi[a][b2] * pb[b2];
        Wp[a] = t;
    }
    // b^, eta^ read the old A^, J^ only through H, v and P (formed above), so
    // every field but A^ is updated in place; J^ on its upper triangle.
    double nA[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double tb = E.b[i], te = -w.q[i];
#pragma unroll
        for (int k = 0; k < N; ++k) {
            tb += E.A[i][k] * w.c[k];
            te += w.A[k][i] * v[k];
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            tb += H[i][a] * Wp[a];
            te -= Pm[a][i] * Wp[a];
        }
        E.b[i] = tb;
        E.e[i] = te;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double ta = 0.0, tc = E.C[i][j];
#pragma unroll
            for (int k = 0; k < N; ++k) ta += E.A[i][k] * w.A[k][j];
#pragma unroll
            for (int a = 0; a < M; ++a) {
                ta -= H[i][a] * WP[a][j];
                tc += H[i][a] * WH[a][j];
            }
            nA[i][j] = ta;
            E.C[i][j] = tc;
        }
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j) {
            double tj = 0.5 * (w.Q[i][j] + w.Q[j][i]);
#pragma unroll
            for (int k = 0; k < N; ++k) tj += 0.5 * (w.A[k][i] * JA[k][j] + w.A[k][j] * JA[k][i]);
#pragma unroll
            for (int a = 0; a < M; ++a) tj -= 0.5 * (Pm[a][i] * WP[a][j] + Pm[a][j] * WP[a][i]);
            E.J[i][j] = tj;
            E.J[j][i] = tj;
            E.A[i][j] = nA[i][j];
            E.A[j][i] = nA[j][i];
        }
    return ok;
}

// ---------------------------------------------------------------------------
// Phase 1: fold of segment s >= 1 into one element at scan entry s (the last
// segment folded onto the terminal element (0, 0, 0, -q_T, Q_T)); segment 0's
// element is never read.
// ---------------------------------------------------------------------------
template <int N, int M>
__global__ __launch_bounds__(64) void k_small_value_fold(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                         const int32_t *__restrict__ seg_start, int batch, int total,
                                                         double *__restrict__ X, int32_t *status)
{
    const int gs = gid();
    if (gs >= total) return;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    if (s == 0) return;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    Elem<N> E;
    const bool last = (s == d.nseg - 1);
    double qT[N];
    ldv(P.qT ? P.qT + d.on : nullptr, qT);
    if (last) ldm(P.QT + d.oQT, E.J);
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
        for (int c = 0; c < N; ++c) {
            E.A[r][c] = (!last && r == c) ? 1.0 : 0.0;
            E.C[r][c] = 0.0;
            if (!last) E.J[r][c] = 0.0;
        }
        E.b[r] = 0.0;
        E.e[r] = last ? -qT[r] : 0.0;
    }
    const bool mr = (P.M != nullptr) || (P.r != nullptr);
    int code = 0, fk = 0;
    constexpr int CH = sweep_chunk<N>();
    for (int kb = k1 - 1; kb >= k0; kb -= CH) {
        Stage<N, M> w[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) load_stage(P, d, max(kb - j, k0), w[j]);   // past k0: stage k0 again, unused
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = kb - j;
            if (k < k0) break;
            if (mr) note1(schur_cross(w[j]), SERR_NOT_PD, k, code, fk);
            note1(fold_stage(w[j], E), SERR_SINGULAR, k, code, fk);
        }
    }
    double *o = X + (int64_t)(d.xbase + s) * 3 * TILE;
    store_map(o, E.A, E.b);
    store_c(o + TILE, E.C);
    double v[N];
#pragma unroll
    for (int r = 0; r < N; ++r) v[r] = -E.e[r];
    store_jv(o + 2 * TILE, E.J, v);
    if (code) report1(status, d.orig, code, fk);
}

// ---------------------------------------------------------------------------
// Phase 2: one Kogge-Stone level of the suffix scan, X_s <- X_s (x) X_{s+dd}
// over entries 1 .. nseg-1 (the same schedule as k_value_ks): with
// Y = (I + C1 J2)^{-1},
//   A = A2 Y A1,  b = A2 Y (b1 + C1 eta2) + b2,  C = A2 Y C1 A2' + C2,
//   eta = A1'Y'(eta2 - J2 b1) + eta1,  J = A1'Y'J2 A1 + J1;
// only (eta, J) once the right operand covers the terminal element.
// ---------------------------------------------------------------------------
// The inputs of one combine: the entry's own A~, C~, J~ and its right
// neighbour's J~ (and A~, C~ unless the neighbour covers the terminal).
template <int N>
struct KsIn {
    double A1[N][N], b1[N], C1[N][N], J1[N][N], v1[N], J2[N][N], v2[N], A2[N][N], b2[N], C2[N][N];
};
// a, bp: the entry's and its neighbour's slots, with A~, C~, J~ KS doubles
// apart (TILE in the scan buffers, (N + 1)^2 in the one-block scans' LDS).
// ks_load reads what the first part of the combine uses (the entry's A~, C~,
// J~ and the neighbour's J~); the neighbour's A~ and C~ are read by
// ks_load_ac, where they are first used (fewer live registers).
template <int N, int KS>
LQK_DEV void ks_load(const double *a, const double *bp, KsIn<N> &in)
{
    load_map(a, in.A1, in.b1);
    load_c(a + KS, in.C1);
    load_jv(a + 2 * KS, in.J1, in.v1);   // v = -eta
    load_jv(bp + 2 * KS, in.J2, in.v2);
}
template <int N, int KS>
LQK_DEV void ks_load_ac(const double *bp, KsIn<N> &in)
{
    load_map(bp, in.A2, in.b2);
    load_c(bp + KS, in.C2);
}
// First part of the combine X_s (x) X_{s+dd} (ks_part_j): Y = (I + C1 J2)^{-1}
// (ks_inv_y, from C1 and J2; false if singular) and the new (eta, J) as (Jn,
// vn = -eta) (ks_j_rest, from A1, b1, J1, v1, J2, v2).
template <int N>
LQK_DEV bool ks_inv_y(const KsIn<N> &in, double (&Y)[N][N])
{
    double X[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double t = (r == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) t += in.C1[r][k] * in.J2[k][c];
            X[r][c] = t;
        }
    return inv_gj<N>(X, Y);
}
template <int N>
LQK_DEV void ks_j_rest(const KsIn<N> &in, const double (&Y)[N][N], double (&Jn)[N][N], double (&vn)[N])
{
    // w = eta2 - J2 b1 = -(v2 + J2 b1);  Y'w;  G = J2 A1;  Y'G
    double w[N], G[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = -in.v2[r];
#pragma unroll
        for (int k = 0; k < N; ++k) t -= in.J2[r][k] * in.b1[k];
        w[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) u += in.J2[r][k] * in.A1[k][c];
            G[r][c] = u;
        }
    }
    double Yw[N], YG[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) t += Y[k][r] * w[k];
        Yw[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) u += Y[k][r] * G[k][c];
            YG[r][c] = u;
        }
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = in.v1[r];   // -eta = -(A1'Y'w + eta1)
#pragma unroll
        for (int k = 0; k < N; ++k) t -= in.A1[k][r] * Yw[k];
        vn[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = in.J1[r][c];
#pragma unroll
            for (int k = 0; k < N; ++k) u += in.A1[k][r] * YG[k][c];
            Jn[r][c] = u;
        }
    }
    sym(Jn);
}
template <int N>
LQK_DEV bool ks_part_j(const KsIn<N> &in, double (&Y)[N][N], double (&Jn)[N][N], double (&vn)[N])
{
    const bool ok = ks_inv_y<N>(in, Y);
    ks_j_rest<N>(in, Y, Jn, vn);
    return ok;
}
// Second part (ks_part_ac), when the right operand does not cover the
// terminal: YA, Y z, YC from Y and in.A1, b1, C1, v2 (ks_ac_y), then the new
// A~ and C~ (An, bn, Cn) with the neighbour's A~, C~ in.A2, b2, C2 (ks_ac_out).
template <int N>
LQK_DEV void ks_ac_y(const KsIn<N> &in, const double (&Y)[N][N], double (&YA)[N][N], double (&yz)[N],
                     double (&YC)[N][N])
{
    // YA = Y A1, y = Y (b1 + C1 eta2), YC = Y C1
    double z[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = in.b1[r];
#pragma unroll
        for (int k = 0; k < N; ++k) t -= in.C1[r][k] * in.v2[k];   // eta2 = -v2
        z[r] = t;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) t += Y[r][k] * z[k];
        yz[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = 0.0, x = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                u += Y[r][k] * in.A1[k][c];
                x += Y[r][k] * in.C1[k][c];
            }
            YA[r][c] = u;
            YC[r][c] = x;
        }
    }
}
template <int N>
LQK_DEV void ks_ac_out(const KsIn<N> &in, const double (&YA)[N][N], const double (&yz)[N], const double (&YC)[N][N],
                       double (&An)[N][N], double (&bn)[N], double (&Cn)[N][N])
{
    double T2[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        double t = in.b2[r];
#pragma unroll
        for (int k = 0; k < N; ++k) t += in.A2[r][k] * yz[k];
        bn[r] = t;
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = 0.0, x = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) {
                u += in.A2[r][k] * YA[k][c];
                x += in.A2[r][k] * YC[k][c];
            }
            An[r][c] = u;
            T2[r][c] = x;
        }
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) {
            double u = in.C2[r][c];
#pragma unroll
            for (int k = 0; k < N; ++k) u += T2[r][k] * in.A2[c][k];
            Cn[r][c] = u;
        }
    sym(Cn);
}
template <int N>
LQK_DEV void ks_part_ac(const KsIn<N> &in, const double (&Y)[N][N], double (&An)[N][N], double (&bn)[N],
                        double (&Cn)[N][N])
{
    double YA[N][N], yz[N], YC[N][N];
    ks_ac_y<N>(in, Y, YA, yz, YC);
    ks_ac_out<N>(in, YA, yz, YC, An, bn, Cn);
}

template <int N>
__global__ __launch_bounds__(64) void k_small_value_ks(const InstDesc *__restrict__ inst,
                                                       const int32_t *__restrict__ x_start, int batch, int total,
                                                       int dd, const double *__restrict__ Xin,
                                                       double *__restrict__ Xout, int32_t *status)
{
    constexpr int N1 = N + 1;
    const int gx = gid();
    if (gx >= total) return;
    const int i = find_inst(x_start, batch, gx);
    const InstDesc d = inst[i];
    const int s = gx - d.xbase;
    const int last = d.nseg - 1;
    if (s == 0 || s > last) return;
    const double *a = Xin + (int64_t)gx * 3 * TILE;
    double *o = Xout + (int64_t)gx * 3 * TILE;
    if (s + dd > last) {   // final already: carry J~ over
#pragma unroll
        for (int r = 0; r < N1 * N1; ++r) o[2 * TILE + r] = a[2 * TILE + r];
        return;
    }
    const bool b_term = (s + 2 * dd - 1 >= last);
    const double *bp = Xin + (int64_t)(gx + dd) * 3 * TILE;
    KsIn<N> in;
    double Y[N][N], Jn[N][N], vn[N];
    ks_load<N, TILE>(a, bp, in);
    const bool ok = ks_part_j<N>(in, Y, Jn, vn);
    store_jv(o + 2 * TILE, Jn, vn);
    if (!b_term) {
        ks_load_ac<N, TILE>(bp, in);
        double An[N][N], bn[N], Cn[N][N];
        ks_part_ac<N>(in, Y, An, bn, Cn);
        store_map(o, An, bn);
        store_c(o + TILE, Cn);
    }
    if (!ok) report1(status, d.orig, SERR_SINGULAR, s * d.L);
}

// Every level of the suffix scan in one workgroup, for a class whose scan has
// at most value_scan1_cap(N) entries: the entries are copied once into LDS
// (compact (N+1)^2 blocks); each level computes its two parts into registers
// from LDS, each followed by a barrier and the in-place write of its results
// (three barriers a level, in place of a launch).  The final entries are
// copied back to the entries' slots of X, in place.  Same schedule and
// arithmetic as the per-level kernel.
constexpr int SCAN1_MAX = 512;
// LDS doubles per entry of the one-block value scan: 3 (n+1)^2, made odd so
// that the lanes' entries start in different banks
constexpr int value_scan1_stride(int n) { return 3 * (n + 1) * (n + 1) | 1; }
// Entries of the one-block value scan, one thread each: within the 160 KiB of
// LDS of one workgroup (273 at n = 4) and, at n = 3, 4, below the measured
// crossover where the one compute unit's FP64 issue rate makes the levels
// slower than per-level launches spread over several (between 321 and 385
// entries at n = 3, 193 and 209 at n = 4).
constexpr int value_scan1_cap(int n)
{
    const int lds = 163840 / (8 * value_scan1_stride(n));
    const int measured = n <= 2 ? SCAN1_MAX : (n == 3 ? 352 : 200);
    return lds < measured ? lds : measured;
}
template <int N>
__global__ __launch_bounds__(SCAN1_MAX) void k_small_value_scan1(const InstDesc *__restrict__ inst,
                                                                  const int32_t *__restrict__ x_start, int batch,
                                                                  int total, int max_nseg, double *__restrict__ X,
                                                                  int32_t *status)
{
    constexpr int N1 = N + 1, KS = N1 * N1, SL = value_scan1_stride(N);
    __shared__ double sh[value_scan1_cap(N) * SL];
    const int t = threadIdx.x;
    for (int idx = t; idx < total * 3 * KS; idx += SCAN1_MAX) {
        const int e = idx / (3 * KS), r = idx - e * 3 * KS, kind = r / KS;
        sh[e * SL + r] = X[(int64_t)e * 3 * TILE + kind * TILE + (r - kind * KS)];
    }
    bool live = t < total;
    int s = 0, last = 0, orig = 0, L = 0;
    if (live) {
        const InstDesc d = inst[find_inst(x_start, batch, t)];
        s = t - d.xbase;
        last = d.nseg - 1;
        orig = d.orig;
        L = d.L;
        live = (s != 0 && s <= last);
    }
    __syncthreads();
    bool ok = true;
    for (int dd = 1; dd < max_nseg - 1; dd *= 2) {
        const bool act = live && (s + dd <= last);
        const bool ac = act && (s + 2 * dd - 1 < last);   // right operand short of the terminal
        double *me = sh + t * SL;
        const double *right = sh + (t + dd) * SL;
        // Each part computes into registers from LDS, waits for the whole
        // group's reads, then writes in place: the new J~ (read by no one in
        // the second part) before the reads of A~, C~, the new A~, C~ after.
        double Y[N][N], Jn[N][N], vn[N], v2[N];
        if (act) {
            // C~ and the neighbour's J~ first; the rest once Y is formed
            KsIn<N> in;
            load_c(me + KS, in.C1);
            load_jv(right + 2 * KS, in.J2, in.v2);
            if (!ks_inv_y<N>(in, Y)) ok = false;
            load_map(me, in.A1, in.b1);
            load_jv(me + 2 * KS, in.J1, in.v1);
            ks_j_rest<N>(in, Y, Jn, vn);
#pragma unroll
            for (int r = 0; r < N; ++r) v2[r] = in.v2[r];
        }
        __syncthreads();
        if (act) store_jv(me + 2 * KS, Jn, vn);
        double An[N][N], bn[N], Cn[N][N];
        if (ac) {
            KsIn<N> in;   // own A~, C~ read again (unchanged), the neighbour's old eta kept
            load_map(me, in.A1, in.b1);
            load_c(me + KS, in.C1);
#pragma unroll
            for (int r = 0; r < N; ++r) in.v2[r] = v2[r];
            double YA[N][N], yz[N], YC[N][N];
            ks_ac_y<N>(in, Y, YA, yz, YC);
            ks_load_ac<N, KS>(right, in);
            ks_ac_out<N>(in, YA, yz, YC, An, bn, Cn);
        }
        __syncthreads();
        if (ac) {
            store_map(me, An, bn);
            store_c(me + KS, Cn);
        }
        __syncthreads();
    }
    if (!ok) report1(status, orig, SERR_SINGULAR, s * L);
    for (int idx = t; idx < total * 3 * KS; idx += SCAN1_MAX) {
        const int e = idx / (3 * KS), r = idx - e * 3 * KS, kind = r / KS;
        X[(int64_t)e * 3 * TILE + kind * TILE + (r - kind * KS)] = sh[e * SL + r];
    }
}

// ---------------------------------------------------------------------------
// Phase 3: Bellman steps over stages k1-1 .. k0 from the carry (the scanned
// value function of entry s + 1, or the terminal cost for the last segment):
//   Q_uu = R + B'S'B,  Q_ux = M' + B'S'A,  q_u = r + B'(S'c + s'),
//   Gamma = -Q_uu^{-1} Q_ux,  gamma = -Q_uu^{-1} q_u,
//   S = sym(Q + A'S'A + Q_ux'Gamma),  s = q + A'(S'c + s') + Q_ux'gamma.
// With Yroll the sweep also composes the segment's closed-loop maps
// Phi = F~_{k1-1} ... F~_{k0}, F~ = [[A + B Gamma, c + B gamma], [0, 1]], and
// writes the rollout scan's entries (Phi at s + 1 for s < nseg - 1, the
// constant map of x0 at 0).  With ckpt the last segment of each group of
// `stride` segments stores its carry in the checkpoint (as k_value_riccati).
// ---------------------------------------------------------------------------
template <int N, int M>
__global__ __launch_bounds__(64) void k_small_value_riccati(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                            const int32_t *__restrict__ seg_start, int batch,
                                                            int total, const double *__restrict__ Xfin, ValPtrs V,
                                                            double *__restrict__ Yroll, double *__restrict__ ckpt,
                                                            int stride, int32_t *status)
{
    const int gs = gid();
    if (gs >= total) return;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const bool last = (s == d.nseg - 1);
    double S[N][N], sv[N];
    if (last) {
        ldm(P.QT + d.oQT, S);
        ldv(P.qT ? P.qT + d.on : nullptr, sv);
    } else {
        load_jv(Xfin + (int64_t)(d.xbase + s + 1) * 3 * TILE + 2 * TILE, S, sv);
    }
    if (ckpt && ((s + 1) % stride == 0 || last))
        store_jv(ckpt + (int64_t)(ckpt_slot(d, i, stride) + s / stride) * TILE, S, sv);
    int code = 0, fk = 0;
    if (last) {
        stm(V.S + d.oS + (int64_t)d.T * N * N, S);
        stv(V.s + d.os + (int64_t)d.T * N, sv);
        bool fin = true;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            fin = fin && isfinite(sv[r]);
#pragma unroll
            for (int c = 0; c < N; ++c) fin = fin && isfinite(S[r][c]);
        }
        note1(fin, SERR_NONFINITE, d.T, code, fk);
    }
    const bool mr = (P.M != nullptr) || (P.r != nullptr);
    const bool roll = (Yroll != nullptr);
    double FA[N][N], Fb[N];   // Phi = [[FA, Fb], [0, 1]]
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
        for (int c = 0; c < N; ++c) FA[r][c] = (r == c) ? 1.0 : 0.0;
        Fb[r] = 0.0;
    }
    constexpr int CH = sweep_chunk<N>();
    for (int kb = k1 - 1; kb >= k0; kb -= CH) {
        Stage<N, M> ws[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) load_stage(P, d, max(kb - j, k0), ws[j]);   // past k0: stage k0 again, unused
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = kb - j;
            if (k < k0) break;
            const Stage<N, M> &w = ws[j];
            const auto &Mk = w.Mx;
            const auto &rk = w.r;
            // Sc = S'c + s',  SA = S'A,  SB = S'B
            double Sc[N], SA[N][N], SB[N][M];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double t = sv[r];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += S[r][k2] * w.c[k2];
                Sc[r] = t;
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double u = 0.0;
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) u += S[r][k2] * w.A[k2][c];
                    SA[r][c] = u;
                }
#pragma unroll
                for (int a = 0; a < M; ++a) {
                    double u = 0.0;
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) u += S[r][k2] * w.B[k2][a];
                    SB[r][a] = u;
                }
            }
            double Quu[M][M], Qux[M][N], qu[M];
#pragma unroll
            for (int a = 0; a < M; ++a) {
#pragma unroll
                for (int b2 = 0; b2 < M; ++b2) {
                    double t = w.R[a][b2];
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) t += w.B[k2][a] * SB[k2][b2];
                    Quu[a][b2] = t;
                }
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double t = Mk[c][a];
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) t += w.B[k2][a] * SA[k2][c];
                    Qux[a][c] = t;
                }
                double t = rk[a];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += w.B[k2][a] * Sc[k2];
                qu[a] = t;
            }
            double Qi[M][M];
            const bool pd = inv_spd<M>(Quu, Qi);
            double G[M][N], g[M];
#pragma unroll
            for (int a = 0; a < M; ++a) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double t = 0.0;
#pragma unroll
                    for (int b2 = 0; b2 < M; ++b2) t -= Qi[a][b2] * Qux[b2][c];
                    G[a][c] = t;
                }
                double t = 0.0;
#pragma unroll
                for (int b2 = 0; b2 < M; ++b2) t -= Qi[a][b2] * qu[b2];
                g[a] = t;
            }
            double Sn[N][N], sn[N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double t = w.Q[r][c];
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) t += w.A[k2][r] * SA[k2][c];
#pragma unroll
                    for (int a = 0; a < M; ++a) t += Qux[a][r] * G[a][c];
                    Sn[r][c] = t;
                }
                double t = w.q[r];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += w.A[k2][r] * Sc[k2];
#pragma unroll
                for (int a = 0; a < M; ++a) t += Qux[a][r] * g[a];
                sn[r] = t;
            }
            sym(Sn);
            bool fin = true;
#pragma unroll
            for (int r = 0; r < N; ++r) {
                fin = fin && isfinite(sn[r]);
#pragma unroll
                for (int c = 0; c < N; ++c) fin = fin && isfinite(Sn[r][c]);
            }
            note1(fin, SERR_NONFINITE, k, code, fk);
            note1(pd, SERR_NOT_PD, k, code, fk);
            stm(V.S + d.oS + (int64_t)k * N * N, Sn);
            stv(V.s + d.os + (int64_t)k * N, sn);
            stm(V.G + d.oG + (int64_t)k * M * N, G);
            stv(V.g + d.og + (int64_t)k * M, g);
            if (roll) {
                // Phi <- Phi F~_k:  FA <- FA (A + B Gamma),  Fb <- FA (c + B gamma) + Fb
                double F[N][N], f[N];
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    double t = w.c[r];
#pragma unroll
                    for (int a = 0; a < M; ++a) t += w.B[r][a] * g[a];
                    f[r] = t;
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        double u = w.A[r][c];
#pragma unroll
                        for (int a = 0; a < M; ++a) u += w.B[r][a] * G[a][c];
                        F[r][c] = u;
                    }
                }
                double nA[N][N], nb[N];
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    double t = Fb[r];
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) t += FA[r][k2] * f[k2];
                    nb[r] = t;
#pragma unroll
                    for (int c = 0; c < N; ++c) {
                        double u = 0.0;
#pragma unroll
                        for (int k2 = 0; k2 < N; ++k2) u += FA[r][k2] * F[k2][c];
                        nA[r][c] = u;
                    }
                }
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    Fb[r] = nb[r];
#pragma unroll
                    for (int c = 0; c < N; ++c) FA[r][c] = nA[r][c];
                }
            }
#pragma unroll
            for (int r = 0; r < N; ++r) {
                sv[r] = sn[r];
#pragma unroll
                for (int c = 0; c < N; ++c) S[r][c] = Sn[r][c];
            }
        }
    }
    if (roll) {
        if (s == 0) {
            double Z[N][N], x0[N];
#pragma unroll
            for (int r = 0; r < N; ++r)
#pragma unroll
                for (int c = 0; c < N; ++c) Z[r][c] = 0.0;
            ldv(P.x0 + d.on, x0);
            store_map(Yroll + (int64_t)d.xbase * TILE, Z, x0);
        }
        if (!last) store_map(Yroll + (int64_t)(d.xbase + s + 1) * TILE, FA, Fb);
    }
    if (code) report1(status, d.orig, code, fk);
}

// ---------------------------------------------------------------------------
// One radix-RAD level of an affine-map scan (the schedule of k_affine_ks):
//   prefix: Y_s <- Y_s Y_{s-dd} ... Y_{s-(RAD-1)dd},
//   suffix: Y_s <- Y_s Y_{s+dd} ... Y_{s+(RAD-1)dd},
// terms outside [0, nseg] left out; the entry no segment reads is skipped.
// [[F1, e1], [0, 1]] [[F2, e2], [0, 1]] = [[F1 F2, F1 e2 + e1], [0, 1]].
// ---------------------------------------------------------------------------
// Entry gx's product Y_gx Y_{gx+step} ... over `terms` terms, entries KS
// doubles apart from base y (TILE in the scan buffers, (N + 1)^2 in LDS).
template <int N, int KS>
LQK_DEV void affine_chain(const double *y, int64_t gx, int64_t step, int terms, double (&F)[N][N], double (&e)[N])
{
    load_map(y + gx * KS, F, e);
    for (int j = 1; j <= terms; ++j) {
        double F2[N][N], e2[N];
        load_map(y + (gx + j * step) * KS, F2, e2);
        double nF[N][N], ne[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            double t = e[r];
#pragma unroll
            for (int k = 0; k < N; ++k) t += F[r][k] * e2[k];
            ne[r] = t;
#pragma unroll
            for (int c = 0; c < N; ++c) {
                double u = 0.0;
#pragma unroll
                for (int k = 0; k < N; ++k) u += F[r][k] * F2[k][c];
                nF[r][c] = u;
            }
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            e[r] = ne[r];
#pragma unroll
            for (int c = 0; c < N; ++c) F[r][c] = nF[r][c];
        }
    }
}

template <int N, int RAD>
__global__ __launch_bounds__(64) void k_small_affine_ks(const InstDesc *__restrict__ inst,
                                                        const int32_t *__restrict__ x_start, int batch, int total,
                                                        int dd, int suffix, const double *__restrict__ Yin,
                                                        double *__restrict__ Yout)
{
    const int gx = gid();
    if (gx >= total) return;
    const int i = find_inst(x_start, batch, gx);
    const InstDesc d = inst[i];
    const int s = gx - d.xbase;
    if (suffix ? (s == 0) : (s == d.nseg)) return;
    const int avail = suffix ? (d.nseg - s) / dd : s / dd;
    double F[N][N], e[N];
    affine_chain<N, TILE>(Yin, gx, suffix ? dd : -dd, min(RAD - 1, avail), F, e);
    store_map(Yout + (int64_t)gx * TILE, F, e);
}

// Every level of an affine-map scan in one workgroup, for a class with at most
// SCAN1_MAX entries: the entries copied once into LDS, each level's products
// formed in registers, a barrier, then written in place; the results copied
// back to the entries' slots of Y, in place.  Same schedule and arithmetic as
// the per-level kernel.
template <int N, int RAD>
__global__ __launch_bounds__(SCAN1_MAX) void k_small_affine_scan1(const InstDesc *__restrict__ inst,
                                                                   const int32_t *__restrict__ x_start, int batch,
                                                                   int total, int max_nseg, int suffix,
                                                                   double *__restrict__ Y)
{
    constexpr int N1 = N + 1, KS = N1 * N1, AS = KS | 1;   // odd LDS stride: lanes' entries in different banks
    __shared__ double sh[SCAN1_MAX * AS];
    const int t = threadIdx.x;
    for (int idx = t; idx < total * KS; idx += SCAN1_MAX) {
        const int e = idx / KS;
        sh[e * AS + (idx - e * KS)] = Y[(int64_t)e * TILE + (idx - e * KS)];
    }
    bool live = t < total;
    int s = 0, nseg = 0;
    if (live) {
        const InstDesc d = inst[find_inst(x_start, batch, t)];
        s = t - d.xbase;
        nseg = d.nseg;
        live = suffix ? (s != 0) : (s != nseg);
    }
    __syncthreads();
    for (int dd = 1; dd < max_nseg; dd *= RAD) {
        double F[N][N], e[N];
        if (live) {
            const int avail = suffix ? (nseg - s) / dd : s / dd;
            affine_chain<N, AS>(sh, t, suffix ? dd : -dd, min(RAD - 1, avail), F, e);
        }
        __syncthreads();
        if (live) store_map(sh + t * AS, F, e);
        __syncthreads();
    }
    for (int idx = t; idx < total * KS; idx += SCAN1_MAX) {
        const int e = idx / KS;
        Y[(int64_t)e * TILE + (idx - e * KS)] = sh[e * AS + (idx - e * KS)];
    }
}

// ---------------------------------------------------------------------------
// States from the segment start (the last column of scanned entry s):
// x_k stored, u_k = Gamma_k x_k + gamma_k, lambda_k = S_k x_k + s_k,
// x_{k+1} = A x_k + B u_k + c; the last segment also writes x_T, lambda_T.
// ---------------------------------------------------------------------------
template <int N, int M>
__global__ __launch_bounds__(64) void k_small_roll_apply(ProbPtrs P, ValPtrs V, const InstDesc *__restrict__ inst,
                                                         const int32_t *__restrict__ seg_start, int batch, int total,
                                                         const double *__restrict__ Yfin, double *__restrict__ x,
                                                         double *__restrict__ u, double *__restrict__ lam)
{
    constexpr int N1 = N + 1;
    const int gs = gid();
    if (gs >= total) return;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const double *ye = Yfin + (int64_t)(d.xbase + s) * TILE;
    double xv[N];
#pragma unroll
    for (int r = 0; r < N; ++r) xv[r] = ye[r * N1 + N];
    // Stages are loaded CH at a time, all loads of a chunk issued together:
    // each lane streams its own segment, and a stage of an n <= 2 array fills
    // a fraction of a cache line, so loading the next stages while the line
    // is still cached saves fetching it again for each of them.  Past the
    // segment's end the last stage is read again (in bounds) and not used.
    constexpr int CH = (N <= 2) ? 4 : 2;
    for (int kb = k0; kb < k1; kb += CH) {
        double A[CH][N][N], B[CH][N][M], c[CH][N], Gm[CH][M][N], g[CH][M], Sk[CH][N][N], sk[CH][N];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = min(kb + j, k1 - 1);
            ldm(P.A + d.oA + (int64_t)k * N * N, A[j]);
            ldm(P.B + d.oB + (int64_t)k * N * M, B[j]);
            ldv(P.c ? P.c + d.oc + (int64_t)k * N : nullptr, c[j]);
            ldm(V.G + d.oG + (int64_t)k * M * N, Gm[j]);
            ldv(V.g + d.og + (int64_t)k * M, g[j]);
            if (lam) {
                ldm(V.S + d.oS + (int64_t)k * N * N, Sk[j]);
                ldv(V.s + d.os + (int64_t)k * N, sk[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = kb + j;
            if (k >= k1) break;
            stv(x + d.os + (int64_t)k * N, xv);
            double uk[M];
#pragma unroll
            for (int a = 0; a < M; ++a) {
                double t = g[j][a];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += Gm[j][a][k2] * xv[k2];
                uk[a] = t;
            }
            stv(u + d.og + (int64_t)k * M, uk);
            if (lam) {
                double l[N];
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    double t = sk[j][r];
#pragma unroll
                    for (int k2 = 0; k2 < N; ++k2) t += Sk[j][r][k2] * xv[k2];
                    l[r] = t;
                }
                stv(lam + d.os + (int64_t)k * N, l);
            }
            double xn[N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double t = c[j][r];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += A[j][r][k2] * xv[k2];
#pragma unroll
                for (int a = 0; a < M; ++a) t += B[j][r][a] * uk[a];
                xn[r] = t;
            }
#pragma unroll
            for (int r = 0; r < N; ++r) xv[r] = xn[r];
        }
    }
    if (k1 == d.T) {
        stv(x + d.os + (int64_t)d.T * N, xv);
        if (lam) {
            double Sk[N][N], sk[N], l[N];
            ldm(V.S + d.oS + (int64_t)d.T * N * N, Sk);
            ldv(V.s + d.os + (int64_t)d.T * N, sk);
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double t = sk[r];
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) t += Sk[r][k2] * xv[k2];
                l[r] = t;
            }
            stv(lam + d.os + (int64_t)d.T * N, l);
        }
    }
}

// ---------------------------------------------------------------------------
// The Newton step's co-state pass (Alg. 1) for n <= 4, one lane per segment:
// lambda_k = A_k' lambda_{k+1} + g_k, i.e. [lambda_k; 1] = M_k [lambda_{k+1}; 1]
// with M_k = [[A_k', g_k], [0, 1]] (A_k, g_k from the linearisation).
// Fold: Psi_s = M_{k0} M_{k0+1} ... M_{k1-1} as an affine map [[F, e], [0, 1]];
// the last segment also writes the terminal element [[0, lambda_T], [0, 1]].
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(64) void k_small_costate_fold(NmpcWork Wk, const InstDesc *__restrict__ inst,
                                                           const int32_t *__restrict__ seg_start, int batch,
                                                           int total, double *__restrict__ Y)
{
    const int gs = gid();
    if (gs >= total) return;
    const int i = find_inst(seg_start, batch, gs);
    if (level_done(Wk.scal, i)) return;
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    if (s == d.nseg - 1) {
        double Z[N][N], lT[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            lT[r] = Wk.lamT[d.on + r];
#pragma unroll
            for (int c = 0; c < N; ++c) Z[r][c] = 0.0;
        }
        store_map(Y + (int64_t)(d.xbase + d.nseg) * TILE, Z, lT);
    }
    if (s == 0) return;
    double F[N][N], e[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        e[r] = 0.0;
#pragma unroll
        for (int c = 0; c < N; ++c) F[r][c] = (r == c) ? 1.0 : 0.0;
    }
    constexpr int CH = (N <= 2) ? 4 : 2;   // stages loaded together, as in the sweeps
    for (int kb = k0; kb < k1; kb += CH) {
        double A[CH][N][N], g[CH][N];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = min(kb + j, k1 - 1);
            ldm(Wk.A + d.oA + (int64_t)k * N * N, A[j]);
            ldv(Wk.g + d.oc + (int64_t)k * N, g[j]);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            if (kb + j >= k1) break;
            double nF[N][N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double t = e[r];
#pragma unroll
                for (int i2 = 0; i2 < N; ++i2) t += F[r][i2] * g[j][i2];
                e[r] = t;
#pragma unroll
                for (int c = 0; c < N; ++c) {
                    double u = 0.0;
#pragma unroll
                    for (int i2 = 0; i2 < N; ++i2) u += F[r][i2] * A[j][c][i2];   // (F A_k')_{rc}
                    nF[r][c] = u;
                }
            }
#pragma unroll
            for (int r = 0; r < N; ++r)
#pragma unroll
                for (int c = 0; c < N; ++c) F[r][c] = nF[r][c];
        }
    }
    store_map(Y + (int64_t)(d.xbase + s) * TILE, F, e);
}

// Co-states inside each segment from lambda at its right end (the last column
// of scanned entry s + 1; for the last segment the terminal element, whose
// lambda_T it also stores).
template <int N>
__global__ __launch_bounds__(64) void k_small_costate_apply(NmpcWork Wk, const InstDesc *__restrict__ inst,
                                                            const int32_t *__restrict__ seg_start, int batch,
                                                            int total, const double *__restrict__ Yfin)
{
    const int gs = gid();
    if (gs >= total) return;
    const int i = find_inst(seg_start, batch, gs);
    if (level_done(Wk.scal, i)) return;
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    double *lam = Wk.lam + d.os;
    double F[N][N], l[N];
    load_map(Yfin + (int64_t)(d.xbase + s + 1) * TILE, F, l);
    if (s == d.nseg - 1) stv(lam + (int64_t)d.T * N, l);
    constexpr int CH = (N <= 2) ? 4 : 2;
    for (int kb = k1 - 1; kb >= k0; kb -= CH) {
        double A[CH][N][N], g[CH][N];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = max(kb - j, k0);
            ldm(Wk.A + d.oA + (int64_t)k * N * N, A[j]);
            ldv(Wk.g + d.oc + (int64_t)k * N, g[j]);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int k = kb - j;
            if (k < k0) break;
            double ln[N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                double t = g[j][r];
#pragma unroll
                for (int i2 = 0; i2 < N; ++i2) t += A[j][i2][r] * l[i2];   // (A_k' lambda)_r
                ln[r] = t;
            }
#pragma unroll
            for (int r = 0; r < N; ++r) l[r] = ln[r];
            stv(lam + (int64_t)k * N, l);
        }
    }
}

unsigned lanes_grid(int64_t total) { return (unsigned)((total + 63) / 64); }

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers: (n, m) in 1..4 x 1..4, one lane per segment or entry.
// ---------------------------------------------------------------------------

#define LQK_SMALL_NM(n, m, CALL)                                                     \
    switch ((n) * 8 + (m)) {                                                         \
    case 9: CALL(1, 1); break;  case 10: CALL(1, 2); break;                          \
    case 11: CALL(1, 3); break; case 12: CALL(1, 4); break;                          \
    case 17: CALL(2, 1); break; case 18: CALL(2, 2); break;                          \
    case 19: CALL(2, 3); break; case 20: CALL(2, 4); break;                          \
    case 25: CALL(3, 1); break; case 26: CALL(3, 2); break;                          \
    case 27: CALL(3, 3); break; case 28: CALL(3, 4); break;                          \
    case 33: CALL(4, 1); break; case 34: CALL(4, 2); break;                          \
    case 35: CALL(4, 3); break; default: CALL(4, 4); break;                          \
    }
#define LQK_SMALL_N(n, CALL)                                                         \
    switch (n) {                                                                     \
    case 1: CALL(1); break; case 2: CALL(2); break;                                  \
    case 3: CALL(3); break; default: CALL(4); break;                                 \
    }

void launch_small_value_fold(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                             const int32_t *seg_start, int batch, double *X, int32_t *status)
{
#define CALL(N, M) hipLaunchKernelGGL((k_small_value_fold<N, M>), dim3(lanes_grid(total)), dim3(64), 0, st, P, inst, seg_start, batch, (int)total, X, status)
    LQK_SMALL_NM(n, m, CALL)
#undef CALL
}

void launch_small_value_ks(int n, int64_t total, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                           int batch, int dd, const double *Xin, double *Xout, int32_t *status)
{
#define CALL(N) hipLaunchKernelGGL((k_small_value_ks<N>), dim3(lanes_grid(total)), dim3(64), 0, st, inst, x_start, batch, (int)total, dd, Xin, Xout, status)
    LQK_SMALL_N(n, CALL)
#undef CALL
}

bool launch_small_value_scan1(int n, int64_t total, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                              int batch, int max_nseg, double *X, int32_t *status)
{
    const char *e = getenv("LQSCAN_SCAN1");   // "0": the per-level kernels always
    if (n < 1 || n > 4 || total > value_scan1_cap(n) || (e && e[0] == '0' && e[1] == 0)) return false;
#define CALL(N) hipLaunchKernelGGL((k_small_value_scan1<N>), dim3(1), dim3(SCAN1_MAX), 0, st, inst, x_start, batch, (int)total, max_nseg, X, status)
    LQK_SMALL_N(n, CALL)
#undef CALL
    return true;
}

void launch_small_value_riccati(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                                const int32_t *seg_start, int batch, const double *Xfin, ValPtrs V, double *Yroll,
                                double *ckpt, int stride, int32_t *status)
{
#define CALL(N, M) hipLaunchKernelGGL((k_small_value_riccati<N, M>), dim3(lanes_grid(total)), dim3(64), 0, st, P, inst, seg_start, batch, (int)total, Xfin, V, Yroll, ckpt, stride, status)
    LQK_SMALL_NM(n, m, CALL)
#undef CALL
}

void launch_small_affine_ks(int n, int radix, int64_t total, hipStream_t st, const InstDesc *inst,
                            const int32_t *x_start, int batch, int dd, int suffix, const double *Yin, double *Yout)
{
#define CALLR(N, RAD) hipLaunchKernelGGL((k_small_affine_ks<N, RAD>), dim3(lanes_grid(total)), dim3(64), 0, st, inst, x_start, batch, (int)total, dd, suffix, Yin, Yout)
#define CALL2(N) CALLR(N, 2)
#define CALL4(N) CALLR(N, 4)
#define CALL8(N) CALLR(N, 8)
#define CALL16(N) CALLR(N, 16)
#define CALL32(N) CALLR(N, 32)
    switch (radix) {
    case 2: LQK_SMALL_N(n, CALL2) break;
    case 8: LQK_SMALL_N(n, CALL8) break;
    case 16: LQK_SMALL_N(n, CALL16) break;
    case 32: LQK_SMALL_N(n, CALL32) break;
    default: LQK_SMALL_N(n, CALL4) break;
    }
#undef CALL2
#undef CALL4
#undef CALL8
#undef CALL16
#undef CALL32
#undef CALLR
}

bool launch_small_affine_scan1(int n, int radix, int64_t total, hipStream_t st, const InstDesc *inst,
                               const int32_t *x_start, int batch, int max_nseg, int suffix, double *Y)
{
    const char *e = getenv("LQSCAN_SCAN1");   // "0": the per-level kernels always
    if (total > SCAN1_MAX || (e && e[0] == '0' && e[1] == 0)) return false;
#define CALLR(N, RAD) hipLaunchKernelGGL((k_small_affine_scan1<N, RAD>), dim3(1), dim3(SCAN1_MAX), 0, st, inst, x_start, batch, (int)total, max_nseg, suffix, Y)
#define CALL2(N) CALLR(N, 2)
#define CALL4(N) CALLR(N, 4)
#define CALL8(N) CALLR(N, 8)
#define CALL16(N) CALLR(N, 16)
#define CALL32(N) CALLR(N, 32)
    switch (radix) {
    case 2: LQK_SMALL_N(n, CALL2) break;
    case 8: LQK_SMALL_N(n, CALL8) break;
    case 16: LQK_SMALL_N(n, CALL16) break;
    case 32: LQK_SMALL_N(n, CALL32) break;
    default: LQK_SMALL_N(n, CALL4) break;
    }
#undef CALL2
#undef CALL4
#undef CALL8
#undef CALL16
#undef CALL32
#undef CALLR
    return true;
}

void launch_small_costate_fold(int n, int64_t total, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                               const int32_t *seg_start, int batch, double *Y)
{
#define CALL(N) hipLaunchKernelGGL((k_small_costate_fold<N>), dim3(lanes_grid(total)), dim3(64), 0, st, Wk, inst, seg_start, batch, (int)total, Y)
    LQK_SMALL_N(n, CALL)
#undef CALL
}

void launch_small_costate_apply(int n, int64_t total, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                                const int32_t *seg_start, int batch, const double *Yfin)
{
#define CALL(N) hipLaunchKernelGGL((k_small_costate_apply<N>), dim3(lanes_grid(total)), dim3(64), 0, st, Wk, inst, seg_start, batch, (int)total, Yfin)
    LQK_SMALL_N(n, CALL)
#undef CALL
}

void launch_small_roll_apply(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                             const int32_t *seg_start, int batch, const double *Yfin, double *x, double *u,
                             double *lam)
{
#define CALL(N, M) hipLaunchKernelGGL((k_small_roll_apply<N, M>), dim3(lanes_grid(total)), dim3(64), 0, st, P, V, inst, seg_start, batch, (int)total, Yfin, x, u, lam)
    LQK_SMALL_NM(n, m, CALL)
#undef CALL
}

}  // namespace lqk
