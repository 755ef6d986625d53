/*
 * lqoracle.c -- plain, sequential FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * GPU solver.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline leg may load it.  It shares no code, header, table or helper with
 * the GPU library and includes nothing from it.
 *
 * Notation follows the paper (arXiv 2409.20027), shifted to 0-based stages:
 * the paper's t = 1..N with terminal x_{N+1} becomes k = 0..T-1 with terminal
 * x_T.  Names: A_k = df_t/dx_t, B_k = df_t/du_t, Q_k = P_t, R_k = R_t + alpha I,
 * M_k = M_t, r_k = d_t, Q_T = P_{N+1}; the paper's value-element matrix Y is
 * called J here.  All matrices are row-major, all arrays stage-major.
 *
 * Contents
 *   oracle_lq_solve        exact LQ minimiser by the backward Bellman
 *                          (Riccati) recursion of Sec. III-C, the affine
 *                          control law eq:value-fun-feedback (with the
 *                          M-transpose reading of its gain) and the forward
 *                          rollout of Sec. III-D, plus co-states.
 *   oracle_value_element   per-stage value element of eq:value-fun-elem-init
 *                          written in the algebraically equal form that never
 *                          inverts P (the paper's q_t, r_t need P^{-1}).
 *   oracle_value_combine   the value-function operator eq:value-fun-param,
 *                          with the last b-term read as the later element's b.
 *   oracle_costate_combine eq:co-states-comb-rule (l and c gradients summed).
 *   oracle_stateprop_combine eq:state-prop-comb-rule.
 *   oracle_lq_states_cv    the optimal states from the prefix conditional
 *                          value functions and the suffix value functions
 *                          of eq:value-fun-prefix-sum.
 *   oracle_lq_adjoint      gradients of a loss of (x, u) through the LQ
 *                          solution by implicit differentiation of its KKT
 *                          system (not in the paper): a second LQ solve with
 *                          the loss gradients as linear terms.
 *   oracle_nmpc_*          the interior-point Newton method of Alg. 4 with
 *                          the log barrier of Sec. II-B, for a synthetic
 *                          tanh-network model and the torque-limited
 *                          pendulum and force-limited cart-pole of Sec. V
 *                          (hand-derived Jacobians and second derivatives).
 *
 * Error codes: 0 ok, -2 not positive definite (stage in *fail_k),
 * -3 singular, -4 non-finite.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define ERR_NOT_PD (-2)
#define ERR_SINGULAR (-3)
#define ERR_NONFINITE (-4)

/* ------------------------------------------------------------------ */
/* Small dense helpers (row-major)                                     */
/* ------------------------------------------------------------------ */

/* C[r x c] = op(X) op(Y) (+ C if acc), op = transpose when tX / tY set.
 * X is stored as (tX ? k x r : r x k), Y as (tY ? c x k : k x c). */
static void gemm(int r, int c, int k, const double *X, int tX, const double *Y, int tY,
                 double *C, int acc)
{
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) {
            double sum = acc ? C[i * c + j] : 0.0;
            for (int p = 0; p < k; ++p) {
                double xv = tX ? X[p * r + i] : X[i * k + p];
                double yv = tY ? Y[j * k + p] : Y[p * c + j];
                sum += xv * yv;
            }
            C[i * c + j] = sum;
        }
}

/* y[r] = op(X) v (+ y if acc) */
static void gemv(int r, int k, const double *X, int tX, const double *v, double *y, int acc)
{
    for (int i = 0; i < r; ++i) {
        double sum = acc ? y[i] : 0.0;
        for (int p = 0; p < k; ++p) sum += (tX ? X[p * r + i] : X[i * k + p]) * v[p];
        y[i] = sum;
    }
}

/* Cholesky a = L L^T (lower, row-major).  Returns 0, or -1 if not PD. */
static int cholesky(int m, const double *a, double *L)
{
    memset(L, 0, sizeof(double) * m * m);
    for (int j = 0; j < m; ++j) {
        double d = a[j * m + j];
        for (int p = 0; p < j; ++p) d -= L[j * m + p] * L[j * m + p];
        if (!(d > 0.0)) return -1;
        double ljj = sqrt(d);
        L[j * m + j] = ljj;
        for (int i = j + 1; i < m; ++i) {
            double v = a[i * m + j];
            for (int p = 0; p < j; ++p) v -= L[i * m + p] * L[j * m + p];
            L[i * m + j] = v / ljj;
        }
    }
    return 0;
}

/* Solve (L L^T) X = Bm in place, Bm is m x nrhs row-major. */
static void chol_solve(int m, const double *L, double *Bm, int nrhs)
{
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < m; ++i) {
            double v = Bm[i * nrhs + c];
            for (int p = 0; p < i; ++p) v -= L[i * m + p] * Bm[p * nrhs + c];
            Bm[i * nrhs + c] = v / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double v = Bm[i * nrhs + c];
            for (int p = i + 1; p < m; ++p) v -= L[p * m + i] * Bm[p * nrhs + c];
            Bm[i * nrhs + c] = v / L[i * m + i];
        }
    }
}

/* LU with partial pivoting of a (n x n, copied into lu); returns 0 or -1. */
static int lu_factor(int n, const double *a, double *lu, int *piv)
{
    memcpy(lu, a, sizeof(double) * n * n);
    for (int p = 0; p < n; ++p) {
        int best = p;
        double bv = fabs(lu[p * n + p]);
        for (int i = p + 1; i < n; ++i)
            if (fabs(lu[i * n + p]) > bv) { bv = fabs(lu[i * n + p]); best = i; }
        piv[p] = best;
        if (!(bv > 0.0)) return -1;
        if (best != p)
            for (int j = 0; j < n; ++j) {
                double t = lu[p * n + j]; lu[p * n + j] = lu[best * n + j]; lu[best * n + j] = t;
            }
        for (int i = p + 1; i < n; ++i) {
            double f = lu[i * n + p] / lu[p * n + p];
            lu[i * n + p] = f;
            for (int j = p + 1; j < n; ++j) lu[i * n + j] -= f * lu[p * n + j];
        }
    }
    return 0;
}

/* Solve a X = Bm in place given lu_factor output; Bm is n x nrhs. */
static void lu_solve(int n, const double *lu, const int *piv, double *Bm, int nrhs)
{
    for (int p = 0; p < n; ++p)
        if (piv[p] != p)
            for (int c = 0; c < nrhs; ++c) {
                double t = Bm[p * nrhs + c]; Bm[p * nrhs + c] = Bm[piv[p] * nrhs + c];
                Bm[piv[p] * nrhs + c] = t;
            }
    for (int c = 0; c < nrhs; ++c) {
        for (int i = 0; i < n; ++i) {
            double v = Bm[i * nrhs + c];
            for (int p = 0; p < i; ++p) v -= lu[i * n + p] * Bm[p * nrhs + c];
            Bm[i * nrhs + c] = v;
        }
        for (int i = n - 1; i >= 0; --i) {
            double v = Bm[i * nrhs + c];
            for (int p = i + 1; p < n; ++p) v -= lu[i * n + p] * Bm[p * nrhs + c];
            Bm[i * nrhs + c] = v / lu[i * n + i];
        }
    }
}

static int all_finite(const double *v, long cnt)
{
    for (long i = 0; i < cnt; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* O1: LQ solve by the backward Bellman recursion + forward rollout    */
/* ------------------------------------------------------------------ */
/*
 * Problem (Sec. III-C, eq:linearized-ocp generalised with an offset c_k, a
 * state-linear term q_k and an initial state x0; the paper's case is c = q = 0,
 * x0 = 0, r = d):
 *   min sum_k [1/2 x'Qx + x'Mu + 1/2 u'Ru + q'x + r'u] + 1/2 x_T'Q_T x_T + q_T'x_T
 *   s.t. x_{k+1} = A x_k + B u_k + c_k,  x_0 = x0.
 * The value function V_k(x) = 1/2 x'S_k x + s_k'x + const (Sec. III-C);
 * eq:value-fun-feedback gives the control law u = Gamma x + gamma with
 *   Q_uu = R + B'S'B, Gamma = -Q_uu^{-1}(M' + B'S'A), gamma = -Q_uu^{-1}(r + B'(S'c + s')).
 * Co-states (Sec. III-B): lambda_k = S_k x_k + s_k.
 * Optional pointers (c, M, q, r, qT and every output) may be NULL.
 */
int oracle_lq_solve(int n, int m, int T,
                    const double *A, const double *B, const double *c,
                    const double *Q, const double *R, const double *M,
                    const double *q, const double *r,
                    const double *QT, const double *qT, const double *x0,
                    double *S, double *s, double *Gam, double *gam,
                    double *x, double *u, double *lam, int *fail_k)
{
    const int nn = n * n, nm = n * m, mm = m * m;
    double *Sbuf = S ? S : (double *)malloc(sizeof(double) * (size_t)(T + 1) * nn);
    double *sbuf = s ? s : (double *)malloc(sizeof(double) * (size_t)(T + 1) * n);
    double *Gbuf = Gam ? Gam : (double *)malloc(sizeof(double) * (size_t)T * nm + 1);
    double *gbuf = gam ? gam : (double *)malloc(sizeof(double) * (size_t)T * m + 1);
    double *SA = malloc(sizeof(double) * nn), *SB = malloc(sizeof(double) * nm);
    double *v = malloc(sizeof(double) * n), *Quu = malloc(sizeof(double) * mm);
    double *L = malloc(sizeof(double) * mm), *Qux = malloc(sizeof(double) * nm);
    double *qu = malloc(sizeof(double) * m), *Sk = malloc(sizeof(double) * nn);
    int status = OK;
    if (fail_k) *fail_k = -1;

    /* terminal: S_T = sym(Q_T), s_T = q_T */
    double *ST = Sbuf + (size_t)T * nn;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) ST[i * n + j] = 0.5 * (QT[i * n + j] + QT[j * n + i]);
    for (int i = 0; i < n; ++i) sbuf[(size_t)T * n + i] = qT ? qT[i] : 0.0;

    for (int k = T - 1; k >= 0; --k) {
        const double *Ak = A + (size_t)k * nn, *Bk = B + (size_t)k * nm;
        const double *Sp = Sbuf + (size_t)(k + 1) * nn, *sp = sbuf + (size_t)(k + 1) * n;
        double *Gk = Gbuf + (size_t)k * nm, *gk = gbuf + (size_t)k * m;
        gemm(n, n, n, Sp, 0, Ak, 0, SA, 0);             /* S'A        */
        gemm(n, m, n, Sp, 0, Bk, 0, SB, 0);             /* S'B        */
        if (c) gemv(n, n, Sp, 0, c + (size_t)k * n, v, 0);
        else memset(v, 0, sizeof(double) * n);
        for (int i = 0; i < n; ++i) v[i] += sp[i];      /* S'c + s'   */
        memcpy(Quu, R + (size_t)k * mm, sizeof(double) * mm);
        gemm(m, m, n, Bk, 1, SB, 0, Quu, 1);            /* R + B'S'B  */
        if (M) {
            const double *Mk = M + (size_t)k * nm;
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < n; ++j) Qux[i * n + j] = Mk[j * m + i];
            gemm(m, n, n, Bk, 1, SA, 0, Qux, 1);        /* M' + B'S'A */
        } else {
            gemm(m, n, n, Bk, 1, SA, 0, Qux, 0);
        }
        for (int i = 0; i < m; ++i) qu[i] = r ? r[(size_t)k * m + i] : 0.0;
        gemv(m, n, Bk, 1, v, qu, 1);                    /* r + B'(S'c + s') */
        if (cholesky(m, Quu, L) != 0) {
            if (fail_k) *fail_k = k;
            status = ERR_NOT_PD;
            goto done;
        }
        for (int i = 0; i < nm; ++i) Gk[i] = -Qux[i];
        chol_solve(m, L, Gk, n);                        /* Gamma */
        for (int i = 0; i < m; ++i) gk[i] = -qu[i];
        chol_solve(m, L, gk, 1);                        /* gamma */
        /* S = Q + A'S'A + Qux'Gamma, symmetrised */
        memcpy(Sk, Q + (size_t)k * nn, sizeof(double) * nn);
        gemm(n, n, n, Ak, 1, SA, 0, Sk, 1);
        gemm(n, n, m, Qux, 1, Gk, 0, Sk, 1);
        double *Sout = Sbuf + (size_t)k * nn;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) Sout[i * n + j] = 0.5 * (Sk[i * n + j] + Sk[j * n + i]);
        /* s = q + A'(S'c + s') + Qux'gamma */
        double *so = sbuf + (size_t)k * n;
        for (int i = 0; i < n; ++i) so[i] = q ? q[(size_t)k * n + i] : 0.0;
        gemv(n, n, Ak, 1, v, so, 1);
        gemv(n, m, Qux, 1, gk, so, 1);
    }

    if (x || u || lam) {
        double *xb = x ? x : (double *)malloc(sizeof(double) * (size_t)(T + 1) * n);
        double *ub = u ? u : (double *)malloc(sizeof(double) * (size_t)T * m + 1);
        memcpy(xb, x0, sizeof(double) * n);
        for (int k = 0; k < T; ++k) {
            const double *xk = xb + (size_t)k * n;
            double *uk = ub + (size_t)k * m, *xn = xb + (size_t)(k + 1) * n;
            memcpy(uk, gbuf + (size_t)k * m, sizeof(double) * m);
            gemv(m, n, Gbuf + (size_t)k * nm, 0, xk, uk, 1);
            if (c) memcpy(xn, c + (size_t)k * n, sizeof(double) * n);
            else memset(xn, 0, sizeof(double) * n);
            gemv(n, n, A + (size_t)k * nn, 0, xk, xn, 1);
            gemv(n, m, B + (size_t)k * nm, 0, uk, xn, 1);
        }
        if (lam)
            for (int k = 0; k <= T; ++k) {
                double *lk = lam + (size_t)k * n;
                memcpy(lk, sbuf + (size_t)k * n, sizeof(double) * n);
                gemv(n, n, Sbuf + (size_t)k * nn, 0, xb + (size_t)k * n, lk, 1);
            }
        if (!all_finite(xb, (long)(T + 1) * n)) status = ERR_NONFINITE;
        if (!x) free(xb);
        if (!u) free(ub);
    }
    if (status == OK && !all_finite(Sbuf, (long)(T + 1) * nn)) status = ERR_NONFINITE;
done:
    if (!S) free(Sbuf);
    if (!s) free(sbuf);
    if (!Gam) free(Gbuf);
    if (!gam) free(gbuf);
    free(SA); free(SB); free(v); free(Quu); free(L); free(Qux); free(qu); free(Sk);
    return status;
}

/* ------------------------------------------------------------------ */
/* Value-function elements and their operator (Sec. III-C)            */
/* ------------------------------------------------------------------ */
/* An element is packed as [A (n*n) | b (n) | C (n*n) | eta (n) | J (n*n)];
 * it parameterises the conditional value function eq:value-fun-elements
 *   V(x_j, x_i) = max_p 1/2 x_j'J x_j - x_j'eta - 1/2 p'C p - p'(x_i - A x_j - b).
 */

/* eq:value-fun-elem-init for one stage, in the form that never inverts P:
 * minimising the stage cost over u for fixed (x_k, x_{k+1}) gives
 *   A_e = A - B R^{-1} M',  b = c - B R^{-1} r,  C = B R^{-1} B',
 *   J = Q - M R^{-1} M',    eta = -(q - M R^{-1} r).
 * M, q, r, c may be NULL (zero). Returns 0 or -2 if R is not PD. */
int oracle_value_element(int n, int m, const double *A, const double *B, const double *c,
                         const double *Q, const double *R, const double *M,
                         const double *q, const double *r, double *e)
{
    const int nn = n * n;
    double *eA = e, *eb = e + nn, *eC = e + nn + n, *eeta = e + 2 * nn + n, *eJ = e + 2 * nn + 2 * n;
    double *L = malloc(sizeof(double) * m * m);
    double *RiBt = malloc(sizeof(double) * m * n);  /* R^{-1} B' (m x n) */
    double *RiMt = malloc(sizeof(double) * m * n);  /* R^{-1} M' (m x n) */
    double *Rir = malloc(sizeof(double) * m);
    if (cholesky(m, R, L) != 0) { free(L); free(RiBt); free(RiMt); free(Rir); return ERR_NOT_PD; }
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            RiBt[i * n + j] = B[j * m + i];
            RiMt[i * n + j] = M ? M[j * m + i] : 0.0;
        }
    chol_solve(m, L, RiBt, n);
    chol_solve(m, L, RiMt, n);
    for (int i = 0; i < m; ++i) Rir[i] = r ? r[i] : 0.0;
    chol_solve(m, L, Rir, 1);
    memcpy(eA, A, sizeof(double) * nn);
    gemm(n, n, m, B, 0, RiMt, 0, eA, 0);
    for (int i = 0; i < nn; ++i) eA[i] = A[i] - eA[i];
    for (int i = 0; i < n; ++i) eb[i] = c ? c[i] : 0.0;
    gemv(n, m, B, 0, Rir, eC /*scratch*/, 0);
    for (int i = 0; i < n; ++i) eb[i] -= eC[i];
    gemm(n, n, m, B, 0, RiBt, 0, eC, 0);
    if (M) {
        gemm(n, n, m, M, 0, RiMt, 0, eJ, 0);
        for (int i = 0; i < nn; ++i) eJ[i] = Q[i] - eJ[i];
        gemv(n, m, M, 0, Rir, eeta, 0);
        for (int i = 0; i < n; ++i) eeta[i] = -((q ? q[i] : 0.0) - eeta[i]);
    } else {
        memcpy(eJ, Q, sizeof(double) * nn);
        for (int i = 0; i < n; ++i) eeta[i] = -(q ? q[i] : 0.0);
    }
    free(L); free(RiBt); free(RiMt); free(Rir);
    return OK;
}

/* The terminal element nu_{N+1}: zero except J = Q_T (and eta = -q_T). */
void oracle_value_terminal(int n, const double *QT, const double *qT, double *e)
{
    const int nn = n * n;
    memset(e, 0, sizeof(double) * (3 * nn + 2 * n));
    memcpy(e + 2 * nn + 2 * n, QT, sizeof(double) * nn);
    for (int i = 0; i < n; ++i) e[2 * nn + n + i] = qT ? -qT[i] : 0.0;
}

/* eq:value-fun-param: out = e1 (earlier, j->t) (x) e2 (later, t->i).
 *   A   = A2 (I + C1 J2)^{-1} A1
 *   J   = A1' (I + J2 C1)^{-1} J2 A1 + J1
 *   C   = A2 (I + C1 J2)^{-1} C1 A2' + C2
 *   eta = A1' (I + J2 C1)^{-1} (eta2 - J2 b1) + eta1
 *   b   = A2 (I + C1 J2)^{-1} (b1 + C1 eta2) + b2
 * The printed b-rule ends in b_{j,i} itself; the later element's b_{t,i} is
 * the reading that makes the operator associative with (I,0,0,0,0) as unit.
 * Returns 0 or -3 if either inverse does not exist. */
int oracle_value_combine(int n, const double *e1, const double *e2, double *out)
{
    const int nn = n * n;
    const double *A1 = e1, *b1 = e1 + nn, *C1 = e1 + nn + n, *eta1 = e1 + 2 * nn + n, *J1 = e1 + 2 * nn + 2 * n;
    const double *A2 = e2, *b2 = e2 + nn, *C2 = e2 + nn + n, *eta2 = e2 + 2 * nn + n, *J2 = e2 + 2 * nn + 2 * n;
    double *X = malloc(sizeof(double) * nn), *Y = malloc(sizeof(double) * nn);
    double *lu = malloc(sizeof(double) * nn), *luY = malloc(sizeof(double) * nn);
    int *piv = malloc(sizeof(int) * n), *pivY = malloc(sizeof(int) * n);
    double *rhs = malloc(sizeof(double) * n * (2 * n + 1));
    double *rhsY = malloc(sizeof(double) * n * (n + 1));
    double *tmp = malloc(sizeof(double) * nn), *vec = malloc(sizeof(double) * n);
    double *o = malloc(sizeof(double) * (3 * nn + 2 * n));
    int status = OK;
    /* X = I + C1 J2, Y = I + J2 C1 */
    gemm(n, n, n, C1, 0, J2, 0, X, 0);
    gemm(n, n, n, J2, 0, C1, 0, Y, 0);
    for (int i = 0; i < n; ++i) { X[i * n + i] += 1.0; Y[i * n + i] += 1.0; }
    if (lu_factor(n, X, lu, piv) != 0 || lu_factor(n, Y, luY, pivY) != 0) {
        status = ERR_SINGULAR;
        goto done;
    }
    /* rhs = [A1 | C1 | b1 + C1 eta2]  (n x (2n+1)) */
    gemv(n, n, C1, 0, eta2, vec, 0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            rhs[i * (2 * n + 1) + j] = A1[i * n + j];
            rhs[i * (2 * n + 1) + n + j] = C1[i * n + j];
        }
        rhs[i * (2 * n + 1) + 2 * n] = b1[i] + vec[i];
    }
    lu_solve(n, lu, piv, rhs, 2 * n + 1);
    /* rhsY = [J2 A1 | eta2 - J2 b1]  (n x (n+1)) */
    gemm(n, n, n, J2, 0, A1, 0, tmp, 0);
    gemv(n, n, J2, 0, b1, vec, 0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) rhsY[i * (n + 1) + j] = tmp[i * n + j];
        rhsY[i * (n + 1) + n] = eta2[i] - vec[i];
    }
    lu_solve(n, luY, pivY, rhsY, n + 1);
    double *oA = o, *ob = o + nn, *oC = o + nn + n, *oeta = o + 2 * nn + n, *oJ = o + 2 * nn + 2 * n;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double sa = 0, sc = 0;
            for (int p = 0; p < n; ++p) {
                sa += A2[i * n + p] * rhs[p * (2 * n + 1) + j];
                sc += A2[i * n + p] * rhs[p * (2 * n + 1) + n + j];
            }
            oA[i * n + j] = sa;
            tmp[i * n + j] = sc;   /* A2 X^{-1} C1 */
        }
        double sb = b2[i];
        for (int p = 0; p < n; ++p) sb += A2[i * n + p] * rhs[p * (2 * n + 1) + 2 * n];
        ob[i] = sb;
    }
    /* C = (A2 X^{-1} C1) A2' + C2 */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double sc = C2[i * n + j];
            for (int p = 0; p < n; ++p) sc += tmp[i * n + p] * A2[j * n + p];
            oC[i * n + j] = sc;
        }
    /* J = A1' [Y^{-1} J2 A1] + J1, eta = A1' [Y^{-1}(eta2 - J2 b1)] + eta1 */
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double sj = J1[i * n + j];
            for (int p = 0; p < n; ++p) sj += A1[p * n + i] * rhsY[p * (n + 1) + j];
            oJ[i * n + j] = sj;
        }
        double se = eta1[i];
        for (int p = 0; p < n; ++p) se += A1[p * n + i] * rhsY[p * (n + 1) + n];
        oeta[i] = se;
    }
    memcpy(out, o, sizeof(double) * (3 * nn + 2 * n));
done:
    free(X); free(Y); free(lu); free(luY); free(piv); free(pivY); free(rhs); free(rhsY);
    free(tmp); free(vec); free(o);
    return status;
}

/* eq:co-states-comb-rule with the l- and c-gradient terms summed into g:
 * an element (g, F) represents lambda -> g + F' lambda (F = df/dx);
 * out = e1 (earlier) o e2 (later): g = g1 + F1' g2, F' = F1' F2'.
 * Elements are packed [g (n) | F (n*n)], F stored untransposed. */
void oracle_costate_combine(int n, const double *e1, const double *e2, double *out)
{
    const int nn = n * n;
    double *o = malloc(sizeof(double) * (n + nn));
    const double *g1 = e1, *F1 = e1 + n, *g2 = e2, *F2 = e2 + n;
    for (int i = 0; i < n; ++i) {
        double v = g1[i];
        for (int p = 0; p < n; ++p) v += F1[p * n + i] * g2[p];
        o[i] = v;
    }
    /* (F1' F2')' = F2 F1 */
    gemm(n, n, n, F2, 0, F1, 0, o + n, 0);
    memcpy(out, o, sizeof(double) * (n + nn));
    free(o);
}

/* eq:state-prop-comb-rule: an element (F, e) is the map x -> F x + e;
 * out = e1 (earlier) then e2 (later): F = F2 F1, e = F2 e1 + e2.
 * Packed [F (n*n) | e (n)]. */
void oracle_stateprop_combine(int n, const double *e1, const double *e2, double *out)
{
    const int nn = n * n;
    double *o = malloc(sizeof(double) * (n + nn));
    gemm(n, n, n, e2, 0, e1, 0, o, 0);
    gemv(n, n, e2, 0, e1 + nn, o + nn, 0);
    for (int i = 0; i < n; ++i) o[nn + i] += e2[nn + i];
    memcpy(out, o, sizeof(double) * (n + nn));
    free(o);
}

/* ------------------------------------------------------------------ */
/* States from conditional value functions (eq:value-fun-prefix-sum)   */
/* ------------------------------------------------------------------ */
/*
 * The forward variant that Alg. 2's scans make possible: with the prefix
 * element P_k = nu_0 (x) ... (x) nu_{k-1} (the conditional value function
 * V(x_0, x_k) of eq:value-fun-def; P_0 the unit) and the value function
 * V_k(x) = 1/2 x'S_k x + s_k'x of the suffix nu_k (x) ... (x) nu_T, the
 * optimal x_k minimises V(x_0, x_k) + V_k(x_k).  In the dual form
 * eq:value-fun-elements the stationarity conditions are
 *   p = S_k x_k + s_k,   x_k = A_P x_0 + b_P - C_P p,
 * so (I + C_P S_k) x_k = A_P x_0 + b_P - C_P s_k.
 * Both scans are done sequentially with oracle_value_combine.
 * x: (T+1) x n.  Returns 0, -2 (an R_k not PD; stage in *fail_k) or -3.
 */
int oracle_lq_states_cv(int n, int m, int T,
                        const double *A, const double *B, const double *c,
                        const double *Q, const double *R, const double *M,
                        const double *q, const double *r,
                        const double *QT, const double *qT, const double *x0,
                        double *x, int *fail_k)
{
    const int nn = n * n, nm = n * m, mm = m * m, es = 3 * nn + 2 * n;
    double *suf = malloc(sizeof(double) * (size_t)(T + 1) * es);   /* V_k */
    double *pre = malloc(sizeof(double) * es), *el = malloc(sizeof(double) * es);
    double *Mx = malloc(sizeof(double) * nn), *lu = malloc(sizeof(double) * nn);
    double *rhs = malloc(sizeof(double) * n);
    int *piv = malloc(sizeof(int) * n);
    int status = OK;
    if (fail_k) *fail_k = -1;
    /* suffix: V_T = nu_T, V_k = nu_k (x) V_{k+1} */
    oracle_value_terminal(n, QT, qT, suf + (size_t)T * es);
    for (int k = T - 1; k >= 0; --k) {
        status = oracle_value_element(n, m, A + (size_t)k * nn, B + (size_t)k * nm, c ? c + (size_t)k * n : NULL,
                                      Q + (size_t)k * nn, R + (size_t)k * mm, M ? M + (size_t)k * nm : NULL,
                                      q ? q + (size_t)k * n : NULL, r ? r + (size_t)k * m : NULL, el);
        if (status != OK) {
            if (fail_k) *fail_k = k;
            goto done;
        }
        status = oracle_value_combine(n, el, suf + (size_t)(k + 1) * es, suf + (size_t)k * es);
        if (status != OK) {
            if (fail_k) *fail_k = k;
            goto done;
        }
    }
    /* prefix: P_0 = (I, 0, 0, 0, 0), P_{k+1} = P_k (x) nu_k */
    memset(pre, 0, sizeof(double) * es);
    for (int i = 0; i < n; ++i) pre[i * n + i] = 1.0;
    for (int k = 0; k <= T; ++k) {
        const double *PA = pre, *Pb = pre + nn, *PC = pre + nn + n;
        const double *Sk = suf + (size_t)k * es + 2 * nn + 2 * n;   /* S_k = J(V_k)     */
        const double *etak = suf + (size_t)k * es + 2 * nn + n;     /* s_k = -eta(V_k)  */
        gemm(n, n, n, PC, 0, Sk, 0, Mx, 0);
        for (int i = 0; i < n; ++i) Mx[i * n + i] += 1.0;           /* I + C_P S_k      */
        gemv(n, n, PA, 0, x0, rhs, 0);
        for (int i = 0; i < n; ++i) rhs[i] += Pb[i];
        gemv(n, n, PC, 0, etak, rhs, 1);                            /* - C_P s_k = + C_P eta_k */
        if (lu_factor(n, Mx, lu, piv) != 0) {
            if (fail_k) *fail_k = k;
            status = ERR_SINGULAR;
            goto done;
        }
        lu_solve(n, lu, piv, rhs, 1);
        memcpy(x + (size_t)k * n, rhs, sizeof(double) * n);
        if (k == T) break;
        oracle_value_element(n, m, A + (size_t)k * nn, B + (size_t)k * nm, c ? c + (size_t)k * n : NULL,
                             Q + (size_t)k * nn, R + (size_t)k * mm, M ? M + (size_t)k * nm : NULL,
                             q ? q + (size_t)k * n : NULL, r ? r + (size_t)k * m : NULL, el);
        status = oracle_value_combine(n, pre, el, pre);
        if (status != OK) {
            if (fail_k) *fail_k = k;
            goto done;
        }
    }
    if (!all_finite(x, (long)(T + 1) * n)) status = ERR_NONFINITE;
done:
    free(suf); free(pre); free(el); free(Mx); free(lu); free(rhs); free(piv);
    return status;
}

/* ------------------------------------------------------------------ */
/* Adjoint of the LQ solve (implicit function theorem on the KKT)      */
/* ------------------------------------------------------------------ */
/*
 * For a loss L(x, u) with gx = dL/dx_k (k = 0..T) and gu = dL/du_k, the
 * adjoint is the same LQ with linear terms (q, r, q_T) = (gx, gu, gx_T),
 * c = 0, x0 = 0; call its solution (dx, du, dlam).  With (x, u, lam) the
 * forward solution:
 *   dL/dA_k = lam_{k+1} dx_k' + dlam_{k+1} x_k'   dL/dB_k = lam_{k+1} du_k' + dlam_{k+1} u_k'
 *   dL/dc_k = dlam_{k+1}                          dL/dx0  = dlam_0
 *   dL/dQ_k = sym(dx_k x_k')                      dL/dR_k = sym(du_k u_k')
 *   dL/dM_k = dx_k u_k' + x_k du_k'               dL/dq_k = dx_k, dL/dr_k = du_k
 *   dL/dQ_T = sym(dx_T x_T'),  dL/dq_T = dx_T.
 * Any gradient output may be NULL.
 */
int oracle_lq_adjoint(int n, int m, int T,
                      const double *A, const double *B, const double *c,
                      const double *Q, const double *R, const double *M,
                      const double *q, const double *r,
                      const double *QT, const double *qT, const double *x0,
                      const double *gx, const double *gu,
                      double *gA, double *gB, double *gc, double *gQ, double *gR,
                      double *gM, double *gq, double *gr, double *gQT, double *gqT,
                      double *gx0, int *fail_k)
{
    const int nn = n * n, nm = n * m, mm = m * m;
    size_t nx = (size_t)(T + 1) * n, nu = (size_t)T * m + 1;
    double *x = malloc(sizeof(double) * nx), *u = malloc(sizeof(double) * nu);
    double *lam = malloc(sizeof(double) * nx);
    double *dx = malloc(sizeof(double) * nx), *du = malloc(sizeof(double) * nu);
    double *dlam = malloc(sizeof(double) * nx);
    double *zero = calloc((size_t)n, sizeof(double));
    int st = oracle_lq_solve(n, m, T, A, B, c, Q, R, M, q, r, QT, qT, x0,
                             NULL, NULL, NULL, NULL, x, u, lam, fail_k);
    if (st == OK)
        st = oracle_lq_solve(n, m, T, A, B, NULL, Q, R, M, gx, gu, QT, gx + (size_t)T * n, zero,
                             NULL, NULL, NULL, NULL, dx, du, dlam, fail_k);
    if (st != OK) goto done;
    for (int k = 0; k < T; ++k) {
        const double *xk = x + (size_t)k * n, *uk = u + (size_t)k * m;
        const double *dxk = dx + (size_t)k * n, *duk = du + (size_t)k * m;
        const double *l1 = lam + (size_t)(k + 1) * n, *dl1 = dlam + (size_t)(k + 1) * n;
        for (int i = 0; i < n; ++i) {
            if (gA) for (int j = 0; j < n; ++j)
                gA[(size_t)k * nn + i * n + j] = l1[i] * dxk[j] + dl1[i] * xk[j];
            if (gB) for (int j = 0; j < m; ++j)
                gB[(size_t)k * nm + i * m + j] = l1[i] * duk[j] + dl1[i] * uk[j];
            if (gc) gc[(size_t)k * n + i] = dl1[i];
            if (gQ) for (int j = 0; j < n; ++j)
                gQ[(size_t)k * nn + i * n + j] = 0.5 * (dxk[i] * xk[j] + xk[i] * dxk[j]);
            if (gM) for (int j = 0; j < m; ++j)
                gM[(size_t)k * nm + i * m + j] = dxk[i] * uk[j] + xk[i] * duk[j];
            if (gq) gq[(size_t)k * n + i] = dxk[i];
        }
        for (int i = 0; i < m; ++i) {
            if (gR) for (int j = 0; j < m; ++j)
                gR[(size_t)k * mm + i * m + j] = 0.5 * (duk[i] * uk[j] + uk[i] * duk[j]);
            if (gr) gr[(size_t)k * m + i] = duk[i];
        }
    }
    {
        const double *xT = x + (size_t)T * n, *dxT = dx + (size_t)T * n;
        for (int i = 0; i < n; ++i) {
            if (gQT) for (int j = 0; j < n; ++j) gQT[i * n + j] = 0.5 * (dxT[i] * xT[j] + xT[i] * dxT[j]);
            if (gqT) gqT[i] = dxT[i];
            if (gx0) gx0[i] = dlam[i];
        }
    }
done:
    free(x); free(u); free(lam); free(dx); free(du); free(dlam); free(zero);
    return st;
}

/* ------------------------------------------------------------------ */
/* Interior-point Newton method for x' = x + h f(x, u)                 */
/* ------------------------------------------------------------------ */
/*
 * Models (one explicit Euler step F(x, u) = x + h f(x, u) of Sec. V):
 *   NMPC_TANH      f = tanh(W x) + B u (synthetic network dynamics);
 *   NMPC_PENDULUM  x = (theta, omega), u = tau, prm = (g, l, m, b):
 *                  theta'' = -(g/l) sin theta + (tau - b omega)/(m l^2);
 *   NMPC_CARTPOLE  x = (p, theta, v, omega), u = F, prm = (g, l, m_c, m_p):
 *                  p''     = (F + m_p s (l omega^2 + g c)) / D,
 *                  theta'' = (-F c - m_p l omega^2 c s - (m_c + m_p) g s) / (l D),
 *                  s = sin theta, c = cos theta, D = m_c + m_p s^2
 *                  (the omega^2 in p'' is the textbook cart-pole's; the
 *                  printed p'' has omega to the first power).
 * Costs: l_k = 1/2 (x - ref_k)'Q(x - ref_k) + 1/2 u'R u,
 *        l_T = 1/2 (x - ref_T)'Q_T(x - ref_T).
 * Box |u_i| bounds as 2 nu inequality constraints (u - umax <= 0,
 * umin - u <= 0) with the log barrier of Sec. II-B:
 *        c(u) = -mu sum_i [log(umax - u_i) + log(u_i - umin)].
 */
#define NMPC_TANH 0
#define NMPC_PENDULUM 1
#define NMPC_CARTPOLE 2

typedef struct {
    int nx, nu, T;
    double h;
    int model;
    const double *prm;
    const double *W, *Bm, *Q, *R, *QT, *xref, *x0;
    double umin, umax;
    /* rho > 0: the ADMM augmentation rho/2 |h(u) - z + v/rho|^2 of Sec. II-C
     * (z, v: [T][2 nu], rows u - umax then umin - u) replaces the barrier */
    double rho;
    const double *z, *v;
} nmpc_prob;

/* Value and derivatives over (theta, omega, F) of a cart-pole quantity. */
typedef struct {
    double v, t, w, F, tt, tw, tF, ww, wF, FF;
} cp_d2;

/* q = N / D with D a function of theta alone (quotient rule, first and
 * second derivatives). */
static cp_d2 cp_quot(cp_d2 N, double D, double Dt, double Dtt)
{
    cp_d2 q;
    const double D2 = D * D, D3 = D2 * D;
    q.v = N.v / D;
    q.t = N.t / D - N.v * Dt / D2;
    q.w = N.w / D;
    q.F = N.F / D;
    q.tt = N.tt / D - 2.0 * N.t * Dt / D2 - N.v * Dtt / D2 + 2.0 * N.v * Dt * Dt / D3;
    q.tw = N.tw / D - N.w * Dt / D2;
    q.tF = N.tF / D - N.F * Dt / D2;
    q.ww = N.ww / D;
    q.wF = N.wF / D;
    q.FF = N.FF / D;
    return q;
}

/* The cart-pole accelerations a3 = p'' and a4 = theta'' with their
 * derivatives over (theta, omega, F). */
static void cp_accel(const double *prm, const double *x, const double *u, cp_d2 *a3, cp_d2 *a4)
{
    const double g = prm[0], l = prm[1], mc = prm[2], mp = prm[3];
    const double s = sin(x[1]), c = cos(x[1]), w = x[3], F = u[0];
    const double D = mc + mp * s * s, Dt = 2.0 * mp * s * c, Dtt = 2.0 * mp * (c * c - s * s);
    cp_d2 N3, N4;
    /* N3 = F + m_p l w^2 s + m_p g s c */
    N3.v = F + mp * l * w * w * s + mp * g * s * c;
    N3.t = mp * l * w * w * c + mp * g * (c * c - s * s);
    N3.w = 2.0 * mp * l * w * s;
    N3.F = 1.0;
    N3.tt = -mp * l * w * w * s - 4.0 * mp * g * s * c;
    N3.tw = 2.0 * mp * l * w * c;
    N3.tF = 0.0;
    N3.ww = 2.0 * mp * l * s;
    N3.wF = 0.0;
    N3.FF = 0.0;
    /* N4 = -F c - m_p l w^2 c s - (m_c + m_p) g s   (theta'' = N4 / (l D)) */
    N4.v = -F * c - mp * l * w * w * c * s - (mc + mp) * g * s;
    N4.t = F * s - mp * l * w * w * (c * c - s * s) - (mc + mp) * g * c;
    N4.w = -2.0 * mp * l * w * c * s;
    N4.F = -c;
    N4.tt = F * c + 4.0 * mp * l * w * w * s * c + (mc + mp) * g * s;
    N4.tw = -2.0 * mp * l * w * (c * c - s * s);
    N4.tF = s;
    N4.ww = -2.0 * mp * l * c * s;
    N4.wF = 0.0;
    N4.FF = 0.0;
    *a3 = cp_quot(N3, D, Dt, Dtt);
    cp_d2 q = cp_quot(N4, D, Dt, Dtt);
    q.v /= l; q.t /= l; q.w /= l; q.F /= l;
    q.tt /= l; q.tw /= l; q.tF /= l; q.ww /= l; q.wF /= l; q.FF /= l;
    *a4 = q;
}

/* Continuous-time right-hand side f(x, u) of the pendulum and cart-pole. */
static void model_f(const nmpc_prob *P, const double *x, const double *u, double *f)
{
    if (P->model == NMPC_PENDULUM) {
        const double g = P->prm[0], l = P->prm[1], m = P->prm[2], b = P->prm[3];
        f[0] = x[1];
        f[1] = -g / l * sin(x[0]) + (u[0] - b * x[1]) / (m * l * l);
    } else {
        cp_d2 a3, a4;
        cp_accel(P->prm, x, u, &a3, &a4);
        f[0] = x[2];
        f[1] = x[3];
        f[2] = a3.v;
        f[3] = a4.v;
    }
}

/* Jacobians fx = df/dx (n x n), fu = df/du (n x m) of the pendulum and
 * cart-pole right-hand sides. */
static void model_jac(const nmpc_prob *P, const double *x, const double *u, double *fx, double *fu)
{
    const int n = P->nx, m = P->nu;
    memset(fx, 0, sizeof(double) * n * n);
    memset(fu, 0, sizeof(double) * n * m);
    if (P->model == NMPC_PENDULUM) {
        const double g = P->prm[0], l = P->prm[1], mm = P->prm[2], b = P->prm[3];
        fx[0 * 2 + 1] = 1.0;
        fx[1 * 2 + 0] = -g / l * cos(x[0]);
        fx[1 * 2 + 1] = -b / (mm * l * l);
        fu[1] = 1.0 / (mm * l * l);
    } else {
        cp_d2 a3, a4;
        cp_accel(P->prm, x, u, &a3, &a4);
        fx[0 * 4 + 2] = 1.0;
        fx[1 * 4 + 3] = 1.0;
        fx[2 * 4 + 1] = a3.t;
        fx[2 * 4 + 3] = a3.w;
        fx[3 * 4 + 1] = a4.t;
        fx[3 * 4 + 3] = a4.w;
        fu[2] = a3.F;
        fu[3] = a4.F;
    }
}

/* Contraction of the second derivatives of f with a co-state lam:
 * Hxx = sum_i lam_i d2f_i/dx2 (n x n), Hxu = sum_i lam_i d2f_i/dxdu (n x m),
 * Huu = sum_i lam_i d2f_i/du2 (m x m). */
static void model_hess(const nmpc_prob *P, const double *x, const double *u, const double *lam, double *Hxx,
                       double *Hxu, double *Huu)
{
    const int n = P->nx, m = P->nu;
    memset(Hxx, 0, sizeof(double) * n * n);
    memset(Hxu, 0, sizeof(double) * n * m);
    memset(Huu, 0, sizeof(double) * m * m);
    if (P->model == NMPC_PENDULUM) {
        const double g = P->prm[0], l = P->prm[1];
        Hxx[0] = lam[1] * (g / l) * sin(x[0]);   /* d2/dtheta2 of -(g/l) sin theta */
    } else {
        cp_d2 a3, a4;
        cp_accel(P->prm, x, u, &a3, &a4);
        const double l3 = lam[2], l4 = lam[3];
        Hxx[1 * 4 + 1] = l3 * a3.tt + l4 * a4.tt;
        Hxx[1 * 4 + 3] = Hxx[3 * 4 + 1] = l3 * a3.tw + l4 * a4.tw;
        Hxx[3 * 4 + 3] = l3 * a3.ww + l4 * a4.ww;
        Hxu[1] = l3 * a3.tF + l4 * a4.tF;
        Hxu[3] = l3 * a3.wF + l4 * a4.wF;
        Huu[0] = l3 * a3.FF + l4 * a4.FF;
    }
}

static void f_step(const nmpc_prob *P, const double *x, const double *u, double *xn)
{
    const int n = P->nx, m = P->nu;
    if (P->model == NMPC_TANH) {
        for (int i = 0; i < n; ++i) {
            double z = 0, bu = 0;
            for (int j = 0; j < n; ++j) z += P->W[i * n + j] * x[j];
            for (int j = 0; j < m; ++j) bu += P->Bm[i * m + j] * u[j];
            xn[i] = x[i] + P->h * (tanh(z) + bu);
        }
    } else {
        double f[4];
        model_f(P, x, u, f);
        for (int i = 0; i < n; ++i) xn[i] = x[i] + P->h * f[i];
    }
}

/* Model check: 0 if (model, n, m) is a known combination. */
static int model_ok(int model, int n, int m, const double *prm)
{
    if (model == NMPC_TANH) return 0;
    if (model == NMPC_PENDULUM) return (n == 2 && m == 1 && prm) ? 0 : -1;
    if (model == NMPC_CARTPOLE) return (n == 4 && m == 1 && prm) ? 0 : -1;
    return -1;
}

/* f(x, u) for tests (pendulum and cart-pole only); returns -1 otherwise. */
int oracle_nmpc_f(int model, const double *prm, int nx, int nu, const double *x, const double *u, double *f)
{
    if (model == NMPC_TANH || model_ok(model, nx, nu, prm) != 0) return -1;
    nmpc_prob P = {nx, nu, 0, 0.0, model, prm, NULL, NULL, NULL, NULL, NULL, NULL, NULL, 0.0, 0.0, 0.0, NULL, NULL};
    model_f(&P, x, u, f);
    return 0;
}

/* Nonlinear rollout from x0 under u; returns 0, or -1 if u is infeasible for
 * the barrier (ADMM iterates may leave the box). */
static int rollout(const nmpc_prob *P, const double *u, double *x)
{
    const int n = P->nx, m = P->nu;
    memcpy(x, P->x0, sizeof(double) * n);
    for (int k = 0; k < P->T; ++k) f_step(P, x + (size_t)k * n, u + (size_t)k * m, x + (size_t)(k + 1) * n);
    if (P->rho > 0.0) return 0;
    for (long i = 0; i < (long)P->T * m; ++i)
        if (!(u[i] < P->umax && u[i] > P->umin)) return -1;
    return 0;
}

/* ADMM residual of stage k, input i: (a, b) = h(u) - z + v / rho for the rows
 * u_i - umax <= 0 and umin - u_i <= 0. */
static void admm_ab(const nmpc_prob *P, int k, int i, double ui, double *a, double *b)
{
    const int m = P->nu;
    const double *zk = P->z + (size_t)k * 2 * m, *vk = P->v + (size_t)k * 2 * m;
    *a = (ui - P->umax) - zk[i] + vk[i] / P->rho;
    *b = (P->umin - ui) - zk[m + i] + vk[m + i] / P->rho;
}

/* J_mu(u): cost of the nonlinear rollout plus the barrier, +inf if infeasible;
 * with rho > 0 the ADMM augmentation instead of the barrier (J_AD of Sec. II-C). */
static double cost_mu(const nmpc_prob *P, const double *u, const double *x, double mu)
{
    const int n = P->nx, m = P->nu;
    double J = 0.0;
    for (int k = 0; k < P->T; ++k) {
        const double *xk = x + (size_t)k * n, *rk = P->xref + (size_t)k * n, *uk = u + (size_t)k * m;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) J += 0.5 * (xk[i] - rk[i]) * P->Q[i * n + j] * (xk[j] - rk[j]);
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) J += 0.5 * uk[i] * P->R[i * m + j] * uk[j];
            if (P->rho > 0.0) {
                double a, b;
                admm_ab(P, k, i, uk[i], &a, &b);
                J += 0.5 * P->rho * (a * a + b * b);
                continue;
            }
            double a = P->umax - uk[i], b = uk[i] - P->umin;
            if (!(a > 0 && b > 0)) return INFINITY;
            J += -mu * (log(a) + log(b));
        }
    }
    const double *xT = x + (size_t)P->T * n, *rT = P->xref + (size_t)P->T * n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) J += 0.5 * (xT[i] - rT[i]) * P->QT[i * n + j] * (xT[j] - rT[j]);
    return J;
}

double oracle_nmpc_cost(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                        const double *Bm, const double *Q, const double *R, const double *QT, const double *xref,
                        const double *x0, double umin, double umax, double rho, const double *z, const double *v,
                        double mu, const double *u)
{
    if (model_ok(model, nx, nu, prm) != 0) return NAN;
    nmpc_prob P = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, rho, z, v};
    double *x = malloc(sizeof(double) * (size_t)(T + 1) * nx);
    double J = rollout(&P, u, x) == 0 ? cost_mu(&P, u, x, mu) : INFINITY;
    free(x);
    return J;
}

/* Nonlinear rollout x [T+1][nx] of u (feasibility not checked). */
int oracle_nmpc_rollout(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                        const double *Bm, const double *x0, const double *u, double *x)
{
    if (model_ok(model, nx, nu, prm) != 0) return -1;
    nmpc_prob P = {nx, nu, T, h, model, prm, W, Bm, NULL, NULL, NULL, NULL, x0, 0.0, 0.0, 1.0, NULL, NULL};
    memcpy(x, x0, sizeof(double) * nx);
    for (int k = 0; k < T; ++k) f_step(&P, x + (size_t)k * nx, u + (size_t)k * nu, x + (size_t)(k + 1) * nx);
    return 0;
}

/*
 * Linearisation, co-states and quadraticisation at the nominal (x, u)
 * (Alg. 1 and the expansion of Sec. III-C), with F = x + h f:
 *   A_k = dF/dx = I + h df/dx,  B_k = dF/du = h df/du,
 *   lam_T = Q_T(x_T - ref_T),  lam_k = Q(x_k - ref_k) + A_k' lam_{k+1}
 *     (eq:co-state-eq; the barrier has no x-dependence),
 *   P_k = Q + h lam_{k+1}' d2f/dx2,  M_k = h lam_{k+1}' d2f/dxdu,
 *   Rh_k = R + d2c/du2 + h lam_{k+1}' d2f/du2
 *        = ... + mu diag(1/(umax-u)^2 + 1/(u-umin)^2),
 *   d_k = R u + dc/du + B_k' lam_{k+1},  P_T = Q_T.
 * For the tanh model z = W x, df/dx = diag(1 - tanh^2 z) W, df/du = B,
 * lam' d2f/dx2 = sum_i lam_i tanh''(z_i) w_i w_i' (w_i = row i of W), and
 * the mixed and control second derivatives vanish.
 * Outputs: A [T][n][n], Bl [T][n][m], lam [T+1][n], P [T][n][n],
 * Rh [T][m][m], d [T][m], M [T][n][m].  Any may be NULL except where a later
 * one needs it.
 */
void oracle_nmpc_expand(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                        const double *Bm, const double *Q, const double *R, const double *QT,
                        const double *xref, double umin, double umax, double rho, const double *z,
                        const double *v, double mu, const double *x, const double *u, double *A, double *Bl,
                        double *lam, double *P, double *Rh, double *d, double *M)
{
    const int n = nx, m = nu;
    if (model_ok(model, nx, nu, prm) != 0) return;
    nmpc_prob Pb = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, NULL, umin, umax, rho, z, v};
    double *th = malloc(sizeof(double) * (size_t)T * n);
    if (model == NMPC_TANH) {
        for (int k = 0; k < T; ++k)
            for (int i = 0; i < n; ++i) {
                double z = 0;
                for (int j = 0; j < n; ++j) z += W[i * n + j] * x[(size_t)k * n + j];
                th[(size_t)k * n + i] = tanh(z);
            }
        for (int k = 0; k < T; ++k) {
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    double t = th[(size_t)k * n + i];
                    A[(size_t)k * n * n + i * n + j] = (i == j ? 1.0 : 0.0) + h * (1.0 - t * t) * W[i * n + j];
                }
            for (int i = 0; i < n * m; ++i) Bl[(size_t)k * n * m + i] = h * Bm[i];
        }
    } else {
        double fx[16], fu[4];
        for (int k = 0; k < T; ++k) {
            model_jac(&Pb, x + (size_t)k * n, u + (size_t)k * m, fx, fu);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) A[(size_t)k * n * n + i * n + j] = (i == j ? 1.0 : 0.0) + h * fx[i * n + j];
            for (int i = 0; i < n * m; ++i) Bl[(size_t)k * n * m + i] = h * fu[i];
        }
    }
    /* co-states */
    for (int i = 0; i < n; ++i) {
        double v = 0;
        for (int j = 0; j < n; ++j) v += QT[i * n + j] * (x[(size_t)T * n + j] - xref[(size_t)T * n + j]);
        lam[(size_t)T * n + i] = v;
    }
    for (int k = T - 1; k >= 0; --k)
        for (int i = 0; i < n; ++i) {
            double v = 0;
            for (int j = 0; j < n; ++j) v += Q[i * n + j] * (x[(size_t)k * n + j] - xref[(size_t)k * n + j]);
            for (int j = 0; j < n; ++j) v += A[(size_t)k * n * n + j * n + i] * lam[(size_t)(k + 1) * n + j];
            lam[(size_t)k * n + i] = v;
        }
    /* second-order terms */
    for (int k = 0; k < T; ++k) {
        double Hxx[16], Hxu[4], Huu[1] = {0.0};
        if (model != NMPC_TANH)
            model_hess(&Pb, x + (size_t)k * n, u + (size_t)k * m, lam + (size_t)(k + 1) * n, Hxx, Hxu, Huu);
        if (P) {
            double *Pk = P + (size_t)k * n * n;
            memcpy(Pk, Q, sizeof(double) * n * n);
            if (model == NMPC_TANH) {
                for (int i = 0; i < n; ++i) {
                    double t = th[(size_t)k * n + i];
                    double w = lam[(size_t)(k + 1) * n + i] * h * (-2.0 * t * (1.0 - t * t));
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b) Pk[a * n + b] += w * W[i * n + a] * W[i * n + b];
                }
            } else {
                for (int i = 0; i < n * n; ++i) Pk[i] += h * Hxx[i];
            }
        }
        if (M) {
            double *Mk = M + (size_t)k * n * m;
            for (int i = 0; i < n * m; ++i) Mk[i] = (model == NMPC_TANH) ? 0.0 : h * Hxu[i];
        }
        if (Rh) {
            double *Rk = Rh + (size_t)k * m * m;
            memcpy(Rk, R, sizeof(double) * m * m);
            for (int i = 0; i < m; ++i) {
                double uu = u[(size_t)k * m + i], a = umax - uu, b = uu - umin;
                Rk[i * m + i] += (rho > 0.0) ? 2.0 * rho : mu * (1.0 / (a * a) + 1.0 / (b * b));
            }
            if (model != NMPC_TANH)
                for (int i = 0; i < m * m; ++i) Rk[i] += h * Huu[i];
        }
        if (d)
            for (int i = 0; i < m; ++i) {
                double v = 0;
                for (int j = 0; j < m; ++j) v += R[i * m + j] * u[(size_t)k * m + j];
                double uu = u[(size_t)k * m + i];
                if (rho > 0.0) {
                    double a, b;
                    admm_ab(&Pb, k, i, uu, &a, &b);
                    v += rho * (a - b);
                } else {
                    v += mu * (1.0 / (umax - uu) - 1.0 / (uu - umin));
                }
                for (int j = 0; j < n; ++j) v += Bl[(size_t)k * n * m + j * m + i] * lam[(size_t)(k + 1) * n + j];
                d[(size_t)k * m + i] = v;
            }
    }
    free(th);
}

/*
 * One iteration of Alg. 4 at barrier level mu, Levenberg-Marquardt weight
 * alpha and growth factor nu_lm (both updated in place):
 *   1-3. linearise, co-states, quadraticise (oracle_nmpc_expand);
 *   4.   LQ step: eq:linearized-ocp with psi_k of eq:linearized-ocp-param
 *        (R + alpha I, cross term M), delta x_0 = 0, solved by oracle_lq_solve;
 *   5.   predicted decrease of the expansion without the alpha term,
 *        pred = -[sum d'du + 1/2 sum (dx'P dx + 2 dx'M du + du'Rh du)
 *                 + 1/2 dx_T'P_T dx_T];
 *   6.   candidate u + du, nonlinear rollout, gain ratio
 *        rho = (J_mu(u) - J_mu(u + du)) / pred;
 *   7.   accept if pred > 0 and rho > 0 (finite): alpha *= max(1/3, 1-(2 rho-1)^3),
 *        nu_lm = 2; else alpha *= nu_lm, nu_lm *= 2.
 *        The paper names this update only by reference (a gain-ratio rule of
 *        Madsen et al.), so it is a reading.  Its ends are pinned by the
 *        tests (an exact quadratic model gives rho = 1 and alpha / 3; a step
 *        out of the box is rejected); its shape for 0 < rho < 1 is parity
 *        unpinned.
 * x, u hold the nominal and are replaced on acceptance.  Returns 1 if
 * accepted, 0 if rejected, -1 for an unknown model; *cost gets J_mu of the
 * (possibly new) nominal, *grad_out max_k,i |d_k,i| = |dJ_mu/du|_inf at the
 * nominal the iteration started from.
 */
int oracle_nmpc_newton_step(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                            const double *Bm, const double *Q, const double *R, const double *QT,
                            const double *xref, const double *x0, double umin, double umax, double admm_rho,
                            const double *z, const double *v, double mu, double *alpha, double *nu_lm, double *x,
                            double *u, double *cost, double *pred_out, double *rho_out, double *grad_out)
{
    const int n = nx, m = nu;
    if (model_ok(model, nx, nu, prm) != 0) return -1;
    nmpc_prob Pb = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, admm_rho, z, v};
    size_t Tn = (size_t)T * n, Tnn = Tn * n, Tm = (size_t)T * m;
    double *A = malloc(sizeof(double) * Tnn), *Bl = malloc(sizeof(double) * Tn * m);
    double *lam = malloc(sizeof(double) * (Tn + n)), *P = malloc(sizeof(double) * Tnn);
    double *Rh = malloc(sizeof(double) * Tm * m), *d = malloc(sizeof(double) * Tm);
    double *Mx = malloc(sizeof(double) * Tn * m);
    double *Ra = malloc(sizeof(double) * Tm * m);
    double *dx = malloc(sizeof(double) * (Tn + n)), *du = malloc(sizeof(double) * Tm);
    double *un = malloc(sizeof(double) * Tm), *xn = malloc(sizeof(double) * (Tn + n));
    double *zero = calloc((size_t)n, sizeof(double));
    int accepted = 0;
    double J0 = cost_mu(&Pb, u, x, mu), pred = 0, rho = -INFINITY;
    oracle_nmpc_expand(nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, umin, umax, admm_rho, z, v, mu, x, u, A, Bl,
                       lam, P, Rh, d, Mx);
    for (size_t k = 0; k < (size_t)T; ++k)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                Ra[k * m * m + i * m + j] = Rh[k * m * m + i * m + j] + (i == j ? *alpha : 0.0);
    int fk;
    int st = oracle_lq_solve(n, m, T, A, Bl, NULL, P, Ra, model == NMPC_TANH ? NULL : Mx, NULL, d, QT, NULL, zero,
                             NULL, NULL, NULL, NULL, dx, du, NULL, &fk);
    if (st == OK) {
        for (size_t k = 0; k < (size_t)T; ++k) {
            const double *dxk = dx + k * n, *duk = du + k * m;
            for (int i = 0; i < m; ++i) pred += d[k * m + i] * duk[i];
            double qf = 0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) qf += dxk[i] * P[k * n * n + i * n + j] * dxk[j];
            if (model != NMPC_TANH)
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < m; ++j) qf += 2.0 * dxk[i] * Mx[k * n * m + i * m + j] * duk[j];
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) qf += duk[i] * Rh[k * m * m + i * m + j] * duk[j];
            pred += 0.5 * qf;
        }
        {
            double qf = 0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) qf += dx[Tn + i] * QT[i * n + j] * dx[Tn + j];
            pred += 0.5 * qf;
        }
        pred = -pred;
        for (size_t i = 0; i < Tm; ++i) un[i] = u[i] + du[i];
        double J1 = rollout(&Pb, un, xn) == 0 ? cost_mu(&Pb, un, xn, mu) : INFINITY;
        if (pred > 0 && isfinite(J1)) {
            rho = (J0 - J1) / pred;
            if (rho > 0) {
                accepted = 1;
                double t = 2.0 * rho - 1.0;
                double f = 1.0 - t * t * t;
                *alpha *= (f > 1.0 / 3.0 ? f : 1.0 / 3.0);
                *nu_lm = 2.0;
                memcpy(u, un, sizeof(double) * Tm);
                memcpy(x, xn, sizeof(double) * (Tn + n));
                J0 = J1;
            }
        }
    }
    if (!accepted) {
        *alpha *= *nu_lm;
        *nu_lm *= 2.0;
    }
    if (cost) *cost = J0;
    if (pred_out) *pred_out = pred;
    if (rho_out) *rho_out = rho;
    if (grad_out) {
        double g = 0.0;
        for (size_t i = 0; i < Tm; ++i) g = fmax(g, fabs(d[i]));
        *grad_out = g;
    }
    free(A); free(Bl); free(lam); free(P); free(Rh); free(d); free(Mx); free(Ra);
    free(dx); free(du); free(un); free(xn); free(zero);
    return accepted;
}

/*
 * The interior-point outer loop of Sec. II-B around Alg. 4 with a fixed
 * number of Newton iterations per barrier level: for each mu in mu_levels
 * (decreasing), run iters iterations.  u holds the strictly feasible initial
 * controls and is overwritten by the result; x gets the final nonlinear
 * rollout.  Traces (length n_levels * iters, any may be NULL) record the
 * cost after each iteration, the accept flag and the Levenberg-Marquardt
 * weight used in it.  Returns 0, or -1 if u starts infeasible or the model
 * is unknown.
 */
int oracle_nmpc_solve(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                      const double *Bm, const double *Q, const double *R, const double *QT, const double *xref,
                      const double *x0, double umin, double umax,
                      const double *mu_levels, int n_levels, int iters,
                      double alpha0, double nu0, double *u, double *x,
                      double *cost_trace, int *accept_trace, double *alpha_trace)
{
    if (model_ok(model, nx, nu, prm) != 0) return -1;
    nmpc_prob Pb = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0, NULL, NULL};
    if (rollout(&Pb, u, x) != 0) return -1;
    double alpha = alpha0, nu_lm = nu0;
    int it = 0;
    for (int lv = 0; lv < n_levels; ++lv)
        for (int i = 0; i < iters; ++i, ++it) {
            double a_used = alpha, cst;
            int acc = oracle_nmpc_newton_step(nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0,
                                              NULL, NULL, mu_levels[lv], &alpha, &nu_lm, x, u, &cst, NULL, NULL, NULL);
            if (cost_trace) cost_trace[it] = cst;
            if (accept_trace) accept_trace[it] = acc;
            if (alpha_trace) alpha_trace[it] = a_used;
        }
    return 0;
}

/*
 * The interior-point method of Sec. II-B with Alg. 4 as its inner solver,
 * as run in the experiments of Sec. V: barrier levels mu = mu0, mu0 zeta,
 * mu0 zeta^2, ... while mu > mu_min, each solved by Newton iterations until
 * one that starts from a nominal with |dJ_mu/du|_inf <= tol (that
 * iteration's step is still taken), or max_iter iterations.  The nominal,
 * alpha and nu_lm carry over from level to level.  Traces of capacity cap
 * (any NULL): barrier weight, cost after, gradient norm before, predicted
 * decrease and accept flag of every iteration; level_iters gets the
 * iteration count of each
 * level.  Returns the total number of iterations, -1 if u starts infeasible
 * or the model is unknown, -2 if cap is too small.
 */
int oracle_nmpc_ip_solve(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                         const double *Bm, const double *Q, const double *R, const double *QT,
                         const double *xref, const double *x0, double umin, double umax, double mu0,
                         double zeta, double mu_min, double tol, int max_iter, double alpha0, double nu0,
                         double *u, double *x, int cap, double *mu_trace, double *cost_trace,
                         double *grad_trace, double *pred_trace, int *accept_trace, int *level_iters)
{
    if (model_ok(model, nx, nu, prm) != 0 || !(zeta > 0.0 && zeta < 1.0) || !(mu0 > 0.0)) return -1;
    nmpc_prob Pb = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0, NULL, NULL};
    if (rollout(&Pb, u, x) != 0) return -1;
    double alpha = alpha0, nu_lm = nu0;
    int it = 0, lv = 0;
    for (double mu = mu0; mu > mu_min; mu *= zeta, ++lv) {
        int li = 0;
        for (; li < max_iter; ++li) {
            double cst, grad, pred;
            if (it >= cap) return -2;
            int acc = oracle_nmpc_newton_step(nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0,
                                              NULL, NULL, mu, &alpha, &nu_lm, x, u, &cst, &pred, NULL, &grad);
            if (mu_trace) mu_trace[it] = mu;
            if (cost_trace) cost_trace[it] = cst;
            if (grad_trace) grad_trace[it] = grad;
            if (pred_trace) pred_trace[it] = pred;
            if (accept_trace) accept_trace[it] = acc;
            ++it;
            if (grad <= tol) {
                ++li;
                break;
            }
        }
        if (level_iters) level_iters[lv] = li;
    }
    return it;
}

/*
 * ADMM consensus and multiplier steps (eq:admm-step-4, eq:admm-step-5) for the
 * control box: w = h(u) = [u - umax; umin - u] per stage ([T][2 nu] rows),
 * C = {w <= 0}, Pi_C(y) = min(0, y):
 *   init:  z = Pi_C(w), v = 0;
 *   else:  z <- Pi_C(w + v / rho), v <- v + rho (w - z),
 *          *rp = |w - z|_inf, *rd = |z - z_prev|_inf.
 */
void oracle_nmpc_admm_update(int T, int nu, double umin, double umax, double rho, const double *u, double *z,
                             double *v, int init, double *rp_out, double *rd_out)
{
    const int m = nu;
    double rp = 0.0, rd = 0.0;
    for (int k = 0; k < T; ++k)
        for (int i = 0; i < 2 * m; ++i) {
            const double ui = u[(size_t)k * m + (i < m ? i : i - m)];
            const double w = (i < m) ? ui - umax : umin - ui;
            const size_t o = (size_t)k * 2 * m + i;
            if (init) {
                z[o] = fmin(0.0, w);
                v[o] = 0.0;
                continue;
            }
            const double zn = fmin(0.0, w + v[o] / rho);
            rd = fmax(rd, fabs(zn - z[o]));
            rp = fmax(rp, fabs(w - zn));
            z[o] = zn;
            v[o] += rho * (w - zn);
        }
    if (rp_out) *rp_out = rp;
    if (rd_out) *rd_out = rd;
}

/*
 * ADMM of Sec. II-C for the control box, with Alg. 4 as the inner solver of
 * eq:admm-min: w(u) = h(u) = [u - umax; umin - u] per stage, C = {w <= 0}.
 *   z0 = Pi_C(h(u0)) = min(0, h(u0)), v0 = 0;
 *   repeat: Newton iterations on J_AD(u) = J(u) + rho/2 sum |h(u) - z + v/rho|^2
 *           until the iteration that starts from |dJ_AD/du|_inf <= tol (or
 *           max_iter); x the nonlinear rollout (eq:admm-step-2);
 *           z <- min(0, h(u) + v/rho) (eq:admm-step-4, the projection on C);
 *           v <- v + rho (h(u) - z) (eq:admm-step-5);
 *           r_p = h(u) - z, r_d = z - z_prev;
 *   until |r_p|_inf <= eps and |r_d|_inf <= eps, or max_admm iterations.
 * alpha and nu_lm carry over from one ADMM iteration to the next.  z, v
 * ([T][2 nu]) are outputs.  Traces of capacity cap (any NULL): Newton
 * iterations, r_p and r_d of every ADMM iteration.  Returns the number of
 * ADMM iterations, -1 for an unknown model or rho <= 0, -2 if cap is too
 * small; *newton_total gets the Newton iterations over all of them.
 */
int oracle_nmpc_admm_solve(int nx, int nu, int T, double h, int model, const double *prm, const double *W,
                           const double *Bm, const double *Q, const double *R, const double *QT,
                           const double *xref, const double *x0, double umin, double umax, double rho, double eps,
                           double tol, int max_iter, int max_admm, double alpha0, double nu0, double *u, double *x,
                           double *z, double *v, int cap, int *inner_trace, double *rp_trace, double *rd_trace,
                           int *newton_total)
{
    if (model_ok(model, nx, nu, prm) != 0 || !(rho > 0.0)) return -1;
    nmpc_prob Pb = {nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, rho, z, v};
    oracle_nmpc_admm_update(T, nu, umin, umax, rho, u, z, v, 1, NULL, NULL);
    rollout(&Pb, u, x);
    double alpha = alpha0, nu_lm = nu0;
    int total = 0, it = 0;
    for (; it < max_admm; ++it) {
        if (it >= cap) return -2;
        int li = 0;
        for (; li < max_iter; ++li) {
            double cst, grad;
            oracle_nmpc_newton_step(nx, nu, T, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, rho, z, v, 0.0,
                                    &alpha, &nu_lm, x, u, &cst, NULL, NULL, &grad);
            if (grad <= tol) {
                ++li;
                break;
            }
        }
        total += li;
        double rp, rd;
        oracle_nmpc_admm_update(T, nu, umin, umax, rho, u, z, v, 0, &rp, &rd);
        if (inner_trace) inner_trace[it] = li;
        if (rp_trace) rp_trace[it] = rp;
        if (rd_trace) rd_trace[it] = rd;
        if (rp <= eps && rd <= eps) {
            ++it;
            break;
        }
    }
    if (newton_total) *newton_total = total;
    return it;
}

/*
 * Receding-horizon simulation (Sec. V, model predictive control): at every
 * step t the interior-point method with a fixed budget (iters Newton
 * iterations at each barrier weight of mu_levels) solves the N-stage problem
 * from the current state, warm-started with the previous solution shifted by
 * one stage (the last control repeated; the first solve starts from u_init);
 * alpha and nu_lm restart from (alpha0, nu0) at every step.  The first
 * control is applied to the plant, one Euler step of the same model.
 * Outputs: x_cl [steps+1][nx] (x_cl[0] = x_init), u_cl [steps][nu].
 * Returns 0, or -1 for an unknown model or an infeasible u_init.
 */
int oracle_nmpc_mpc_simulate(int nx, int nu, int N, double h, int model, const double *prm, const double *W,
                             const double *Bm, const double *Q, const double *R, const double *QT,
                             const double *xref, const double *x_init, const double *u_init, double umin,
                             double umax, const double *mu_levels, int n_levels, int iters, double alpha0,
                             double nu0, int steps, double *x_cl, double *u_cl)
{
    const int n = nx, m = nu;
    if (model_ok(model, nx, nu, prm) != 0) return -1;
    double *u = malloc(sizeof(double) * (size_t)N * m), *x = malloc(sizeof(double) * (size_t)(N + 1) * n);
    double x0[16];
    memcpy(u, u_init, sizeof(double) * (size_t)N * m);
    memcpy(x0, x_init, sizeof(double) * n);
    memcpy(x_cl, x_init, sizeof(double) * n);
    int st = 0;
    for (int t = 0; t < steps && st == 0; ++t) {
        nmpc_prob Pb = {nx, nu, N, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0, NULL, NULL};
        if (rollout(&Pb, u, x) != 0) {
            st = -1;
            break;
        }
        double alpha = alpha0, nu_lm = nu0;
        for (int lv = 0; lv < n_levels; ++lv)
            for (int i = 0; i < iters; ++i)
                oracle_nmpc_newton_step(nx, nu, N, h, model, prm, W, Bm, Q, R, QT, xref, x0, umin, umax, 0.0, NULL,
                                        NULL, mu_levels[lv], &alpha, &nu_lm, x, u, NULL, NULL, NULL, NULL);
        double xn[16];
        f_step(&Pb, x0, u, xn);
        for (int i = 0; i < m; ++i) u_cl[(size_t)t * m + i] = u[i];
        memcpy(x0, xn, sizeof(double) * n);
        memcpy(x_cl + (size_t)(t + 1) * n, xn, sizeof(double) * n);
        for (int k = 0; k + 1 < N; ++k)
            for (int i = 0; i < m; ++i) u[(size_t)k * m + i] = u[(size_t)(k + 1) * m + i];
    }
    free(u);
    free(x);
    return st;
}
