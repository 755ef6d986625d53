// lq_value.hip -- the value-function pass (Sec. III-C, Alg. 2) on gfx950.
//
// Homogeneous form.  With the constant coordinate appended (n1 = n + 1), a
// value element (A, b, C, eta, J) of eq:value-fun-elements becomes three
// (n+1) x (n+1) matrices
//   A~ = [[A, b], [0, 1]],  C~ = [[C, 0], [0, 0]],  J~ = [[J, -eta], [-eta', const]],
// and the operator eq:value-fun-param becomes pure matrix algebra:
//   X = I + C~1 J~2,  A~ = A~2 X^{-1} A~1,  C~ = A~2 X^{-1} C~1 A~2' + C~2,
//   J~ = A~1' X^{-T} J~2 A~1 + J~1
// (the b and eta rules of eq:value-fun-param are the last columns of the A~
// and J~ rules; the constant J~(n, n) never feeds back into S or s).  The
// value function of stage k is S~_k = J~(nu_k (x) ... (x) nu_{N+1}), i.e.
// S_k = top-left block and s_k = -eta = last column.
//
// Segmented scan, three phases per instance:
//   1. k_value_fold: each wave folds one segment of L stages right to left
//      into one element.  A stage element has C = G G' of rank m, so the
//      operator with a stage element on the left needs only an m x m inverse
//      (Woodbury):  X^{-1} = I - G W^{-1} G'J^,  W = I + G'J^ G.
//   2. k_value_ks: Kogge-Stone suffix scan over the segment elements plus the
//      terminal element, one launch per level, general operator with an
//      (n+1) x (n+1) Gauss-Jordan inverse.
//   3. k_value_riccati: inside each segment the suffix is completed from the
//      right neighbour's value function by the Bellman step (the operator
//      applied to a stage element and a terminal-type element), which also
//      yields the control law of eq:value-fun-feedback.
#include "lq_kernels.hpp"

namespace lqk {

constexpr int ERR_NOT_PD = -2;
constexpr int ERR_SINGULAR = -3;
constexpr int ERR_NONFINITE = -4;

struct StageElem {
    Tile Ab;  // A~ - G N      ((n+1) x (n+1))
    Tile G;   // B~ L^{-T}     ((n+1) x m), C~ = G G'
    Tile J;   // Q~ - N' N     ((n+1) x (n+1)),  N = L^{-1} M~'
};

// Raw stage data of the element build, loaded one stage ahead of its use.
struct StageRaw {
    Tile A, Q;                // A~ and Q~ (homogeneous)
    double brow[4][MMAX];     // B at this lane's four rows
    double R[MMAX][MMAX];     // R (identity-padded)
    double mt[MMAX];          // M~ at this lane's column: M[c][b] (c < n) or r[b] (c == n)
};

LQK_DEV void load_stage_raw(const ProbPtrs &P, const InstDesc &d, int k, StageRaw &w)
{
    const int n = d.n, m = d.m, c = tcol();
    w.A = load_Ah(P, d, k);
    w.Q = load_Qh(P, d, k);
    const double *Bk = P.B + d.oB + (int64_t)k * n * m;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
#pragma unroll
        for (int b = 0; b < MMAX; ++b) w.brow[r][b] = ldz(Bk, (int64_t)i * m + b, i < n && b < m);
    }
    const double *Rk = P.R + d.oR + (int64_t)k * m * m;
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
            const int ii = i < m ? i : 0, jj = j < m ? j : 0;
            const double v = Rk[ii * m + jj];
            w.R[i][j] = (i < m && j < m) ? v : (i == j ? 1.0 : 0.0);
        }
    const double *Mk = P.M ? P.M + d.oB + (int64_t)k * n * m : nullptr;
    const double *rk = P.r ? P.r + d.og + (int64_t)k * m : nullptr;
#pragma unroll
    for (int b = 0; b < MMAX; ++b)
        w.mt[b] = *(Mk && c < n && b < m ? Mk + c * m + b : (rk && c == n && b < m ? rk + b : zptr()));
}

// Stage element of eq:value-fun-elem-init in the P^{-1}-free form, from the
// stage data (R = L L').  Returns false if R is not positive definite.
template <int PR>
LQK_DEV bool build_from_raw(const StageRaw &w, const InstDesc &d, bool has_mr, StageElem &e, double *s0,
                            double *s1)
{
    const int n = d.n, m = d.m, c = tcol();
    double li[MMAX][MMAX];
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) li[i][j] = w.R[i][j];
    const bool ok = small_chol(li);
    small_tri_inv(li);
    // row c of L^{-1}: G[i][c] = sum_b B[i][b] Linv[c][b]
    double lrow[MMAX];
#pragma unroll
    for (int b = 0; b < MMAX; ++b) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < MMAX; ++a) t = (a == c) ? li[a][b] : t;
        lrow[b] = t;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < MMAX; ++b) v += w.brow[r][b] * lrow[b];
        e.G.v[r] = (i < n && c < m) ? v : 0.0;
    }
    e.Ab = w.A;
    e.J = w.Q;
    if (has_mr) {
        // N[a][j] = sum_b Linv[a][b] M~[j][b]; rows a < m <= 4 are register 0 of lane group a.
        const int g = tgrp();
        Tile N = tzero();
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < MMAX; ++b) {
            double lg = 0.0;
#pragma unroll
            for (int a = 0; a < MMAX; ++a) lg = (a == g) ? li[a][b] : lg;
            v += lg * w.mt[b];
        }
        N.v[0] = (g < m) ? v : 0.0;
        e.Ab = tsub(e.Ab, mmk<1, PR, false, false>(e.G, N, s0, s1));
        e.J = tsub(e.J, mmk<1, PR, true, false>(N, N, s0, s1));
    }
    return ok;
}

template <int PR>
LQK_DEV bool build_stage_elem(const ProbPtrs &P, const InstDesc &d, int k, StageElem &e, double *s0, double *s1)
{
    StageRaw w;
    load_stage_raw(P, d, k, w);
    return build_from_raw<PR>(w, d, (P.M != nullptr) || (P.r != nullptr), e, s0, s1);
}

// Left fold of a stage element into an aggregate E = (A^, C^, J^):
// E <- e_k (x) E with the rank-m Woodbury form of the operator.
// Returns false if W = I + G'J^G is singular.
template <int NK, int PR>
LQK_DEV bool fold_left(const StageElem &e, Tile &Ah, Tile &Ch, Tile &Jh, int m,
                       double *s0, double *s1, double *s2, double *s3)
{
    const d4 z = (d4){0.0, 0.0, 0.0, 0.0};
    wsync();
    sputp<PR>(s0, Jh);
    sputp<PR>(s1, e.G);
    sputp<PR>(s2, Ah);
    sputp<PR>(s3, e.Ab);
    wsync();
    Tile JG, H, JA, AA;
    JG.v = mfma_k<NK, PR, false, false>(s0, s1, z);   // J^ G
    H.v = mfma_k<NK, PR, false, false>(s2, s1, z);    // A^ G
    JA.v = mfma_k<NK, PR, false, false>(s0, s3, z);   // J^ Ab
    AA.v = mfma_k<NK, PR, false, false>(s2, s3, z);   // A^ Ab
    wsync();
    sputp<PR>(s0, JG);
    sputp<PR>(s2, JA);
    wsync();
    Tile W, P, Jn;
    W.v = mfma_k<NK, PR, true, false>(s1, s0, tident(m).v);  // I + G'J^G
    P.v = mfma_k<NK, PR, true, false>(s1, s2, z);             // G'J^ Ab
    Jn.v = mfma_k<NK, PR, true, false>(s3, s2, e.J.v);        // Ab'J^ Ab + J
    Tile Wi;
    const bool ok = gen_inverse_small(W, m, Wi, s0);
    wsync();
    sputp<PR>(s0, Wi);
    sputp<PR>(s1, P);
    sputp<PR>(s2, H);
    wsync();
    Tile WP, WH;
    WP.v = mfma_k<1, PR, false, false>(s0, s1, z);   // W^{-1} P
    WH.v = mfma_k<1, PR, false, true>(s0, s2, z);    // W^{-1} H'
    wsync();
    sputp<PR>(s3, WP);
    sputp<PR>(s0, WH);
    wsync();
    Tile t;
    t.v = mfma_k<1, PR, false, false>(s2, s3, z);    // H W^{-1} P
    Ah.v = AA.v - t.v;
    Ch.v = mfma_k<1, PR, false, false>(s2, s0, Ch.v); // C^ + H W^{-1} H'
    t.v = mfma_k<1, PR, true, false>(s1, s3, z);      // P' W^{-1} P
    Jh.v = Jn.v - t.v;
    wsync();
    return ok;
}

// ---------------------------------------------------------------------------
// Element build (materialised)
// ---------------------------------------------------------------------------
template <int PR>
__global__ __launch_bounds__(64) void k_build_elements(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                       const int64_t *__restrict__ elem_start, int batch,
                                                       double *__restrict__ elems, int32_t *status)
{
    __shared__ double lds[2 * SLOT];
    const int64_t ge = blockIdx.x;
    const int i = find_inst64(elem_start, batch, ge);
    const InstDesc d = inst[i];
    const int k = (int)(ge - d.elem0);
    double *out = elems + ge * 4 * TILE;
    if (k == d.T) {  // terminal element nu_{N+1}
        gstore(out, corner(d.n));
        gstore(out + TILE, tzero());
        gstore(out + 2 * TILE, load_terminal_J(P, d, lds));
        gstore(out + 3 * TILE, tzero());
        return;
    }
    StageElem e;
    const bool ok = build_stage_elem<PR>(P, d, k, e, lds, lds + SLOT);
    const Tile C = mmk<1, PR, false, true>(e.G, e.G, lds, lds + SLOT);
    gstore(out, e.Ab);
    gstore(out + TILE, C);
    gstore(out + 2 * TILE, e.J);
    gstore(out + 3 * TILE, e.G);
    if (!ok) report(status, i, ERR_NOT_PD, k);
}

// ---------------------------------------------------------------------------
// Phase 1: fold each segment into one element; also write the terminal
// element after the last segment of each instance.
// Scan buffer entry = 3 tiles (A~, C~, J~).
// ---------------------------------------------------------------------------
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_fold(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                   const int32_t *__restrict__ seg_start, int batch,
                                                   const double *__restrict__ elems, double *__restrict__ X,
                                                   int32_t *status)
{
    __shared__ double lds[4 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT, *s2 = lds + 2 * SLOT, *s3 = lds + 3 * SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n1 = d.n + 1, m = d.m;
    Tile Ah = tident(n1), Ch = tzero(), Jh = tzero();
    int code = 0, fk = 0;
    (void)n1;
    if (s == d.nseg - 1) {  // terminal element after the last segment
        double *t = X + (int64_t)(d.xbase + d.nseg) * 3 * TILE;
        gstore(t, corner(d.n));
        gstore(t + TILE, tzero());
        gstore(t + 2 * TILE, load_terminal_J(P, d, s0));
    }
    // The element of segment 0 is never read: the Bellman steps of segment s
    // start from the scanned element s + 1.
    if (s == 0) return;
    if (elems) {
        for (int k = k1 - 1; k >= k0; --k) {
            StageElem e;
            const double *ep = elems + (d.elem0 + k) * 4 * TILE;
            e.Ab = gload(ep);
            e.J = gload(ep + 2 * TILE);
            e.G = gload(ep + 3 * TILE);
            if (!fold_left<NK, PR>(e, Ah, Ch, Jh, m, s0, s1, s2, s3) && !code) {
                code = ERR_SINGULAR;
                fk = k;
            }
        }
    } else {
        // fused element build; the raw data of stage k-1 is loaded while stage k is folded
        const bool has_mr = (P.M != nullptr) || (P.r != nullptr);
        StageRaw cur, nxt;
        load_stage_raw(P, d, k1 - 1, cur);
        for (int k = k1 - 1; k >= k0; --k) {
            if (k > k0) load_stage_raw(P, d, k - 1, nxt);
            StageElem e;
            if (!build_from_raw<PR>(cur, d, has_mr, e, s0, s1) && !code) {
                code = ERR_NOT_PD;
                fk = k;
            }
            if (!fold_left<NK, PR>(e, Ah, Ch, Jh, m, s0, s1, s2, s3) && !code) {
                code = ERR_SINGULAR;
                fk = k;
            }
            if (k > k0) cur = nxt;
        }
    }
    double *o = X + (int64_t)(d.xbase + s) * 3 * TILE;
    gstore(o, Ah);
    gstore(o + TILE, Ch);
    gstore(o + 2 * TILE, Jh);
    if (code) report(status, i, code, fk);
}

// ---------------------------------------------------------------------------
// Phase 2: one Kogge-Stone level of the suffix scan, X_s <- X_s (x) X_{s+dd}.
// Before the level, X_s covers segments [s, s+dd-1] (clipped at the terminal
// index nseg); it is terminal-type (A~ = corner, C~ = 0, only J~ meaningful)
// once it covers nseg.  Terminal-type entries are only ever right operands.
// ---------------------------------------------------------------------------
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_ks(const InstDesc *__restrict__ inst,
                                                 const int32_t *__restrict__ x_start, int batch, int dd,
                                                 const double *__restrict__ Xin, double *__restrict__ Xout,
                                                 int32_t *status)
{
    __shared__ double lds[4 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT, *s2 = lds + 2 * SLOT, *s3 = lds + 3 * SLOT;
    const int gx = blockIdx.x;
    const int i = find_inst(x_start, batch, gx);
    const InstDesc d = inst[i];
    const int s = gx - d.xbase;
    const int nseg = d.nseg;
    const double *a = Xin + (int64_t)gx * 3 * TILE;
    double *o = Xout + (int64_t)gx * 3 * TILE;
    if (s == 0) return;   // never read (see k_value_fold)
    if (s + dd > nseg) {  // already final (terminal-type): carry J~ over
        gstore(o + 2 * TILE, gload(a + 2 * TILE));
        return;
    }
    const double *b = Xin + (int64_t)(gx + dd) * 3 * TILE;
    const bool b_term = (s + 2 * dd - 1 >= nseg);
    const int n1 = d.n + 1;
    const d4 z = (d4){0.0, 0.0, 0.0, 0.0};
    const Tile A1 = gload(a), C1 = gload(a + TILE), J1 = gload(a + 2 * TILE);
    const Tile J2 = gload(b + 2 * TILE);
    // X = I + C~1 J~2
    sputp<PR>(s0, C1);
    sputp<PR>(s1, J2);
    wsync();
    Tile Xt;
    Xt.v = mfma_k<NK, PR, false, false>(s0, s1, tident(n1).v);
    const bool ok = gj_inverse(Xt, n1, s2);
    wsync();
    sputp<PR>(s3, Xt);  // X^{-1}
    wsync();
    Tile T3;
    T3.v = mfma_k<NK, PR, false, false>(s1, s3, z);   // J~2 X^{-1} = (X^{-T} J~2)'
    wsync();
    sputp<PR>(s0, T3);
    sputp<PR>(s2, A1);
    wsync();
    Tile T4;
    T4.v = mfma_k<NK, PR, true, false>(s0, s2, z);    // X^{-T} J~2 A~1
    wsync();
    sputp<PR>(s1, T4);
    wsync();
    Tile Jn;
    Jn.v = mfma_k<NK, PR, true, false>(s2, s1, J1.v); // A~1' X^{-T} J~2 A~1 + J~1
    Jn = tsym(Jn, s0);
    gstore(o + 2 * TILE, Jn);
    if (!b_term) {
        const Tile A2 = gload(b), C2 = gload(b + TILE);
        wsync();
        sputp<PR>(s0, A2);
        wsync();
        Tile T1;
        T1.v = mfma_k<NK, PR, false, false>(s0, s3, z);   // A~2 X^{-1}
        wsync();
        sputp<PR>(s1, T1);
        wsync();
        Tile An;
        An.v = mfma_k<NK, PR, false, false>(s1, s2, z);   // A~2 X^{-1} A~1
        wsync();
        sputp<PR>(s3, C1);
        wsync();
        Tile T2;
        T2.v = mfma_k<NK, PR, false, false>(s1, s3, z);   // A~2 X^{-1} C~1
        wsync();
        sputp<PR>(s2, T2);
        wsync();
        Tile Cn;
        Cn.v = mfma_k<NK, PR, false, true>(s2, s0, C2.v); // ... A~2' + C~2
        Cn = tsym(Cn, s1);
        gstore(o, An);
        gstore(o + TILE, Cn);
    }
    if (!ok) report(status, i, ERR_SINGULAR, s);
}

// ---------------------------------------------------------------------------
// Phase 3: Bellman steps inside each segment from the right neighbour's value
// function S~' (the carry), writing S_k, s_k, Gamma_k, gamma_k.
//   S~'B~, S~'A~;  Q_uu = R + B~'S~'B~;  Q_ux~ = M~' + B~'S~'A~;
//   Gamma~ = -Q_uu^{-1} Q_ux~ = [Gamma, gamma];
//   S~ = sym(Q~ + A~'S~'A~ + Q_ux~' Gamma~).
// ---------------------------------------------------------------------------
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_riccati(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      const double *__restrict__ Xfin, ValPtrs V,
                                                      int32_t *status)
{
    __shared__ double lds[4 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT, *s2 = lds + 2 * SLOT, *s3 = lds + 3 * SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    const d4 z = (d4){0.0, 0.0, 0.0, 0.0};
    const bool has_mr = (P.M != nullptr) || (P.r != nullptr);
    Tile St = gload(Xfin + (int64_t)(d.xbase + s + 1) * 3 * TILE + 2 * TILE);
    if (s == d.nseg - 1) {
        gstore_rm(V.S + d.oS + (int64_t)d.T * n * n, St, n, n, n);
        store_vec(V.s + d.os + (int64_t)d.T * n, St, n, n);
    }
    int code = 0, fk = 0;
    // stage data of stage k-1 is loaded while stage k is processed
    Tile nAh = load_Ah(P, d, k1 - 1), nBh = load_Bh(P, d, k1 - 1), nQh = load_Qh(P, d, k1 - 1);
    Tile nRk = load_R(P, d, k1 - 1), nMhT = has_mr ? load_MhT(P, d, k1 - 1) : tzero();
    for (int k = k1 - 1; k >= k0; --k) {
        const Tile Ah = nAh, Bh = nBh, Qh = nQh, Rk = nRk, MhT = nMhT;
        if (k > k0) {
            nAh = load_Ah(P, d, k - 1);
            nBh = load_Bh(P, d, k - 1);
            nQh = load_Qh(P, d, k - 1);
            nRk = load_R(P, d, k - 1);
            if (has_mr) nMhT = load_MhT(P, d, k - 1);
        }
        wsync();
        sputp<PR>(s0, St);
        sputp<PR>(s1, Bh);
        sputp<PR>(s2, Ah);
        wsync();
        Tile SB, SA;
        SB.v = mfma_k<NK, PR, false, false>(s0, s1, z);
        SA.v = mfma_k<NK, PR, false, false>(s0, s2, z);
        wsync();
        sputp<PR>(s3, SB);
        sputp<PR>(s0, SA);
        wsync();
        Tile Quu, Qux, Sn;
        Quu.v = mfma_k<NK, PR, true, false>(s1, s3, Rk.v);
        Qux.v = mfma_k<NK, PR, true, false>(s1, s0, MhT.v);
        Sn.v = mfma_k<NK, PR, true, false>(s2, s0, Qh.v);
        Tile Qi;
        if (!spd_inverse(Quu, m, Qi, s3) && !code) {
            code = ERR_NOT_PD;
            fk = k;
        }
        wsync();
        sputp<PR>(s3, Qi);
        sputp<PR>(s1, Qux);
        wsync();
        Tile Gh;
        Gh.v = -mfma_k<1, PR, false, false>(s3, s1, z);
        wsync();
        sputp<PR>(s3, Gh);
        wsync();
        Sn.v = mfma_k<1, PR, true, false>(s1, s3, Sn.v);
        St = tsym(Sn, s0);
        gstore_rm(V.S + d.oS + (int64_t)k * n * n, St, n, n, n);
        store_vec(V.s + d.os + (int64_t)k * n, St, n, n);
        gstore_rm(V.G + d.oG + (int64_t)k * m * n, Gh, m, n, n);
        store_vec(V.g + d.og + (int64_t)k * m, Gh, m, n);
    }
    const bool bad = !(isfinite(St.v[0]) && isfinite(St.v[1]) && isfinite(St.v[2]) && isfinite(St.v[3]));
    if (__ballot(bad) && !code) {
        code = ERR_NONFINITE;
        fk = k0;
    }
    if (code) report(status, i, code, fk);
}

// ---------------------------------------------------------------------------
// Host launchers (the contraction slice count NK = ceil((n_max + 1) / 4) is a
// template parameter so that every product is fully unrolled).
// ---------------------------------------------------------------------------

void launch_value_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *elems, double *X, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_value_fold<K, R>), dim3(grid), dim3(64), 0, st, P, inst, seg_start, batch, elems, X, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_value_ks(int nk, int pr, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                     int batch, int dd, const double *Xin, double *Xout, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_value_ks<K, R>), dim3(grid), dim3(64), 0, st, inst, x_start, batch, dd, Xin, Xout, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_value_riccati(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                          const int32_t *seg_start, int batch, const double *Xfin, ValPtrs V, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_value_riccati<K, R>), dim3(grid), dim3(64), 0, st, P, inst, seg_start, batch, Xfin, V, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

// Diagnostic: D = op(X) op(Y) (+ Z) for row-major 16 x 16 inputs.
template <int PR>
__global__ __launch_bounds__(64) void k_selftest_mm(const double *X, const double *Y, const double *Z,
                                                    double *D, int tx, int ty)
{
    __shared__ double lds[2 * SLOT];
    const Tile x = gload_rm(X, 16, 16, 16), y = gload_rm(Y, 16, 16, 16);
    const Tile zt = Z ? gload_rm(Z, 16, 16, 16) : tzero();
    Tile d;
    if (tx && ty)
        d = mmak<4, PR, true, true>(x, y, zt, lds, lds + SLOT);
    else if (tx)
        d = mmak<4, PR, true, false>(x, y, zt, lds, lds + SLOT);
    else if (ty)
        d = mmak<4, PR, false, true>(x, y, zt, lds, lds + SLOT);
    else
        d = mmak<4, PR, false, false>(x, y, zt, lds, lds + SLOT);
    gstore_rm(D, d, 16, 16, 16);
}

void launch_build_elements(int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                           const int64_t *elem_start, int batch, double *elems, int32_t *status)
{
    if (pr)
        hipLaunchKernelGGL(k_build_elements<1>, dim3(grid), dim3(64), 0, st, P, inst, elem_start, batch, elems, status);
    else
        hipLaunchKernelGGL(k_build_elements<0>, dim3(grid), dim3(64), 0, st, P, inst, elem_start, batch, elems, status);
}

void launch_selftest_mm(int pr, hipStream_t st, const double *X, const double *Y, const double *Z, double *D, int tx,
                        int ty)
{
    if (pr)
        hipLaunchKernelGGL(k_selftest_mm<1>, dim3(1), dim3(64), 0, st, X, Y, Z, D, tx, ty);
    else
        hipLaunchKernelGGL(k_selftest_mm<0>, dim3(1), dim3(64), 0, st, X, Y, Z, D, tx, ty);
}

}  // namespace lqk
