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
//      into one element (the last segment onto the terminal element, so its
//      element is already a whole suffix).  A stage element has
//      C~ = B~ R^{-1} B~' of rank m, so
//      the operator with a stage element on the left needs only an m x m
//      inverse (Woodbury):  X^{-1} = I - B~ W^{-1} B~'J^,  W = R + B~'J^ B~,
//      and no factorisation of R itself (R enters only through W).
//   2. k_value_ks: Kogge-Stone suffix scan over the segment elements 1 ..
//      nseg-1, one launch per level, general operator with an
//      (n+1) x (n+1) Gauss-Jordan inverse (of X', which is what the products
//      need).
//   3. k_value_riccati: inside each segment the suffix is completed from the
//      right neighbour's value function by the Bellman step (the operator
//      applied to a stage element and a terminal-type element), which also
//      yields the control law of eq:value-fun-feedback.
#include "lq_kernels.hpp"

// Every product is P'Q of register tiles (tn in lq_tile.hpp); the fold keeps
// the aggregate A^ transposed so that none of its products needs a transpose.
namespace lqk {

constexpr int ERR_NOT_PD = -2;
constexpr int ERR_SINGULAR = -3;
constexpr int ERR_NONFINITE = -4;

// Stage element of eq:value-fun-elem-init for the fold, in the form
// C~ = B~ W0^{-1} B~' (W0 = R from the problem data, W0 = I for a stored
// element whose B~ is already B~ L^{-T}).
struct StageElem {
    Tile Ab;  // A~ - B~ R^{-1} M~'   ((n+1) x (n+1))
    Tile B;   // B~                    ((n+1) x m)
    Tile J;   // Q~ - M~ R^{-1} M~'    ((n+1) x (n+1))
    Tile W0;  // R                     (m x m)
};

// Stage data of the fused element build, loaded ahead of its use.  MR: the
// cross-term tiles M~' and B~' are needed (M or r present).
template <bool MR>
struct StageRaw {
    Tile A, Q, B, R;   // A~, Q~, B~, R
    Tile MT, BT;       // M~' = [M', r] and B~' (MR only)
};

// The stage element from its data.  With cross terms the Schur complement
// needs R^{-1}: false if R is not positive definite.
template <int PR, bool MR>
LQK_DEV bool build_from_raw(const StageRaw<MR> &w, const InstDesc &d, StageElem &e)
{
    e.Ab = w.A;
    e.B = w.B;
    e.J = w.Q;
    e.W0 = w.R;
    bool ok = true;
    if constexpr (MR) {
        Tile RiT;
        ok = spd_inverse_t(w.R, d.m, RiT);
        const Tile K = tnz<1, PR>(RiT, w.MT);   // R^{-1} M~'
        e.Ab.v -= tn<1, PR>(w.BT, K, (d4){0.0, 0.0, 0.0, 0.0});
        e.J.v -= tn<1, PR>(w.MT, K, (d4){0.0, 0.0, 0.0, 0.0});
    }
    return ok;
}

// Left fold of a stage element into an aggregate E = (A^, C^, J^), A^ held as
// U = A^': E <- e_k (x) E with the rank-m Woodbury form of the operator:
//   W = W0 + B~'J^B~,  P = B~'J^A~,  H = A^B~,
//   A^ <- A^A~ - H W^{-1} P,  C^ <- C^ + H W^{-1} H',  J^ <- J~ + A~'J^A~ - P'W^{-1}P.
// NB: contraction slices over the rows of B~ (its homogeneous row is zero, so
// ceil(n / 4) slices suffice).  W comes first: the m x m inverse (vector
// instructions) then overlaps the five products that do not depend on it
// (matrix instructions).  Returns false if W is singular.
template <int NK, int NB, int PR>
LQK_DEV bool fold_left(const StageElem &e, Tile &U, Tile &Ch, Tile &Jh, int m)
{
    const d4 z = (d4){0.0, 0.0, 0.0, 0.0};
    const Tile JG = tnz<NB, PR>(Jh, e.B);         // J^ B~
    const Tile W = tna<NB, PR>(e.B, JG, e.W0);    // W0 + B~'J^B~
    Tile WiT;
    const bool ok = gen_inverse_t(W, m, WiT);
    const Tile JA = tnz<NK, PR>(Jh, e.Ab);        // J^ A~
    const Tile Pm = tnz<NB, PR>(e.B, JA);         // B~'J^A~
    const Tile Jn = tna<NK, PR>(e.Ab, JA, e.J);   // J~ + A~'J^A~
    const Tile Ht = tnz<NB, PR>(e.B, U);          // H' = B~'A^'
    const Tile AAt = tnz<NK, PR>(e.Ab, U);        // (A^A~)'
    const Tile WP = tnz<1, PR>(WiT, Pm);          // W^{-1} P
    const Tile WHt = tnz<1, PR>(WiT, Ht);         // W^{-1} H'
    U.v = AAt.v - tn<1, PR>(WP, Ht, z);           // (A^A~ - H W^{-1} P)'
    Ch = tna<1, PR>(Ht, WHt, Ch);                 // C^ + H W^{-1} H'
    Jh.v = Jn.v - tn<1, PR>(Pm, WP, z);           // ... - P'W^{-1}P
    return ok;
}

// First failure of a segment, recorded without branching: code/fk keep the
// first (largest k, the fold runs right to left) failing stage.
LQK_DEV void note(bool ok, int err, int k, int &code, int &fk)
{
    const bool first = !ok && (code == 0);
    code = first ? err : code;
    fk = first ? k : fk;
}

// Fused element build + fold over stages k1-1 .. k0 (right to left).  The
// stage data comes through LDS (sweep_ahead2 / gather), loaded two stages
// ahead.
//
// J^ is symmetrised after every stage, as the Bellman sweep does with S: its
// update carries a rounding error whose antisymmetric part the Riccati
// contraction does not damp, so over a long segment with unstable dynamics it
// grows like the products of the stages' A (measured: 3e-11 relative after
// 137 stages of a random n = 13 instance, 3e-16 with the symmetrisation).
template <int NK, int NB, int PR, bool MR>
LQK_DEV void fold_fused(const ProbPtrs &P, const InstDesc &d, int k0, int k1, Tile &U, Tile &Ch, Tile &Jh,
                        int &code, int &fk, double *stg, double *lds)
{
    constexpr int SZ = stage_buf_size<NK>();
    const int n = d.n, m = d.m;
    const StageLayout L = stage_layout(n, m);
    const ValueStage<NK, MR> VS = value_stage<NK, MR>(P, d, L);
    stage_consts(stg);
    stage_consts(stg + SZ);
    sweep_ahead2<typename ValueStage<NK, MR>::Regs>(stg, SZ, VS.a, L.trash, k1 - 1, k1 - k0, -1,
                                                     [&](int k, const double *cur) {
        StageRaw<MR> w;
        w.A = gather(cur, gmap_Ah(L, n));
        w.Q = gather(cur, gmap_Qh(L, n));
        w.B = gather(cur, gmap_Bh(L, n, m));
        w.R = gather(cur, gmap_R(L, m));
        if constexpr (MR) {
            w.MT = gather(cur, gmap_MhT(L, n, m));
            w.BT = gather(cur, gmap_BhT(L, n, m));
        }
        StageElem e;
        note(build_from_raw<PR, MR>(w, d, e), ERR_NOT_PD, k, code, fk);
        note(fold_left<NK, NB, PR>(e, U, Ch, Jh, d.m), ERR_SINGULAR, k, code, fk);
        Jh = tsym(Jh, lds);
    });
}

// The fused fold for the slice count of B~'s rows: NK - 1 when n is a multiple
// of 4 (then B~'s rows fit one slice fewer than n + 1), NK otherwise.
template <int NK, int PR, bool MR>
LQK_DEV void fold_fused_nb(const ProbPtrs &P, const InstDesc &d, int k0, int k1, Tile &U, Tile &Ch, Tile &Jh,
                           int &code, int &fk, double *stg, double *lds)
{
    if (NK > 1 && (d.n & 3) == 0)
        fold_fused<NK, (NK > 1 ? NK - 1 : 1), PR, MR>(P, d, k0, k1, U, Ch, Jh, code, fk, stg, lds);
    else
        fold_fused<NK, NK, PR, MR>(P, d, k0, k1, U, Ch, Jh, code, fk, stg, lds);
}

// ---------------------------------------------------------------------------
// Element build (materialised): A~ - G N, C~ = G G', J~ - N'N, G = B~ L^{-T},
// N = L^{-1} M~', R = L L'.
// ---------------------------------------------------------------------------
template <int PR>
__global__ __launch_bounds__(64) void k_build_elements(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                       const int64_t *__restrict__ elem_start, int batch,
                                                       double *__restrict__ elems, int32_t *status)
{
    __shared__ double lds[SLOT];
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
    const bool has_mr = (P.M != nullptr) || (P.r != nullptr);
    const Tile BT = load_BhT(P, d, k);
    double li[MMAX][MMAX];
    small_from_tile(load_R(P, d, k), d.m, li);
    const bool ok = small_chol_inv(li);
    const Tile Lt = small_to_tile<true>(li, d.m);   // L^{-T}
    const Tile G = tnz<1, PR>(BT, Lt);              // B~ L^{-T}
    const Tile GT = tnz<1, PR>(Lt, BT);             // L^{-1} B~'
    Tile Ab = load_Ah(P, d, k), J = load_Qh(P, d, k);
    if (has_mr) {
        const Tile N = tnz<1, PR>(Lt, load_MhT(P, d, k));
        Ab.v -= tn<1, PR>(GT, N, (d4){0.0, 0.0, 0.0, 0.0});
        J.v -= tn<1, PR>(N, N, (d4){0.0, 0.0, 0.0, 0.0});
    }
    gstore(out, Ab);
    gstore(out + TILE, tnz<1, PR>(GT, GT));
    gstore(out + 2 * TILE, J);
    gstore(out + 3 * TILE, G);
    if (!ok) report(status, d.orig, ERR_NOT_PD, k);
}

// ---------------------------------------------------------------------------
// Phase 1: fold each segment s >= 1 into one element at entry s, the last
// segment onto the terminal element.
// Scan buffer entry = 3 tiles (A~, C~, J~), each stored compactly: its n1 x n1
// block row-major at the start of a TILE slot (gload_c / gstore_c).
// ---------------------------------------------------------------------------
//
// prefix = 1 lays the entries out for the prefix scan of the conditional-value
// states instead: the unit element at entry 0, segment s's element at entry
// s + 1 (the last segment's element is never read), no terminal element.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_fold(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                   const int32_t *__restrict__ seg_start, int batch,
                                                   const double *__restrict__ elems, double *__restrict__ X,
                                                   int prefix, int32_t *status)
{
    __shared__ double lds[SLOT];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n1 = d.n + 1, m = d.m;
    Tile U = tident(n1), Ch = tzero(), Jh = tzero();
    int code = 0, fk = 0;
    if (prefix) {
        if (s == 0) {
            double *t = X + (int64_t)d.xbase * 3 * TILE;
            gstore_c(t, tident(n1), n1);
            gstore_c(t + TILE, tzero(), n1);
            gstore_c(t + 2 * TILE, tzero(), n1);
        }
        if (s == d.nseg - 1) return;
    } else {
        // The element of segment 0 is never read: the Bellman steps of
        // segment s start from the scanned element s + 1 (the last segment's
        // from the terminal element itself).
        if (s == 0) return;
        // The last segment folds onto the terminal element, so its entry is
        // already the whole suffix (terminal-type) and the scan has one entry
        // less.
        if (s == d.nseg - 1) {
            U = corner(d.n);
            Jh = load_terminal_J(P, d, lds);
        }
    }
    if (elems) {
        for (int k = k1 - 1; k >= k0; --k) {
            StageElem e;
            const double *ep = elems + (d.elem0 + k) * 4 * TILE;
            e.Ab = gload(ep);
            e.J = gload(ep + 2 * TILE);
            e.B = gload(ep + 3 * TILE);
            e.W0 = tident(m);
            note(fold_left<NK, NK, PR>(e, U, Ch, Jh, m), ERR_SINGULAR, k, code, fk);
            Jh = tsym(Jh, lds);   // as in fold_fused
        }
    } else {
        // fused element build
        __shared__ double stg[2 * stage_buf_size<NK>()];
        if ((P.M != nullptr) || (P.r != nullptr))
            fold_fused_nb<NK, PR, true>(P, d, k0, k1, U, Ch, Jh, code, fk, stg, lds);
        else
            fold_fused_nb<NK, PR, false>(P, d, k0, k1, U, Ch, Jh, code, fk, stg, lds);
    }
    double *o = X + (int64_t)(d.xbase + s + prefix) * 3 * TILE;
    gstore_c(o, ttrans(U, lds), n1);
    gstore_c(o + TILE, tsym(Ch, lds), n1);
    gstore_c(o + 2 * TILE, tsym(Jh, lds), n1);
    if (code) report(status, d.orig, code, fk);
}

// ---------------------------------------------------------------------------
// Phase 2: one Kogge-Stone level of the suffix scan, X_s <- X_s (x) X_{s+dd}.
// Before the level, X_s covers segments [s, s+dd-1] (clipped at the last
// segment nseg-1, whose element includes the terminal); it is terminal-type
// (A~ = corner, C~ = 0, only J~ meaningful) once it covers nseg-1.
// Terminal-type entries are only ever right operands.
// With Y = X^{-1}, the products are
//   Z = Y A~1,  J~ = Z'(J~2 A~1) + J~1,  A~ = A~2 Z,  C~ = A~2 (Y C~1) A~2' + C~2,
// all P'Q of register tiles given R(Y') (the inverse of X' = I + J~2 C~1) and
// R(A~2') (one LDS transpose).
// ---------------------------------------------------------------------------
//
// prefix = 1: the inclusive prefix scan X_s <- X_{s-dd} (x) X_s over entries
// 0 .. nseg-1 (laid out by k_value_fold with prefix = 1), general elements
// throughout; an entry with s < dd is final and copied.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_ks(const InstDesc *__restrict__ inst,
                                                 const int32_t *__restrict__ x_start, int batch, int dd,
                                                 int prefix, const double *__restrict__ Xin,
                                                 double *__restrict__ Xout, int32_t *status)
{
    __shared__ double lds[SLOT];
    const int gx = blockIdx.x;
    const int i = find_inst(x_start, batch, gx);
    const InstDesc d = inst[i];
    const int s = gx - d.xbase;
    const int nseg = d.nseg;
    const int n1 = d.n + 1;
    double *o = Xout + (int64_t)gx * 3 * TILE;
    const double *a, *b;
    bool b_term;
    if (prefix) {
        if (s >= nseg) return;
        const double *e = Xin + (int64_t)gx * 3 * TILE;
        if (s < dd) {
            gstore_c(o, gload_c(e, n1), n1);
            gstore_c(o + TILE, gload_c(e + TILE, n1), n1);
            gstore_c(o + 2 * TILE, gload_c(e + 2 * TILE, n1), n1);
            return;
        }
        a = Xin + (int64_t)(gx - dd) * 3 * TILE;
        b = e;
        b_term = false;
    } else {
        // entries 1 .. nseg-1; the last already covers the terminal element
        a = Xin + (int64_t)gx * 3 * TILE;
        const int last = nseg - 1;
        if (s == 0 || s > last) return;   // never read (see k_value_fold)
        if (s + dd > last) {              // already final (terminal-type): carry J~ over
            gstore_c(o + 2 * TILE, gload_c(a + 2 * TILE, n1), n1);
            return;
        }
        b = Xin + (int64_t)(gx + dd) * 3 * TILE;
        b_term = (s + 2 * dd - 1 >= last);
    }
    const Tile A1 = gload_c(a, n1), C1 = gload_c(a + TILE, n1), J1 = gload_c(a + 2 * TILE, n1);
    const Tile A2 = gload_c(b, n1), C2 = gload_c(b + TILE, n1), J2 = gload_c(b + 2 * TILE, n1);
    Tile YT = tna<NK, PR>(J2, C1, tident(n1));   // X' = I + J~2 C~1 = [[I + J C, 0], [-eta' C, 1]]
    const bool ok = gj_inverse<NK>(YT, n1, true);   // X^{-T}
    const Tile Z = tnz<NK, PR>(YT, A1);          // X^{-1} A~1
    const Tile JA = tnz<NK, PR>(J2, A1);         // J~2 A~1
    const Tile Jn = tna<NK, PR>(Z, JA, J1);      // A~1'X^{-T}J~2 A~1 + J~1
    gstore_c(o + 2 * TILE, tsym(Jn, lds), n1);
    if (!b_term) {
        const Tile A2T = ttrans(A2, lds);
        const Tile Y = tnz<NK, PR>(YT, C1);      // X^{-1} C~1
        const Tile Vt = tnz<NK, PR>(Y, A2T);     // (A~2 X^{-1} C~1)'
        gstore_c(o, tnz<NK, PR>(A2T, Z), n1);          // A~2 X^{-1} A~1
        gstore_c(o + TILE, tsym(tna<NK, PR>(Vt, A2T, C2), lds), n1);
    }
    if (!ok) report(status, d.orig, ERR_SINGULAR, s * d.L);
}

// ---------------------------------------------------------------------------
// Phase 3: Bellman steps inside each segment from the right neighbour's value
// function S~' (the carry), writing S_k, s_k, Gamma_k, gamma_k.
//   S~'B~, S~'A~;  Q_uu = R + B~'S~'B~;  Q_ux~ = M~' + B~'S~'A~;
//   Gamma~ = -Q_uu^{-1} Q_ux~ = [Gamma, gamma];
//   S~ = sym(Q~ + A~'S~'A~ + Q_ux~' Gamma~).
// ---------------------------------------------------------------------------
//
// With Yroll != nullptr the sweep also folds the segment's closed-loop maps
// for the rollout, Phi_s = F~_{k1-1} ... F~_{k0} with F~_k = A~_k + B~_k Gamma~_k
// (kept as Phi' across the sweep), and writes the rollout scan's entries:
// Phi_s at s + 1 (s < nseg - 1) and the constant map of x0 at 0.
// The sweep over stages k1-1 .. k0 from the carry St.  The stage data comes
// through LDS as in the fused fold (loaded two stages ahead).  MR: cross
// terms present; ROLL: fold the rollout maps.
template <int NK, int PR, bool MR, bool ROLL>
LQK_DEV void riccati_sweep(const ProbPtrs &P, const InstDesc &d, const ValPtrs &V, int k0, int k1, Tile &St,
                           Tile &PhiT, int &code, int &fk, double *lds, double *stg)
{
    constexpr int SZ = stage_buf_size<NK>();
    const int n = d.n, m = d.m;
    const StageLayout L = stage_layout(n, m);
    const ValueStage<NK, MR> VS = value_stage<NK, MR>(P, d, L);
    stage_consts(stg);
    stage_consts(stg + SZ);
    sweep_ahead2<typename ValueStage<NK, MR>::Regs>(stg, SZ, VS.a, L.trash, k1 - 1, k1 - k0, -1,
                                                     [&](int k, const double *cur) {
        const Tile Ah = gather(cur, gmap_Ah(L, n)), Bh = gather(cur, gmap_Bh(L, n, m));
        const Tile Qh = gather(cur, gmap_Qh(L, n)), Rk = gather(cur, gmap_R(L, m));
        const Tile MhT = MR ? gather(cur, gmap_MhT(L, n, m)) : tzero();
        const Tile BhT = ROLL ? gather(cur, gmap_BhT(L, n, m)) : tzero();
        const Tile SB = tnz<NK, PR>(St, Bh);          // S~'B~
        const Tile SA = tnz<NK, PR>(St, Ah);          // S~'A~
        const Tile Quu = tna<NK, PR>(Bh, SB, Rk);     // R + B~'S~'B~
        const Tile Qux = tna<NK, PR>(Bh, SA, MhT);    // M~' + B~'S~'A~
        Tile Sn = tna<NK, PR>(Ah, SA, Qh);            // Q~ + A~'S~'A~
        Tile QiT;
        const bool pd = spd_inverse_t(Quu, m, QiT);
        Tile Gh = tnz<1, PR>(QiT, Qux);
        Gh.v = -Gh.v;                                 // -Q_uu^{-1} Q_ux~
        Sn = tna<1, PR>(Qux, Gh, Sn);                 // + Q_ux~' Gamma~
        if (ROLL) PhiT = tnz<NK, PR>(tna<1, PR>(BhT, Gh, Ah), PhiT);   // (Phi F~_k)' = F~_k' Phi'
        St = tsym(Sn, lds);
        // Every entry of the stage's data (A, B, c, Q, R, M, q, r) reaches
        // S~_k, so a NaN or Inf among them is reported at this stage, ahead of
        // the positive-definiteness test that a non-finite Q_uu also fails.
        note(tfinite(St), ERR_NONFINITE, k, code, fk);
        note(pd, ERR_NOT_PD, k, code, fk);
        gstore_rm(V.S + d.oS + (int64_t)k * n * n, St, n, n, n);
        store_vec(V.s + d.os + (int64_t)k * n, St, n, n);
        gstore_rm(V.G + d.oG + (int64_t)k * m * n, Gh, m, n, n);
        store_vec(V.g + d.og + (int64_t)k * m, Gh, m, n);
    });
}

// With ckpt != nullptr the last segment of each group of `stride` segments
// also stores its carry (the value function at the group's right end; the
// terminal element for the instance's last group) in checkpoint slot
// ckpt_slot(...) + s / stride, from which k_value_recompute restarts the
// sweep of the whole group.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_riccati(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      const double *__restrict__ Xfin, ValPtrs V,
                                                      double *__restrict__ Yroll, double *__restrict__ ckpt,
                                                      int stride, int32_t *status)
{
    __shared__ double lds[SLOT];
    __shared__ double stg[2 * stage_buf_size<NK>()];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n;
    const bool has_mr = (P.M != nullptr) || (P.r != nullptr);
    // the carry: the scanned suffix from segment s + 1, or for the last
    // segment the terminal element
    Tile St = (s == d.nseg - 1) ? load_terminal_J(P, d, lds)
                                : gload_c(Xfin + (int64_t)(d.xbase + s + 1) * 3 * TILE + 2 * TILE, n + 1);
    if (ckpt && ((s + 1) % stride == 0 || s == d.nseg - 1))
        gstore_c(ckpt + (int64_t)(ckpt_slot(d, i, stride) + s / stride) * TILE, St, n + 1);
    int code = 0, fk = 0;
    if (s == d.nseg - 1) {
        gstore_rm(V.S + d.oS + (int64_t)d.T * n * n, St, n, n, n);
        store_vec(V.s + d.os + (int64_t)d.T * n, St, n, n);
        note(tfinite(St), ERR_NONFINITE, d.T, code, fk);   // Q_T, q_T
    }
    const bool roll = (Yroll != nullptr);
    Tile PhiT = tident(n + 1);
    if (has_mr) {
        if (roll)
            riccati_sweep<NK, PR, true, true>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
        else
            riccati_sweep<NK, PR, true, false>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
    } else {
        if (roll)
            riccati_sweep<NK, PR, false, true>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
        else
            riccati_sweep<NK, PR, false, false>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
    }
    if (roll) {
        if (s == 0) gstore_c(Yroll + (int64_t)d.xbase * TILE, load_vec(P.x0 + d.on, n, n, n), d.n + 1);
        if (s < d.nseg - 1) gstore_c(Yroll + (int64_t)(d.xbase + s + 1) * TILE, ttrans(PhiT, lds), d.n + 1);
    }
    if (code) report(status, d.orig, code, fk);
}

// ---------------------------------------------------------------------------
// Recompute of the value functions and the control law from a checkpoint
// (level checkpointing of the differentiated solve): one wave per group of
// `stride` consecutive segments, restarting from the group's stored carry and
// running the Bellman steps of eq:value-fun-param (in the Riccati form of
// k_value_riccati) over all its stages right to left.  The results equal the
// forward's up to the association order inside the group (bit for bit when
// stride = 1: the same carry and the same sweep).  Block g serves slot g;
// slots between one instance's last group and the next instance's first are
// idle.
// ---------------------------------------------------------------------------
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_value_recompute(ProbPtrs P, const InstDesc *__restrict__ inst,
                                                        const int32_t *__restrict__ seg_start, int batch, int stride,
                                                        const double *__restrict__ ckpt, ValPtrs V, int32_t *status)
{
    __shared__ double lds[SLOT];
    __shared__ double stg[2 * stage_buf_size<NK>()];
    const int g = blockIdx.x;
    // instance owning slot g: the largest i with seg_start[i] / stride + i <= g
    int lo = 0, hi = batch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_start[mid] / stride + mid <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int i = lo;
    const InstDesc d = inst[i];
    const int j = g - ckpt_slot(d, i, stride);
    const int groups = (d.nseg + stride - 1) / stride;
    if (j >= groups) return;
    const int n = d.n;
    const int k0 = j * stride * d.L, k1 = min(k0 + stride * d.L, d.T);
    Tile St = gload_c(ckpt + (int64_t)g * TILE, n + 1);
    int code = 0, fk = 0;
    if (j == groups - 1) {
        gstore_rm(V.S + d.oS + (int64_t)d.T * n * n, St, n, n, n);
        store_vec(V.s + d.os + (int64_t)d.T * n, St, n, n);
        note(tfinite(St), ERR_NONFINITE, d.T, code, fk);
    }
    Tile PhiT = tzero();
    if ((P.M != nullptr) || (P.r != nullptr))
        riccati_sweep<NK, PR, true, false>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
    else
        riccati_sweep<NK, PR, false, false>(P, d, V, k0, k1, St, PhiT, code, fk, lds, stg);
    if (code) report(status, d.orig, code, fk);
}

// ---------------------------------------------------------------------------
// Conditional-value states at the segment starts (eq:value-fun-prefix-sum).
// With the prefix element (A~, C~) of stages 0 .. k0-1 and the value function
// S~ = [[S, s], [s', 0]] of stage k0, the optimal state minimises
// V(x0, x) + V_k0(x), which in the dual form eq:value-fun-elements gives
//   x~ = (I + C~ S~)^{-1} A~ x~0
// (the last column of a tile whose other columns are zero, the form the
// rollout's scan entries have).  (I + C~ S~)' = I + S~ C~ has last column
// e_n, so the homogeneous Gauss-Jordan applies.
// ---------------------------------------------------------------------------
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_cv_start(ProbPtrs P, ValPtrs V, const InstDesc *__restrict__ inst,
                                                 const int32_t *__restrict__ seg_start, int batch,
                                                 const double *__restrict__ Xfin, double *__restrict__ Y,
                                                 int32_t *status)
{
    __shared__ double lds[SLOT];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int n1 = d.n + 1;
    const double *e = Xfin + (int64_t)(d.xbase + s) * 3 * TILE;
    const Tile Ah = gload_c(e, n1), Ch = gload_c(e + TILE, n1);
    const Tile Sh = load_Sh(V.S, V.s, d, s * d.L);
    const Tile X0 = load_vec(P.x0 + d.on, d.n, d.n, d.n);
    Tile YT = tna<NK, PR>(Sh, Ch, tident(n1));          // (I + C~ S~)'
    const bool ok = gj_inverse<NK>(YT, n1, true);      // (I + C~ S~)^{-T}
    const Tile AX = tnz<NK, PR>(ttrans(Ah, lds), X0);   // A~ x~0
    gstore_c(Y + (int64_t)(d.xbase + s) * TILE, tnz<NK, PR>(YT, AX), d.n + 1);
    if (!ok) report(status, d.orig, ERR_SINGULAR, s * d.L);
}

// ---------------------------------------------------------------------------
// Host launchers (the contraction slice count NK = ceil((n_max + 1) / 4) is a
// template parameter so that every product is fully unrolled).
// ---------------------------------------------------------------------------

void launch_value_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *elems, double *X, int prefix,
                       int32_t *status)
{
#define CALL(K, R) \
    hipLaunchKernelGGL((k_value_fold<K, R>), dim3(grid), dim3(64), 0, st, P, inst, seg_start, batch, elems, X, prefix, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_value_ks(int nk, int pr, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                     int batch, int dd, int prefix, const double *Xin, double *Xout, int32_t *status)
{
#define CALL(K, R) \
    hipLaunchKernelGGL((k_value_ks<K, R>), dim3(grid), dim3(64), 0, st, inst, x_start, batch, dd, prefix, Xin, Xout, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_cv_start(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                     const int32_t *seg_start, int batch, const double *Xfin, double *Y, int32_t *status)
{
#define CALL(K, R) \
    hipLaunchKernelGGL((k_cv_start<K, R>), dim3(grid), dim3(64), 0, st, P, V, inst, seg_start, batch, Xfin, Y, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_value_riccati(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                          const int32_t *seg_start, int batch, const double *Xfin, ValPtrs V, double *Yroll,
                          double *ckpt, int stride, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_value_riccati<K, R>), dim3(grid), dim3(64), 0, st, P, inst, seg_start, batch, Xfin, V, Yroll, ckpt, stride, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_value_recompute(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                            const int32_t *seg_start, int batch, int stride, const double *ckpt, ValPtrs V,
                            int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_value_recompute<K, R>), dim3(grid), dim3(64), 0, st, P, inst, seg_start, batch, stride, ckpt, V, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

// Diagnostic: D = op(X) op(Y) (+ Z) for row-major 16 x 16 inputs, through the
// same register product and LDS transpose as the solver.
template <int PR>
__global__ __launch_bounds__(64) void k_selftest_mm(const double *X, const double *Y, const double *Z,
                                                    double *D, int tx, int ty)
{
    __shared__ double lds[SLOT];
    const Tile x = gload_rm(X, 16, 16, 16), y = gload_rm(Y, 16, 16, 16);
    const Tile zt = Z ? gload_rm(Z, 16, 16, 16) : tzero();
    const Tile xf = tx ? x : ttrans(x, lds);   // R(op(X)')
    const Tile yf = ty ? ttrans(y, lds) : y;   // R(op(Y))
    gstore_rm(D, tna<4, PR>(xf, yf, zt), 16, 16, 16);
}

// Diagnostic: the register Gauss-Jordan inverse of the leading n1 x n1 block
// of a row-major 16 x 16 input; *ok = success.
__global__ __launch_bounds__(64) void k_selftest_inv(const double *X, double *Xi, int n1, int homog, int32_t *ok)
{
    Tile x = gload_rm(X, n1, n1, 16);
    const bool good = gj_inverse<4>(x, n1, homog != 0);
    gstore_rm(Xi, x, 16, 16, 16);
    if (lane() == 0) *ok = good ? 1 : 0;
}

void launch_selftest_inv(hipStream_t st, const double *X, double *Xi, int n1, int homog, int32_t *ok)
{
    hipLaunchKernelGGL(k_selftest_inv, dim3(1), dim3(64), 0, st, X, Xi, n1, homog, ok);
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
