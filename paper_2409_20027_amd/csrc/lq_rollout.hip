// lq_rollout.hip -- the state propagation pass (Sec. III-D, Alg. 3) and the
// generic affine-map scan level shared with the adjoint.
//
// An affine map x -> F x + e is the homogeneous matrix [[F, e], [0, 1]], so
// the operator eq:state-prop-comb-rule is a matrix product and a vector is
// the constant map [[0, x], [0, 1]] (its last column).  The closed-loop map
// of stage k is F~_k = A~_k + B~_k Gamma~_k with Gamma~ = [Gamma, gamma].
// The first element of the prefix scan is the constant map of x0, which is
// eq:state-prop-init-elem-init.
//
//   k_roll_fold   : per segment, Phi_s = F~_{k1-1} ... F~_{k0}; the block of
//                   segment 0 also writes the x0 element.
//   k_affine_ks   : one Kogge-Stone level, prefix (Y_s <- Y_s Y_{s-dd}) or
//                   suffix (Y_s <- Y_s Y_{s+dd}); one tile per entry.
//   k_roll_apply  : from the state at the segment start, x_{k+1} = F~ x~,
//                   u_k = Gamma~ x~, lambda_k = S~_k x~ (top rows).
#include "lq_kernels.hpp"

namespace lqk {

// R(F~') of the closed-loop map F~ = A~ + B~ Gamma~:  A~' + Gamma~' B~'.
template <int PR>
LQK_DEV Tile closed_loop_t(const Tile &AhT, const Tile &Gh, const Tile &BhT)
{
    return tna<1, PR>(Gh, BhT, AhT);
}

template <int NK, int PR>
__global__ __launch_bounds__(64) void k_roll_fold(ProbPtrs P, ValPtrs V, const InstDesc *__restrict__ inst,
                                                  const int32_t *__restrict__ seg_start, int batch,
                                                  double *__restrict__ Y)
{
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    if (s == 0) gstore(Y + (int64_t)d.xbase * TILE, load_vec(P.x0 + d.on, d.n, d.n, d.n));
    // The map of the last segment is never read: segment s starts from the
    // scanned entry s.
    if (s == d.nseg - 1) return;
    Tile Phi = tident(d.n + 1);
    for (int k = k0; k < k1; ++k)
        Phi = tnz<NK, PR>(closed_loop_t<PR>(load_AhT(P, d, k), load_Gh(V.G, V.g, d, k), load_BhT(P, d, k)), Phi);   // F~ Phi
    gstore(Y + (int64_t)(d.xbase + s + 1) * TILE, Phi);
}

// One radix-4 Kogge-Stone level over entries [xbase, xbase + nseg] of each
// instance, distance dd:
//   prefix (suffix = 0): Y_s <- Y_s Y_{s-dd} Y_{s-2dd} Y_{s-3dd}
//   suffix (suffix = 1): Y_s <- Y_s Y_{s+dd} Y_{s+2dd} Y_{s+3dd}
// with the terms that fall outside [0, nseg] left out; after the level with
// distance dd an entry covers 4 dd entries, so dd = 1, 4, 16, ... reaches
// every prefix (suffix) in ceil(log4(nseg + 1)) levels.  The product is
// carried transposed (P' <- Y_j' P' is a register product), so a level takes
// two LDS transposes whatever the number of terms.  The entry that no segment
// reads (the last of a prefix scan, the first of a suffix scan) is skipped.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_affine_ks(const InstDesc *__restrict__ inst,
                                                  const int32_t *__restrict__ x_start, int batch, int dd,
                                                  int suffix, const double *__restrict__ Yin,
                                                  double *__restrict__ Yout)
{
    __shared__ double lds[SLOT];
    const int gx = blockIdx.x;
    const int i = find_inst(x_start, batch, gx);
    const InstDesc d = inst[i];
    const int s = gx - d.xbase;
    if (suffix ? (s == 0) : (s == d.nseg)) return;   // entries that are never read
    const Tile a = gload(Yin + (int64_t)gx * TILE);
    const int avail = suffix ? (d.nseg - s) / dd : s / dd;   // terms that exist on that side
    const int terms = min(3, avail);
    if (terms == 0) {
        gstore(Yout + (int64_t)gx * TILE, a);
        return;
    }
    const int64_t step = suffix ? dd : -dd;
    // issue every term's load before the first product
    const Tile b1 = gload(Yin + (gx + step) * TILE);
    const Tile b2 = terms >= 2 ? gload(Yin + (gx + 2 * step) * TILE) : tzero();
    const Tile b3 = terms >= 3 ? gload(Yin + (gx + 3 * step) * TILE) : tzero();
    Tile PT = tnz<NK, PR>(b1, ttrans(a, lds));     // (a b1)'
    if (terms >= 2) PT = tnz<NK, PR>(b2, PT);      // (a b1 b2)'
    if (terms >= 3) PT = tnz<NK, PR>(b3, PT);      // (a b1 b2 b3)'
    gstore(Yout + (int64_t)gx * TILE, ttrans(PT, lds));
}

// From the state at the segment start: u_k = Gamma~ x~, lambda_k = S~_k x~,
// x~_{k+1} = A~ x~ + B~ u_k (x~ = [x; 1] in the last column of X).
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_roll_apply(ProbPtrs P, ValPtrs V, const InstDesc *__restrict__ inst,
                                                   const int32_t *__restrict__ seg_start, int batch,
                                                   const double *__restrict__ Yfin, double *__restrict__ x,
                                                   double *__restrict__ u, double *__restrict__ lam)
{
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    Tile X = gload(Yfin + (int64_t)(d.xbase + s) * TILE);   // [[0, x_k0], [0, 1]]
    for (int k = k0; k < k1; ++k) {
        const Tile GhT = load_GhT(V.G, V.g, d, k), AhT = load_AhT(P, d, k), BhT = load_BhT(P, d, k);
        const Tile Sh = lam ? load_Sh(V.S, V.s, d, k) : tzero();
        store_vec(x + d.os + (int64_t)k * n, X, n, n);
        const Tile Uk = tnz<NK, PR>(GhT, X);                       // Gamma~ x~
        store_vec(u + d.og + (int64_t)k * m, Uk, m, n);
        if (lam) store_vec(lam + d.os + (int64_t)k * n, tnz<NK, PR>(Sh, X), n, n);
        X = tna<1, PR>(BhT, Uk, tnz<NK, PR>(AhT, X));              // A~ x~ + B~ u
    }
    if (k1 == d.T) {
        store_vec(x + d.os + (int64_t)d.T * n, X, n, n);
        if (lam) store_vec(lam + d.os + (int64_t)d.T * n, tnz<NK, PR>(load_Sh(V.S, V.s, d, d.T), X), n, n);
    }
}

}  // namespace lqk

namespace lqk {

void launch_roll_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                      const int32_t *seg_start, int batch, double *Y)
{
#define CALL(K, R) hipLaunchKernelGGL((k_roll_fold<K, R>), dim3(grid), dim3(64), 0, st, P, V, inst, seg_start, batch, Y)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_affine_ks(int nk, int pr, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start, int batch,
                      int dd, int suffix, const double *Yin, double *Yout)
{
#define CALL(K, R) hipLaunchKernelGGL((k_affine_ks<K, R>), dim3(grid), dim3(64), 0, st, inst, x_start, batch, dd, suffix, Yin, Yout)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}

void launch_roll_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *Yfin, double *x, double *u, double *lam)
{
#define CALL(K, R) hipLaunchKernelGGL((k_roll_apply<K, R>), dim3(grid), dim3(64), 0, st, P, V, inst, seg_start, batch, Yfin, x, u, lam)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
}  // namespace lqk
