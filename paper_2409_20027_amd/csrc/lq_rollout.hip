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
//   k_affine_ks   : one Kogge-Stone level of radix 2..32, prefix
//                   (Y_s <- Y_s Y_{s-dd} ...) or suffix (Y_s <- Y_s Y_{s+dd} ...);
//                   one tile per entry.
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
    if (s == 0) gstore_c(Y + (int64_t)d.xbase * TILE, load_vec(P.x0 + d.on, d.n, d.n, d.n), d.n + 1);
    // The map of the last segment is never read: segment s starts from the
    // scanned entry s.
    if (s == d.nseg - 1) return;
    Tile Phi = tident(d.n + 1);
    for (int k = k0; k < k1; ++k)
        Phi = tnz<NK, PR>(closed_loop_t<PR>(load_AhT(P, d, k), load_Gh(V.G, V.g, d, k), load_BhT(P, d, k)), Phi);   // F~ Phi
    gstore_c(Y + (int64_t)(d.xbase + s + 1) * TILE, Phi, d.n + 1);
}

// One radix-RAD Kogge-Stone level over entries [xbase, xbase + nseg] of each
// instance, distance dd:
//   prefix (suffix = 0): Y_s <- Y_s Y_{s-dd} Y_{s-2dd} ... Y_{s-(RAD-1)dd}
//   suffix (suffix = 1): Y_s <- Y_s Y_{s+dd} Y_{s+2dd} ... Y_{s+(RAD-1)dd}
// with the terms that fall outside [0, nseg] left out; after the level with
// distance dd an entry covers RAD dd entries, so dd = 1, RAD, RAD^2, ...
// reaches every prefix (suffix) in ceil(log_RAD(nseg + 1)) levels.  Every
// term's load is issued before the first product (an absent term re-reads the
// entry itself and is not used).  The product is carried transposed
// (P' <- Y_j' P' is a register product), so a level takes two LDS transposes
// whatever the number of terms.  The entry that no segment reads (the last of
// a prefix scan, the first of a suffix scan) is skipped.
template <int NK, int PR, int RAD>
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
    const Tile a = gload_c(Yin + (int64_t)gx * TILE, d.n + 1);
    const int avail = suffix ? (d.nseg - s) / dd : s / dd;   // terms that exist on that side
    const int terms = min(RAD - 1, avail);
    if (terms == 0) {
        gstore_c(Yout + (int64_t)gx * TILE, a, d.n + 1);
        return;
    }
    const int64_t step = suffix ? dd : -dd;
    Tile b[RAD - 1];
#pragma unroll
    for (int j = 0; j < RAD - 1; ++j) b[j] = gload_c(Yin + (gx + (j < terms ? (j + 1) * step : 0)) * TILE, d.n + 1);
    Tile PT = tnz<NK, PR>(b[0], ttrans(a, lds));   // (a b1)'
#pragma unroll
    for (int j = 1; j < RAD - 1; ++j)
        if (j < terms) PT = tnz<NK, PR>(b[j], PT);  // (a b1 ... b_{j+1})'
    gstore_c(Yout + (int64_t)gx * TILE, ttrans(PT, lds), d.n + 1);
}

// Rows [0, len) of column col of a tile to dst[0, len) in LDS; the other
// lanes write to their own slot of trash (64 doubles), so there is no branch.
LQK_DEV void lds_vec(double *dst, double *trash, const Tile &t, int len, int col)
{
    const bool mine = (tcol() == col);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        *((mine && i < len) ? dst + i : trash + lane()) = t.v[r];
    }
}

// From the state at the segment start: u_k = Gamma~ x~, lambda_k = S~_k x~,
// x~_{k+1} = A~ x~ + B~ u_k (x~ = [x; 1] in the last column of X).
//
// Memory order of a stage k: the stores of stage k - 1's x, u and lambda
// (from a two-slot LDS ring), then the loads of stage k + 2, then stage k's
// products, then stage k + 1's data (loaded during stage k - 1) to LDS.  The
// vector memory counter completes in issue order, so a store issued after a
// load could only be waited for together with that load; with the stores
// first, the waits before the next stage's use of their registers leave the
// later loads in flight, and two stages of products cover each load.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_roll_apply(ProbPtrs P, ValPtrs V, const InstDesc *__restrict__ inst,
                                                   const int32_t *__restrict__ seg_start, int batch,
                                                   const double *__restrict__ Yfin, double *__restrict__ x,
                                                   double *__restrict__ u, double *__restrict__ lam)
{
    // stage data through LDS, loaded two stages ahead
    constexpr int NM = 4 * NK - 1;
    constexpr int SZ = 2 + 2 * NM * NM + 2 * NM + 2 * NM * MMAX + MMAX + 64;
    constexpr int RS = 2 * NM + MMAX;   // ring slot: x_k, u_k, lambda_k
    __shared__ double stg[2 * SZ];
    __shared__ double ring[2 * RS + 64];
    double *otr = ring + 2 * RS;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    const int oA = 2, oc = oA + n * n, oB = oc + n, oG = oB + n * m, og = oG + m * n, oS = og + m, os = oS + n * n,
              trash = os + n;
    const StageArr arr[7] = {stage_arr(P.A + d.oA, n * n, n * n, oA),
                             stage_arr(P.c ? P.c + d.oc : nullptr, n, n, oc),
                             stage_arr(P.B + d.oB, n * m, n * m, oB),
                             stage_arr(V.G + d.oG, m * n, m * n, oG),
                             stage_arr(V.g ? V.g + d.og : nullptr, m, m, og),
                             stage_arr(lam ? V.S + d.oS : nullptr, n * n, n * n, oS),
                             stage_arr(lam ? V.s + d.os : nullptr, n, n, os)};
    constexpr int SA = (NM * NM + 63) / 64;
    // Gamma~' = [[Gamma'], [gamma']], A~' = [[A', 0], [c', 1]], B~' = [B', 0], S~ = [[S, s], [s', 0]]
    const GMap gG = gmap_of([&](int r, int c) { return (c < m && r < n) ? oG + c * n + r : (c < m && r == n) ? og + c : 0; });
    const GMap gA = gmap_of([&](int r, int c) {
        return (r < n && c < n) ? oA + c * n + r : (r == n && c < n) ? oc + c : (r == n && c == n) ? 1 : 0;
    });
    const GMap gB = gmap_of([&](int r, int c) { return (r < m && c < n) ? oB + c * m + r : 0; });
    const GMap gS = gmap_of([&](int r, int c) {
        return (r < n && c < n) ? oS + r * n + c : (c == n && r < n) ? os + r : (r == n && c < n) ? os + c : 0;
    });
    stage_consts(stg);
    stage_consts(stg + SZ);
    // The segment's start state is loaded ahead of the first stage's data, so
    // it has arrived when that data is written to LDS and no wait for it is
    // left inside the loop.
    Tile X = gload_c(Yfin + (int64_t)(d.xbase + s) * TILE, d.n + 1);   // [[0, x_k0], [0, 1]]
    // Two register sets: stage k + 2's loads are issued at the top of stage k
    // and written to LDS at the end of stage k + 1.
    StageRegs<SA, 1, 1, 1, 1, SA, 1> fa, fb;
    arr_fetch(arr, k0, fa);
    arr_put(stg, arr, trash, fa);
    arr_fetch(arr, min(k0 + 1, k1 - 1), fb);
    wsync();
    double *const xo = x ? x + d.os : nullptr, *const uo = u ? u + d.og : nullptr,
                 *const lo = lam ? lam + d.os : nullptr;
    // stage kk's outputs from ring slot sl to memory (cnt = 0: nothing)
    auto flush = [&](int kk, const double *sl, int cnt) __attribute__((always_inline)) {
        const int l = lane();
        bstore(brsrc(xo, (kk + 1) * n), (l < n && cnt) ? 8 * (kk * n + l) : BOOB, sl[l < n ? l : 0]);
        bstore(brsrc(uo, (kk + 1) * m), (l < m && cnt) ? 8 * (kk * m + l) : BOOB, sl[l < m ? NM + l : 0]);
        bstore(brsrc(lo, (kk + 1) * n), (l < n && cnt) ? 8 * (kk * n + l) : BOOB, sl[l < n ? NM + MMAX + l : 0]);
    };
    auto stage = [&](int k, const double *cur, double *nxt, StageRegs<SA, 1, 1, 1, 1, SA, 1> &fnew,
                     const StageRegs<SA, 1, 1, 1, 1, SA, 1> &fput) __attribute__((always_inline)) {
        double *sl = ring + (k & 1) * RS;
        flush(k - 1, ring + ((k - 1) & 1) * RS, k > k0);
        arr_fetch(arr, min(k + 2, k1 - 1), fnew);
        const Tile GhT = gather(cur, gG), AhT = gather(cur, gA), BhT = gather(cur, gB);
        lds_vec(sl, otr, X, n, n);
        const Tile Uk = tnz<NK, PR>(GhT, X);                       // Gamma~ x~
        lds_vec(sl + NM, otr, Uk, m, n);
        lds_vec(sl + NM + MMAX, otr, tnz<NK, PR>(gather(cur, gS), X), n, n);   // zero without lam (S~ reads as 0)
        X = tna<1, PR>(BhT, Uk, tnz<NK, PR>(AhT, X));              // A~ x~ + B~ u
        arr_put(nxt, arr, trash, fput);
        wsync();
    };
    // Both halves in the loop body (no path skips the second one back to the
    // top with the first one's loads in flight); an odd last stage after it.
    int k = k0;
    for (; k + 1 < k1; k += 2) {
        stage(k, stg, stg + SZ, fa, fb);
        stage(k + 1, stg + SZ, stg, fb, fa);
    }
    if (k < k1) stage(k, stg, stg + SZ, fa, fb);
    flush(k1 - 1, ring + ((k1 - 1) & 1) * RS, 1);
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

void launch_affine_ks(int nk, int pr, int radix, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                      int batch, int dd, int suffix, const double *Yin, double *Yout)
{
#define CALLR(K, R, RAD) \
    hipLaunchKernelGGL((k_affine_ks<K, R, RAD>), dim3(grid), dim3(64), 0, st, inst, x_start, batch, dd, suffix, Yin, Yout)
#define CALL2(K, R) CALLR(K, R, 2)
#define CALL4(K, R) CALLR(K, R, 4)
#define CALL8(K, R) CALLR(K, R, 8)
#define CALL16(K, R) CALLR(K, R, 16)
#define CALL32(K, R) CALLR(K, R, 32)
    switch (radix) {
    case 2: LQK_DISPATCH(nk, pr, CALL2) break;
    case 8: LQK_DISPATCH(nk, pr, CALL8) break;
    case 16: LQK_DISPATCH(nk, pr, CALL16) break;
    case 32: LQK_DISPATCH(nk, pr, CALL32) break;
    default: LQK_DISPATCH(nk, pr, CALL4) break;
    }
#undef CALL2
#undef CALL4
#undef CALL8
#undef CALL16
#undef CALL32
#undef CALLR
}

void launch_roll_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *Yfin, double *x, double *u, double *lam)
{
#define CALL(K, R) hipLaunchKernelGGL((k_roll_apply<K, R>), dim3(grid), dim3(64), 0, st, P, V, inst, seg_start, batch, Yfin, x, u, lam)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
}  // namespace lqk
