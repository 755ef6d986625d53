// lq_adjoint.hip -- reverse-mode derivative of the LQ solution.
//
// Implicit differentiation of the LQ's KKT system: for a loss L(x, u) with
// gx = dL/dx, gu = dL/du, the adjoint is the same LQ with linear terms
// (gx, gu), no offset and x0 = 0.  It shares the forward value matrices S_k and
// gains Gamma_k, so only two affine scans are needed, both in the homogeneous
// form of lq_rollout.hip:
//
//   backward (suffix): s~_k = h_k + F_k' s~_{k+1}, s~_T = gx_T,
//       h_k = gx_k + Gamma_k' gu_k, F_k = A_k + B_k Gamma_k,
//       map Y~_k = [[F_k', h_k], [0, 1]];  inside each segment also
//       gamma~_k = -(R_k + B_k'S_{k+1}B_k)^{-1} (gu_k + B_k' s~_{k+1});
//   forward (prefix): dx_{k+1} = F_k dx_k + B_k gamma~_k, dx_0 = 0,
//       du_k = Gamma_k dx_k + gamma~_k, dlam_k = S_k dx_k + s~_k,
//   and per stage the outer-product gradients of include/lqscan.h.
#include "lq_kernels.hpp"

namespace lqk {

constexpr int ADJ_ERR_NOT_PD = -2;

// Segment fold of the backward maps, Psi_s = Y~_{k0} ... Y~_{k1-1}, kept as
// Psi' (Psi' <- Y~_k' Psi' is a register product); the block of the last
// segment also writes the terminal vector map [[0, gx_T], [0, 1]].
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_back_fold(ProbPtrs P, AdjPtrs J, const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      double *__restrict__ Y)
{
    __shared__ double lds[SLOT];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    if (s == d.nseg - 1)
        gstore_c(Y + (int64_t)(d.xbase + d.nseg) * TILE, load_vec(J.gx + d.os + (int64_t)d.T * n, n, n, n), d.n + 1);
    if (s == 0) return;   // never read: segment s starts from entry s + 1
    // stage data through LDS, loaded two stages ahead (sweep_ahead2)
    constexpr int NM = 4 * NK - 1, SA = (NM * NM + 63) / 64, SB = (NM * MMAX + 63) / 64;
    constexpr int SZ = 2 + NM * NM + 2 * NM * MMAX + MMAX + NM + 64;
    __shared__ double stg[2 * SZ];
    const int oA = 2, oG = oA + n * n, oB = oG + m * n, ou = oB + n * m, ox = ou + m, trash = ox + n;
    const StageArr arr[5] = {stage_arr(P.A + d.oA, n * n, n * n, oA), stage_arr(J.G + d.oG, m * n, m * n, oG),
                             stage_arr(P.B + d.oB, n * m, n * m, oB), stage_arr(J.gu + d.og, m, m, ou),
                             stage_arr(J.gx + d.os, n, n, ox)};
    // A_noc~' = [[A', 0], [0, 1]], Gamma_0~ = [Gamma, 0], B~' = [B', 0], gu and gx in column n
    const GMap gA = gmap_of([&](int r, int c) { return (r < n && c < n) ? oA + c * n + r : (r == n && c == n) ? 1 : 0; });
    const GMap gG = gmap_of([&](int r, int c) { return (r < m && c < n) ? oG + r * n + c : 0; });
    const GMap gB = gmap_of([&](int r, int c) { return (r < m && c < n) ? oB + c * m + r : 0; });
    const GMap gU = gmap_of([&](int r, int c) { return (c == n && r < m) ? ou + r : 0; });
    const GMap gX = gmap_of([&](int r, int c) { return (c == n && r < n) ? ox + r : 0; });
    stage_consts(stg);
    stage_consts(stg + SZ);
    Tile PsiT = tident(n + 1);
    // a stage's chain (five products) is shorter than a load's latency: the
    // loads run two stages ahead
    sweep_ahead2<StageRegs<SA, SB, SB, 1, 1>>(stg, SZ, arr, trash, k0, k1 - k0, 1, [&](int k, const double *cur) {
        // R(Y~_k) = A_noc~' + Gamma_0~'(B~' + [gu in column n]) + [gx in column n]
        const Tile AnT = gather(cur, gA), G0 = gather(cur, gG), BhT = gather(cur, gB);
        const Tile GU = gather(cur, gU), GX = gather(cur, gX);
        const Tile Yk = tna<1, PR>(G0, tadd(BhT, GU), tadd(AnT, GX));
        PsiT = tnz<NK, PR>(Yk, PsiT);   // (Psi Y~_k)' = Y~_k' Psi'
    });
    gstore_c(Y + (int64_t)(d.xbase + s) * TILE, ttrans(PsiT, lds), d.n + 1);
}

// Inside each segment, from s~ at its right end: s~_k and gamma~_k.
//   s~_k = F_k' s~_{k+1} + gx_k + Gamma_k' gu_k,
//   gamma~_k = -(R_k + B~'S~_{k+1}B~)^{-1} (gu_k + B~' s~_{k+1}).
// gamma~_k completes the derivative's closed-loop map of stage k,
// F'_k = [[A + B Gamma, B gamma~], [0, 1]], so the same sweep folds the
// forward scan's segment maps Phi_s = F'_{k1-1} ... F'_{k0} (kept as Phi') and
// writes the forward scan's entries into Yfwd: Phi_s at s + 1 (s < nseg - 1)
// and the zero map of dx_0 at 0.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_back_apply(ProbPtrs P, AdjPtrs J, const InstDesc *__restrict__ inst,
                                                       const int32_t *__restrict__ seg_start, int batch,
                                                       const double *__restrict__ Yfin, double *__restrict__ Yfwd,
                                                       int32_t *status)
{
    __shared__ double lds[SLOT];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    Tile SV = gload_c(Yfin + (int64_t)(d.xbase + s + 1) * TILE, d.n + 1);   // [[0, s~_{k1}], [0, 1]]
    if (s == d.nseg - 1) store_vec(J.st + d.os + (int64_t)d.T * n, SV, n, n);
    int code = 0, fk = 0;
    // stage data through LDS, loaded two stages ahead (sweep_ahead2)
    constexpr int NM = 4 * NK - 1, SA = (NM * NM + 63) / 64, SB = (NM * MMAX + 63) / 64;
    constexpr int SZ = 2 + 2 * NM * NM + 2 * NM * MMAX + MMAX * MMAX + 2 * NM + MMAX + 64;
    __shared__ double stg[2 * SZ];
    const int oA = 2, oB = oA + n * n, oR = oB + n * m, oG = oR + m * m, oS = oG + m * n, os = oS + n * n,
              ou = os + n, ox = ou + m, trash = ox + n;
    // S~ and s~ of stage k + 1 with stage k's data
    const StageArr arr[8] = {stage_arr(P.A + d.oA, n * n, n * n, oA),   stage_arr(P.B + d.oB, n * m, n * m, oB),
                             stage_arr(P.R + d.oR, m * m, m * m, oR),   stage_arr(J.G + d.oG, m * n, m * n, oG),
                             stage_arr(J.S + d.oS + n * n, n * n, n * n, oS), stage_arr(J.s + d.os + n, n, n, os),
                             stage_arr(J.gu + d.og, m, m, ou),          stage_arr(J.gx + d.os, n, n, ox)};
    // B~, B~', S~ = [[S, s], [s', 0]], R, A_noc~ = [[A, 0], [0, 1]], Gamma_0~ = [Gamma, 0], gu and gx in column n
    const GMap gBh = gmap_of([&](int r, int c) { return (r < n && c < m) ? oB + r * m + c : 0; });
    const GMap gBt = gmap_of([&](int r, int c) { return (r < m && c < n) ? oB + c * m + r : 0; });
    const GMap gS = gmap_of([&](int r, int c) {
        return (r < n && c < n) ? oS + r * n + c : (c == n && r < n) ? os + r : (r == n && c < n) ? os + c : 0;
    });
    const GMap gR = gmap_of([&](int r, int c) { return (r < m && c < m) ? oR + r * m + c : 0; });
    const GMap gA = gmap_of([&](int r, int c) { return (r < n && c < n) ? oA + r * n + c : (r == n && c == n) ? 1 : 0; });
    const GMap gG = gmap_of([&](int r, int c) { return (r < m && c < n) ? oG + r * n + c : 0; });
    const GMap gU = gmap_of([&](int r, int c) { return (c == n && r < m) ? ou + r : 0; });
    const GMap gX = gmap_of([&](int r, int c) { return (c == n && r < n) ? ox + r : 0; });
    stage_consts(stg);
    stage_consts(stg + SZ);
    Tile PhiT = tident(n + 1);
    sweep_ahead2<StageRegs<SA, SB, 1, SB, SA, 1, 1, 1>>(stg, SZ, arr, trash, k1 - 1, k1 - k0, -1,
                                                        [&](int k, const double *cur) {
        const Tile Bh = gather(cur, gBh), BhT = gather(cur, gBt), Sh = gather(cur, gS);
        const Tile Rk = gather(cur, gR), An = gather(cur, gA), G0 = gather(cur, gG);
        const Tile GU = gather(cur, gU), GX = gather(cur, gX);
        const Tile SB = tnz<NK, PR>(Sh, Bh);                 // S~_{k+1} B~
        const Tile Quu = tna<NK, PR>(Bh, SB, Rk);            // R + B~'S~B~
        Tile QiT;
        const bool okq = spd_inverse_t(Quu, m, QiT);
        const bool first = !okq && (code == 0);
        code = first ? ADJ_ERR_NOT_PD : code;
        fk = first ? k : fk;
        const Tile BS = tna<NK, PR>(Bh, SV, GU);             // gu + B~'s~_{k+1}
        Tile Gt = tnz<1, PR>(QiT, BS);
        Gt.v = -Gt.v;
        store_vec(J.gt + d.og + (int64_t)k * m, Gt, m, n);
        // F~ = A_noc~ + B~ Gamma_0~;  s~_k = F~'s~_{k+1} + gx + Gamma_0~'gu
        const Tile F = tna<1, PR>(BhT, G0, An);
        PhiT = tnz<NK, PR>(tna<1, PR>(BhT, Gt, F), PhiT);   // (Phi F'_k)' = F'_k' Phi'
        SV = tna<NK, PR>(F, SV, tna<1, PR>(G0, GU, GX));
        store_vec(J.st + d.os + (int64_t)k * n, SV, n, n);
    });
    if (s == 0) gstore_c(Yfwd + (int64_t)d.xbase * TILE, load_vec(nullptr, n, n, n), d.n + 1);   // dx_0 = 0
    if (s < d.nseg - 1) gstore_c(Yfwd + (int64_t)(d.xbase + s + 1) * TILE, ttrans(PhiT, lds), d.n + 1);
    if (code) report(status, d.orig, code, fk);
}

template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_fwd_apply(ProbPtrs P, AdjPtrs J, GradPtrs Gr,
                                                      const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      const double *__restrict__ Yfin)
{
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    Tile DX = gload_c(Yfin + (int64_t)(d.xbase + s) * TILE, d.n + 1);   // [[0, dx_k0], [0, 1]]
    if (s == 0 && Gr.x0) store_vec(Gr.x0 + d.on, tnz<NK, PR>(load_Sh(J.S, J.st, d, 0), DX), n, n);
    // stage data through LDS, loaded two stages ahead (sweep_ahead2)
    constexpr int NM = 4 * NK - 1, SA = (NM * NM + 63) / 64, SB = (NM * MMAX + 63) / 64;
    constexpr int SZ = 2 + 2 * NM * NM + 2 * NM * MMAX + 4 * NM + 2 * MMAX + 64;
    __shared__ double stg[2 * SZ];
    const int oG = 2, og = oG + m * n, oB = og + m, oA = oB + n * m, oS = oA + n * n, os = oS + n * n, ox = os + n,
              ou = ox + n, ol = ou + m, trash = ol + n;
    // S~, s~ and lambda of stage k + 1 with stage k's data
    const StageArr arr[9] = {stage_arr(J.G + d.oG, m * n, m * n, oG),   stage_arr(J.gt + d.og, m, m, og),
                             stage_arr(P.B + d.oB, n * m, n * m, oB),   stage_arr(P.A + d.oA, n * n, n * n, oA),
                             stage_arr(J.S + d.oS + n * n, n * n, n * n, oS), stage_arr(J.st + d.os + n, n, n, os),
                             stage_arr(J.x + d.os, n, n, ox),           stage_arr(J.u + d.og, m, m, ou),
                             stage_arr(J.lam + d.os + n, n, n, ol)};
    // Gamma~' = [[Gamma'], [gamma~']], B~', A_noc~', S~, x, u, lambda in column n
    const GMap gG = gmap_of([&](int r, int c) { return (c < m && r < n) ? oG + c * n + r : (c < m && r == n) ? og + c : 0; });
    const GMap gB = gmap_of([&](int r, int c) { return (r < m && c < n) ? oB + c * m + r : 0; });
    const GMap gA = gmap_of([&](int r, int c) { return (r < n && c < n) ? oA + c * n + r : (r == n && c == n) ? 1 : 0; });
    const GMap gS = gmap_of([&](int r, int c) {
        return (r < n && c < n) ? oS + r * n + c : (c == n && r < n) ? os + r : (r == n && c < n) ? os + c : 0;
    });
    // x, u, lambda at each lane's rows, and x, u at its column (the outer
    // products' operands, read straight from the buffer)
    const GMap gXr = gmap_of([&](int r, int c) { return r < n ? ox + r : 0; });
    const GMap gUr = gmap_of([&](int r, int c) { return r < m ? ou + r : 0; });
    const GMap gLr = gmap_of([&](int r, int c) { return r < n ? ol + r : 0; });
    const int iXc = tcol() < n ? ox + tcol() : 0, iUc = tcol() < m ? ou + tcol() : 0;
    stage_consts(stg);
    stage_consts(stg + SZ);
    sweep_ahead2<StageRegs<SB, 1, SB, SA, SA, 1, 1, 1, 1>>(stg, SZ, arr, trash, k0, k1 - k0, 1,
                                                           [&](int k, const double *cur) {
        const Tile GhT = gather(cur, gG), BhT = gather(cur, gB), AnT = gather(cur, gA);
        const Tile S1 = gather(cur, gS);
        const d4 x_r = gather(cur, gXr).v, u_r = gather(cur, gUr).v, l1_r = gather(cur, gLr).v;
        const double x_c = cur[iXc], u_c = cur[iUc];
        const Tile DU = tnz<NK, PR>(GhT, DX);                          // Gamma dx + gamma~
        const Tile DXn = tna<1, PR>(BhT, DU, tnz<NK, PR>(AnT, DX));    // A dx + B du
        const Tile DL1 = tnz<NK, PR>(S1, DXn);                         // S dx' + s~'
        const d4 dx_r = vrows(DX, n), du_r = vrows(DU, n), dl1_r = vrows(DL1, n);
        const double dx_c = vcol(DX, n), du_c = vcol(DU, n);
        // Every gradient is formed and stored without a branch (an absent
        // one goes to an empty range), so that the waits for the loads two
        // stages ahead count the stores exactly.
        const int64_t kn = (int64_t)k * n;
        Tile o;
        o.v = l1_r * dx_c + dl1_r * x_c;
        gstore_rm(Gr.A ? Gr.A + d.oA + kn * n : nullptr, o, n, n, n);
        o.v = l1_r * du_c + dl1_r * u_c;
        gstore_rm(Gr.B ? Gr.B + d.oB + kn * m : nullptr, o, n, m, m);
        store_vec(Gr.c ? Gr.c + d.oc + kn : nullptr, DL1, n, n);
        o.v = 0.5 * (dx_r * x_c + x_r * dx_c);
        gstore_rm(Gr.Q ? Gr.Q + d.oA + kn * n : nullptr, o, n, n, n);
        o.v = 0.5 * (du_r * u_c + u_r * du_c);
        gstore_rm(Gr.R ? Gr.R + d.oR + (int64_t)k * m * m : nullptr, o, m, m, m);
        o.v = dx_r * u_c + x_r * du_c;
        gstore_rm(Gr.M ? Gr.M + d.oB + kn * m : nullptr, o, n, m, m);
        store_vec(Gr.q ? Gr.q + d.oc + kn : nullptr, DX, n, n);
        store_vec(Gr.r ? Gr.r + d.og + (int64_t)k * m : nullptr, DU, m, n);
        DX = DXn;
    });
    if (k1 == d.T) {
        const Tile X = load_vec(J.x + d.os + (int64_t)d.T * n, n, n, -1);
        const d4 dx_r = vrows(DX, n), x_r = vrows(X, n);
        const double dx_c = vcol(DX, n), x_c = vcol(X, n);
        if (Gr.QT) {
            Tile o;
            o.v = 0.5 * (dx_r * x_c + x_r * dx_c);
            gstore_rm(Gr.QT + d.oQT, o, n, n, n);
        }
        if (Gr.qT) store_vec(Gr.qT + d.on, DX, n, n);
    }
}


void launch_adj_back_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, const InstDesc *inst,
                          const int32_t *seg_start, int batch, double *Y)
{
#define CALL(K, R) hipLaunchKernelGGL((k_adj_back_fold<K, R>), dim3(grid), dim3(64), 0, st, P, J, inst, seg_start, batch, Y)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
void launch_adj_back_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, const InstDesc *inst,
                           const int32_t *seg_start, int batch, const double *Yfin, double *Yfwd, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_adj_back_apply<K, R>), dim3(grid), dim3(64), 0, st, P, J, inst, seg_start, batch, Yfin, Yfwd, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
void launch_adj_fwd_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, GradPtrs Gr,
                          const InstDesc *inst, const int32_t *seg_start, int batch, const double *Yfin)
{
#define CALL(K, R) hipLaunchKernelGGL((k_adj_fwd_apply<K, R>), dim3(grid), dim3(64), 0, st, P, J, Gr, inst, seg_start, batch, Yfin)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
}  // namespace lqk
