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
        gstore(Y + (int64_t)(d.xbase + d.nseg) * TILE, load_vec(J.gx + d.os + (int64_t)d.T * n, n, n, n));
    if (s == 0) return;   // never read: segment s starts from entry s + 1
    Tile PsiT = tident(n + 1);
    for (int k = k0; k < k1; ++k) {
        // R(Y~_k) = A_noc~' + Gamma_0~'(B~' + [gu in column n]) + [gx in column n]
        const Tile AnT = load_AhT(P, d, k, false);
        const Tile G0 = load_Gh(J.G, nullptr, d, k);
        const Tile BhT = load_BhT(P, d, k);
        const Tile GU = load_vec(J.gu + d.og + (int64_t)k * m, m, n, -1);
        const Tile GX = load_vec(J.gx + d.os + (int64_t)k * n, n, n, -1);
        const Tile Yk = tna<1, PR>(G0, tadd(BhT, GU), tadd(AnT, GX));
        PsiT = tnz<NK, PR>(Yk, PsiT);   // (Psi Y~_k)' = Y~_k' Psi'
    }
    gstore(Y + (int64_t)(d.xbase + s) * TILE, ttrans(PsiT, lds));
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
    Tile SV = gload(Yfin + (int64_t)(d.xbase + s + 1) * TILE);   // [[0, s~_{k1}], [0, 1]]
    if (s == d.nseg - 1) store_vec(J.st + d.os + (int64_t)d.T * n, SV, n, n);
    int code = 0, fk = 0;
    Tile PhiT = tident(n + 1);
    for (int k = k1 - 1; k >= k0; --k) {
        const Tile Bh = load_Bh(P, d, k), BhT = load_BhT(P, d, k), Sh = load_Sh(J.S, J.s, d, k + 1);
        const Tile Rk = load_R(P, d, k), An = load_Ah(P, d, k, false), G0 = load_Gh(J.G, nullptr, d, k);
        const Tile GU = load_vec(J.gu + d.og + (int64_t)k * m, m, n, -1);
        const Tile GX = load_vec(J.gx + d.os + (int64_t)k * n, n, n, -1);
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
    }
    if (s == 0) gstore(Yfwd + (int64_t)d.xbase * TILE, load_vec(nullptr, n, n, n));   // dx_0 = 0
    if (s < d.nseg - 1) gstore(Yfwd + (int64_t)(d.xbase + s + 1) * TILE, ttrans(PhiT, lds));
    if (code) report(status, i, code, fk);
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
    Tile DX = gload(Yfin + (int64_t)(d.xbase + s) * TILE);   // [[0, dx_k0], [0, 1]]
    if (s == 0 && Gr.x0) store_vec(Gr.x0 + d.on, tnz<NK, PR>(load_Sh(J.S, J.st, d, 0), DX), n, n);
    for (int k = k0; k < k1; ++k) {
        const Tile GhT = load_GhT(J.G, J.gt, d, k), BhT = load_BhT(P, d, k), AnT = load_AhT(P, d, k, false);
        const Tile S1 = load_Sh(J.S, J.st, d, k + 1);
        const Tile X = load_vec(J.x + d.os + (int64_t)k * n, n, n, -1), U = load_vec(J.u + d.og + (int64_t)k * m, m, n, -1);
        const Tile L1 = load_vec(J.lam + d.os + (int64_t)(k + 1) * n, n, n, -1);
        const Tile DU = tnz<NK, PR>(GhT, DX);                          // Gamma dx + gamma~
        const Tile DXn = tna<1, PR>(BhT, DU, tnz<NK, PR>(AnT, DX));    // A dx + B du
        const Tile DL1 = tnz<NK, PR>(S1, DXn);                         // S dx' + s~'
        const d4 dx_r = vrows(DX, n), x_r = vrows(X, n), du_r = vrows(DU, n), u_r = vrows(U, n);
        const d4 l1_r = vrows(L1, n), dl1_r = vrows(DL1, n);
        const double dx_c = vcol(DX, n), x_c = vcol(X, n), du_c = vcol(DU, n), u_c = vcol(U, n);
        if (Gr.A) {
            Tile o;
            o.v = l1_r * dx_c + dl1_r * x_c;
            gstore_rm(Gr.A + d.oA + (int64_t)k * n * n, o, n, n, n);
        }
        if (Gr.B) {
            Tile o;
            o.v = l1_r * du_c + dl1_r * u_c;
            gstore_rm(Gr.B + d.oB + (int64_t)k * n * m, o, n, m, m);
        }
        if (Gr.c) store_vec(Gr.c + d.oc + (int64_t)k * n, DL1, n, n);
        if (Gr.Q) {
            Tile o;
            o.v = 0.5 * (dx_r * x_c + x_r * dx_c);
            gstore_rm(Gr.Q + d.oA + (int64_t)k * n * n, o, n, n, n);
        }
        if (Gr.R) {
            Tile o;
            o.v = 0.5 * (du_r * u_c + u_r * du_c);
            gstore_rm(Gr.R + d.oR + (int64_t)k * m * m, o, m, m, m);
        }
        if (Gr.M) {
            Tile o;
            o.v = dx_r * u_c + x_r * du_c;
            gstore_rm(Gr.M + d.oB + (int64_t)k * n * m, o, n, m, m);
        }
        if (Gr.q) store_vec(Gr.q + d.oc + (int64_t)k * n, DX, n, n);
        if (Gr.r) store_vec(Gr.r + d.og + (int64_t)k * m, DU, m, n);
        DX = DXn;
    }
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
