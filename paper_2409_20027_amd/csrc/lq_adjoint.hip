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

// [[A, 0], [0, 1]]: the dynamics without their offset.
LQK_DEV Tile load_A_noc(const ProbPtrs &P, const InstDesc &d, int k)
{
    const int n = d.n;
    Tile t = gload_rm(P.A + d.oA + (int64_t)k * n * n, n, n, n);
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (trow(r) == n && c == n) t.v[r] = 1.0;
    return t;
}

// Backward map Y~_k = [[F_k', h_k], [0, 1]].
template <int NK, int PR>
LQK_DEV Tile back_map(const ProbPtrs &P, const AdjPtrs &J, const InstDesc &d, int k, double *s0, double *s1)
{
    const int n = d.n, m = d.m;
    const Tile Gh = load_Gh(J.G, J.g, d, k);
    const Tile F = mmak<1, PR, false, false>(load_Bh(P, d, k), Gh, load_A_noc(P, d, k), s0, s1);
    Tile Ft = ttrans(F, s0);
    const Tile GU = load_vec(J.gu + d.og + (int64_t)k * m, m, n, -1);
    const Tile H = mmk<1, PR, true, false>(Gh, GU, s0, s1);  // column n: Gamma' gu (rows < n)
    const Tile GX = load_vec(J.gx + d.os + (int64_t)k * n, n, n, -1);
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        if (i == n)
            Ft.v[r] = (c == n) ? 1.0 : 0.0;
        else if (c == n)
            Ft.v[r] = (i < n) ? GX.v[r] + H.v[r] : 0.0;
    }
    return Ft;
}

// Segment fold of the backward maps: Psi_s = Y~_{k0} ... Y~_{k1-1}; the block
// of the last segment also writes the terminal vector map [[0, gx_T], [0, 1]].
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_back_fold(ProbPtrs P, AdjPtrs J, const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      double *__restrict__ Y)
{
    __shared__ double lds[2 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    if (s == d.nseg - 1)
        gstore(Y + (int64_t)(d.xbase + d.nseg) * TILE, load_vec(J.gx + d.os + (int64_t)d.T * d.n, d.n, d.n, d.n));
    if (s == 0) return;   // never read: segment s starts from entry s + 1
    Tile Psi = tident(d.n + 1);
    for (int k = k0; k < k1; ++k) Psi = mmk<NK, PR, false, false>(Psi, back_map<NK, PR>(P, J, d, k, s0, s1), s0, s1);
    gstore(Y + (int64_t)(d.xbase + s) * TILE, Psi);
}

// Inside each segment, from s~ at its right end: s~_k and gamma~_k.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_back_apply(ProbPtrs P, AdjPtrs J, const InstDesc *__restrict__ inst,
                                                       const int32_t *__restrict__ seg_start, int batch,
                                                       const double *__restrict__ Yfin, int32_t *status)
{
    __shared__ double lds[3 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT, *s2 = lds + 2 * SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    Tile SV = gload(Yfin + (int64_t)(d.xbase + s + 1) * TILE);   // [[0, s~_{k1}], [0, 1]]
    if (s == d.nseg - 1) store_vec(J.st + d.os + (int64_t)d.T * n, SV, n, n);
    int code = 0, fk = 0;
    for (int k = k1 - 1; k >= k0; --k) {
        const Tile Bh = load_Bh(P, d, k);
        const Tile SB = mmk<NK, PR, false, false>(load_Sh(J.S, J.s, d, k + 1), Bh, s0, s1);
        const Tile Quu = mmak<NK, PR, true, false>(Bh, SB, load_R(P, d, k), s0, s1);
        Tile Qi;
        if (!spd_inverse(Quu, m, Qi, s2) && !code) {
            code = ADJ_ERR_NOT_PD;
            fk = k;
        }
        const Tile BS = mmak<NK, PR, true, false>(Bh, SV, load_vec(J.gu + d.og + (int64_t)k * m, m, n, -1), s0, s1);
        Tile Gt = mmk<1, PR, false, false>(Qi, BS, s0, s1);
        Gt.v = -Gt.v;
        store_vec(J.gt + d.og + (int64_t)k * m, Gt, m, n);
        SV = mmk<NK, PR, false, false>(back_map<NK, PR>(P, J, d, k, s0, s1), SV, s0, s1);
        store_vec(J.st + d.os + (int64_t)k * n, SV, n, n);
    }
    if (code) report(status, i, code, fk);
}

// Closed-loop map of the derivative: [[A + B Gamma, B gamma~], [0, 1]].
template <int PR>
LQK_DEV Tile fwd_map(const ProbPtrs &P, const AdjPtrs &J, const InstDesc &d, int k, double *s0, double *s1)
{
    return mmak<1, PR, false, false>(load_Bh(P, d, k), load_Gh(J.G, J.gt, d, k), load_A_noc(P, d, k), s0, s1);
}

template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_fwd_fold(ProbPtrs P, AdjPtrs J, const InstDesc *__restrict__ inst,
                                                     const int32_t *__restrict__ seg_start, int batch,
                                                     double *__restrict__ Y)
{
    __shared__ double lds[2 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    if (s == 0) gstore(Y + (int64_t)d.xbase * TILE, load_vec(nullptr, d.n, d.n, d.n));   // dx_0 = 0
    if (s == d.nseg - 1) return;   // never read: segment s starts from entry s
    Tile Phi = tident(d.n + 1);
    for (int k = k0; k < k1; ++k) Phi = mmk<NK, PR, false, false>(fwd_map<PR>(P, J, d, k, s0, s1), Phi, s0, s1);
    gstore(Y + (int64_t)(d.xbase + s + 1) * TILE, Phi);
}

// Outer product a b' of two vectors held in column `col`, rows from a, columns from b.
LQK_DEV Tile outer(const d4 &ar, double bc)
{
    Tile o;
    o.v = ar * bc;
    return o;
}

template <int NK, int PR>
__global__ __launch_bounds__(64) void k_adj_fwd_apply(ProbPtrs P, AdjPtrs J, GradPtrs Gr,
                                                      const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      const double *__restrict__ Yfin)
{
    __shared__ double lds[2 * SLOT];
    double *s0 = lds, *s1 = lds + SLOT;
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n, m = d.m;
    Tile DX = gload(Yfin + (int64_t)(d.xbase + s) * TILE);   // [[0, dx_k0], [0, 1]]
    if (s == 0 && Gr.x0) {
        const Tile DL0 = mmk<NK, PR, false, false>(load_Sh(J.S, J.st, d, 0), DX, s0, s1);
        store_vec(Gr.x0 + d.on, DL0, n, n);
    }
    for (int k = k0; k < k1; ++k) {
        const Tile Gh = load_Gh(J.G, J.gt, d, k);
        const Tile Bh = load_Bh(P, d, k);
        const Tile DU = mmk<NK, PR, false, false>(Gh, DX, s0, s1);
        const Tile DXn = mmak<1, PR, false, false>(Bh, DU, mmk<NK, PR, false, false>(load_A_noc(P, d, k), DX, s0, s1), s0, s1);
        const Tile DL1 = mmk<NK, PR, false, false>(load_Sh(J.S, J.st, d, k + 1), DXn, s0, s1);
        const Tile X = load_vec(J.x + d.os + (int64_t)k * n, n, n, -1);
        const Tile U = load_vec(J.u + d.og + (int64_t)k * m, m, n, -1);
        const Tile L1 = load_vec(J.lam + d.os + (int64_t)(k + 1) * n, n, n, -1);
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
                           const int32_t *seg_start, int batch, const double *Yfin, int32_t *status)
{
#define CALL(K, R) hipLaunchKernelGGL((k_adj_back_apply<K, R>), dim3(grid), dim3(64), 0, st, P, J, inst, seg_start, batch, Yfin, status)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
void launch_adj_fwd_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, const InstDesc *inst,
                         const int32_t *seg_start, int batch, double *Y)
{
#define CALL(K, R) hipLaunchKernelGGL((k_adj_fwd_fold<K, R>), dim3(grid), dim3(64), 0, st, P, J, inst, seg_start, batch, Y)
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
