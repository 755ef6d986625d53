// lq_desc.hpp -- instance descriptors shared by the host plan and the kernels,
// plus the loaders that assemble a stage's data into homogeneous tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lq_tile.hpp"

namespace lqk {

// Per-instance sizes and offsets (in doubles) into the packed arrays.
struct InstDesc {
    int32_t n, m, T;
    int32_t nseg;       // segments of this instance
    int32_t L;          // stages per segment (last one may be shorter)
    int32_t seg0;       // first global segment index
    int32_t xbase;      // first index in the scan buffers (seg0 + instance index)
    int32_t orig;       // index of the instance in the caller's batch (its status word)
    int64_t elem0;      // first element index (T + 1 elements per instance)
    int64_t oA, oB, oR, oc, oQT, on;   // offsets: A/Q (T n n), B/M (T n m), R (T m m),
                                       // c/q (T n), QT (n n), qT/x0 (n)
    int64_t oS, os, oG, og;            // S ((T+1) n n), s/x/lambda ((T+1) n),
                                       // Gamma (T m n), gamma/u/r (T m)
};

struct ProbPtrs {
    const double *A, *B, *c, *Q, *R, *M, *q, *r, *QT, *qT, *x0;
};

struct ValPtrs {
    double *S, *s, *G, *g;
};

// Adjoint inputs (forward solution, loss gradients) and its workspace vectors
// s~ (same packing as s) and gamma~ (same packing as gamma).
struct AdjPtrs {
    const double *S, *s, *G, *g;
    const double *x, *u, *lam;
    const double *gx, *gu;
    double *st, *gt;
};

struct GradPtrs {
    double *A, *B, *c, *Q, *R, *M, *q, *r, *QT, *qT, *x0;
};

// Newton / interior-point: device scalars (indices match include/lqscan.h).
enum { NMPC_MU = 0, NMPC_ALPHA = 1, NMPC_NU = 2, NMPC_COST = 3, NMPC_PRED = 4, NMPC_RHO = 5,
       NMPC_ACCEPTED = 6, NMPC_COST_NEW = 7, NMPC_GRAD = 8, NMPC_RP = 9, NMPC_RD = 10, NMPC_LEVEL_TOL = 11,
       NMPC_LEVEL_MAX = 12, NMPC_LEVEL_ITERS = 13, NMPC_LEVEL_DONE = 14, NMPC_NSCAL = 15 };
enum { MODEL_TANH = 0, MODEL_PENDULUM = 1, MODEL_CARTPOLE = 2 };

// A batch of `batch` instances of equal sizes (nx, nu, T): per-instance arrays
// are packed instance by instance (x0 [batch][nx], trajectories, workspace,
// scalars [batch][NMPC_NSCAL]); model, costs, bounds and reference are shared.
struct NmpcPtrs {
    int nx, nu, T, batch;
    double h;
    const double *W, *Bm, *Q, *R, *QT, *xref, *x0;
    double umin, umax;
    int model;
    double prm[4];
    // rho > 0: the ADMM augmentation rho/2 |h(u) - z + v/rho|^2 (z, v: [T][2 nu],
    // rows u - umax then umin - u) replaces the barrier
    double rho;
    double *z, *v;
};

// Newton workspace arrays (stage-major like the LQ problem arrays).
struct NmpcWork {
    double *QTb;   // Q_T replicated per instance (the LQ step takes one per instance)
    double *A, *B, *P, *M, *Rt, *Rh, *d, *th, *g, *lam, *lamT;
    double *S, *s, *G, *gm, *dx, *du, *xc, *uc, *zero;
    int32_t *status;
    double *scal;   // the state's device scalars (level control), NMPC_NSCAL per instance
};

// A barrier level of instance b ended on the device (scal[NMPC_LEVEL_DONE] is
// 0 while it runs, 0.5 after its last iteration, 1 from the next step on):
// the Newton kernels leave the instance unchanged.  `last_ok` lets the commit
// of the last iteration itself (0.5) through.
LQK_DEV bool level_done(const double *scal, int64_t b, bool last_ok = false)
{
    if (!scal) return false;
    const double d = scal[b * NMPC_NSCAL + NMPC_LEVEL_DONE];
    return last_ok ? (d >= 1.0) : (d >= 0.5);
}

// First checkpoint slot of instance i when one carry is kept per group of
// `stride` segments: seg0 / stride + i.  The instance needs
// ceil(nseg / stride) slots, and floor((seg0 + nseg) / stride) + i + 1 >=
// floor(seg0 / stride) + i + ceil(nseg / stride), so the slots of
// consecutive instances never overlap and total_seg / stride + batch slots
// hold them all, without a table that depends on the stride.
LQK_DEV int ckpt_slot(const InstDesc &d, int i, int stride) { return d.seg0 / stride + i; }

// Index of the instance owning global item g, by binary search over the
// prefix array start[0..batch] (start[0] = 0, start[batch] = total).
LQK_DEV int find_inst(const int32_t *start, int batch, int64_t g)
{
    int lo = 0, hi = batch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((int64_t)start[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}
LQK_DEV int find_inst64(const int64_t *start, int batch, int64_t g)
{
    int lo = 0, hi = batch - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Homogeneous stage tiles (n1 = n + 1; the extra coordinate is the constant 1)
// ---------------------------------------------------------------------------

// A~ = [[A, c], [0, 1]]; with_c = false drops the offset: [[A, 0], [0, 1]].
LQK_DEV Tile load_Ah(const ProbPtrs &P, const InstDesc &d, int k, bool with_c = true)
{
    const int n = d.n, c = tcol();
    const double *A = P.A + d.oA + (int64_t)k * n * n;
    const double *cc = (with_c && P.c) ? P.c + d.oc + (int64_t)k * n : nullptr;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *a = zptr();
        if (i < n && c < n)
            a = A + i * n + c;
        else if (c == n && i < n && cc)
            a = cc + i;
        else if (c == n && i == n)
            a = optr();
        t.v[r] = ldg(a);
    }
    return t;
}

// A~' = [[A', 0], [c', 1]]; with_c = false drops the offset: [[A', 0], [0, 1]].
LQK_DEV Tile load_AhT(const ProbPtrs &P, const InstDesc &d, int k, bool with_c = true)
{
    const int n = d.n, c = tcol();
    const double *A = P.A + d.oA + (int64_t)k * n * n;
    const double *cc = (with_c && P.c) ? P.c + d.oc + (int64_t)k * n : nullptr;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *a = zptr();
        if (i < n && c < n)
            a = A + c * n + i;
        else if (i == n && c < n && cc)
            a = cc + c;
        else if (i == n && c == n)
            a = optr();
        t.v[r] = ldg(a);
    }
    return t;
}

// B~' = [B', 0]   (m x (n+1))
LQK_DEV Tile load_BhT(const ProbPtrs &P, const InstDesc &d, int k)
{
    return gload_rm_t(P.B + d.oB + (int64_t)k * d.n * d.m, d.m, d.n, d.m);
}

// Q~ = [[Q, q], [q', 0]]
LQK_DEV Tile load_Qh(const ProbPtrs &P, const InstDesc &d, int k)
{
    const int n = d.n, c = tcol();
    const double *Q = P.Q + d.oA + (int64_t)k * n * n;
    const double *qq = P.q ? P.q + d.oc + (int64_t)k * n : nullptr;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *a = zptr();
        if (i < n && c < n)
            a = Q + i * n + c;
        else if (qq && c == n && i < n)
            a = qq + i;
        else if (qq && i == n && c < n)
            a = qq + c;
        t.v[r] = ldg(a);
    }
    return t;
}

// M~' = [M', r]   (m x (n+1))
LQK_DEV Tile load_MhT(const ProbPtrs &P, const InstDesc &d, int k)
{
    const int n = d.n, m = d.m, c = tcol();
    const double *M = P.M ? P.M + d.oB + (int64_t)k * n * m : nullptr;
    const double *rr = P.r ? P.r + d.og + (int64_t)k * m : nullptr;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = trow(r);
        const double *p = zptr();
        if (M && a < m && c < n)
            p = M + c * m + a;
        else if (rr && a < m && c == n)
            p = rr + a;
        t.v[r] = ldg(p);
    }
    return t;
}

// R (m x m)
LQK_DEV Tile load_R(const ProbPtrs &P, const InstDesc &d, int k)
{
    return gload_rm(P.R + d.oR + (int64_t)k * d.m * d.m, d.m, d.m, d.m);
}

// Terminal J~ = [[sym(Q_T), q_T], [q_T', 0]]
LQK_DEV Tile load_terminal_J(const ProbPtrs &P, const InstDesc &d, double *s)
{
    const int n = d.n;
    Tile t = gload_rm(P.QT + d.oQT, n, n, n);
    t = tsym(t, s);
    if (P.qT) {
        const double *qq = P.qT + d.on;
        const int c = tcol();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = trow(r);
            const bool col = (c == n && i < n), row = (i == n && c < n);
            if (col || row) t.v[r] = qq[col ? i : c];
        }
    }
    return t;
}

// The corner tile E_nn (the homogeneous part of a terminal-type A~).
LQK_DEV Tile corner(int n)
{
    Tile t = tzero();
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) t.v[r] = (trow(r) == n && c == n) ? 1.0 : 0.0;
    return t;
}

// Gamma~ = [Gamma, gamma]   (m x (n+1)) from the control-law outputs
// (gam = nullptr: [Gamma, 0]).
LQK_DEV Tile load_Gh(const double *Gam, const double *gam, const InstDesc &d, int k)
{
    const int n = d.n, m = d.m, c = tcol();
    const double *G = Gam + d.oG + (int64_t)k * m * n;
    const double *gg = gam ? gam + d.og + (int64_t)k * m : nullptr;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = trow(r);
        const double *p = zptr();
        if (a < m && c < n)
            p = G + a * n + c;
        else if (a < m && c == n && gg)
            p = gg + a;
        t.v[r] = ldg(p);
    }
    return t;
}

// S~ = [[S, s], [s', 0]] from the value outputs (stage k = 0..T).
LQK_DEV Tile load_Sh(const double *S, const double *s, const InstDesc &d, int k)
{
    const int n = d.n, c = tcol();
    const double *Sk = S + d.oS + (int64_t)k * n * n;
    const double *ss = s + d.os + (int64_t)k * n;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *p = zptr();
        if (i < n && c < n)
            p = Sk + i * n + c;
        else if (c == n && i < n)
            p = ss + i;
        else if (i == n && c < n)
            p = ss + c;
        t.v[r] = ldg(p);
    }
    return t;
}

// A vector v (length len) held in column `col` of a tile, with an optional
// homogeneous 1 at row `one_row` (-1 = none).
LQK_DEV Tile load_vec(const double *v, int len, int col, int one_row)
{
    const int c = tcol();
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *p = zptr();
        if (c == col && i < len && v)
            p = v + i;
        else if (c == col && i == one_row)
            p = optr();
        t.v[r] = ldg(p);
    }
    return t;
}
LQK_DEV void store_vec(double *v, const Tile &t, int len, int col)
{
    const __amdgpu_buffer_rsrc_t rs = brsrc(v, len > 0 ? len : 0);   // null or empty: every store dropped
    const bool mine = (tcol() == col);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double x = t.v[r];
        bstore(rs, (mine && i < len) ? 8 * i : BOOB, x);
    }
}

// ---------------------------------------------------------------------------
// Stage data staged through LDS.
//
// One stage's problem arrays are copied into a wave-private LDS buffer with
// coalesced loads (lane l reads elements l, l + 64, ... of each array) and
// the homogeneous tiles are then gathered from the buffer with per-lane LDS
// addresses that depend only on (n, m) and the lane; padding entries read two
// constant slots (0.0 and 1.0).  The loads of the next stage are issued into
// registers before the current stage's compute and written to the other of
// two buffers after it, so their latency hides behind a stage.  This replaces
// per-entry address selection (a chain of per-lane conditions for every
// register of every tile) by one LDS read per register.
// ---------------------------------------------------------------------------

// Buffer layout in doubles: [0] = 0.0, [1] = 1.0, then A, c, Q, q, B, R, M, r
// of one stage, then 64 doubles of write-off space for lanes past an array.
struct StageLayout {
    int oA, oc, oQ, oq, oB, oR, oM, orr, trash;
};
LQK_DEV StageLayout stage_layout(int n, int m)
{
    StageLayout L;
    L.oA = 2;
    L.oc = L.oA + n * n;
    L.oQ = L.oc + n;
    L.oq = L.oQ + n * n;
    L.oB = L.oq + n;
    L.oR = L.oB + n * m;
    L.oM = L.oR + m * m;
    L.orr = L.oM + n * m;
    L.trash = L.orr + m;
    return L;
}

// Buffer size in doubles for n <= 4 NK - 1, m <= MMAX.
template <int NK>
constexpr int stage_buf_size()
{
    constexpr int nm = 4 * NK - 1;
    return 2 + 2 * nm * nm + 2 * nm + 2 * nm * MMAX + MMAX * MMAX + MMAX + 64;
}

// One array of a stage's data: stage k's elements are
// base[k * stride .. k * stride + len), copied to buffer offset off.  A null
// array reads as zeros: an empty range over a valid address.
struct StageArr {
    const double *base;
    int stride, bytes, len, off;   // stage offsets inside one instance's array fit 32 bits
};
LQK_DEV StageArr stage_arr(const double *p, int stride, int len, int off)
{
    StageArr a;
    a.base = p ? p : zptr();
    a.stride = p ? stride : 0;
    a.bytes = p ? 8 * len : 0;
    a.len = len;
    a.off = off;
    return a;
}

// Register slots of the arrays in flight: S_j = ceil(max len_j / 64).
template <int... S>
struct StageRegs {
    double v[(S + ... + 0)];
};

// Lane l loads elements l, l + 64, ... of stage k's array (0 past its end).
template <int S>
LQK_DEV void fetch_arr(const StageArr &a, int k, double *v)
{
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.base + (uint32_t)(k * a.stride)), (short)0, a.bytes, kRawBufferWord3);
#pragma unroll
    for (int j = 0; j < S; ++j) v[j] = bload(r, lane() + 64 * j);
}
// ... and writes them to the buffer (lanes past the array to the write-off area).
template <int S>
LQK_DEV void put_arr(double *buf, const StageArr &a, int trash, const double *v)
{
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const int idx = lane() + 64 * j;
        buf[idx < a.len ? a.off + idx : trash + lane()] = v[j];
    }
}

template <int... S>
LQK_DEV void arr_fetch(const StageArr *a, int k, StageRegs<S...> &f)
{
    int j = 0, o = 0;
    ((fetch_arr<S>(a[j], k, f.v + o), o += S, ++j), ...);
}
template <int... S>
LQK_DEV void arr_put(double *buf, const StageArr *a, int trash, const StageRegs<S...> &f)
{
    int j = 0, o = 0;
    ((put_arr<S>(buf, a[j], trash, f.v + o), o += S, ++j), ...);
}

// body(k, cur) for the stages k = kfirst + dir j, j = 0 .. cnt - 1, each
// stage's arrays staged through the two LDS buffers stg and stg + SZ.  Two
// register sets hold stages in flight: stage j + 2's loads are issued before
// body(j) and written to LDS after body(j + 1), so every load has two stages
// of products to arrive in.  Both halves of the unrolled pair sit in the loop
// body (no path back to the top leaves a load's wait to the next pass).
// Loads issued before the call have arrived when the first stage's data is
// written, so none of them is waited for inside the loop.
template <class Regs, class Body>
LQK_DEV void sweep_ahead2(double *stg, int SZ, const StageArr *arr, int trash, int kfirst, int cnt, int dir,
                          Body &&body)
{
    auto kat = [&](int j) { return kfirst + dir * min(j, cnt - 1); };
    Regs fa, fb;
    arr_fetch(arr, kat(0), fa);
    arr_put(stg, arr, trash, fa);
    arr_fetch(arr, kat(1), fb);
    wsync();
    auto step = [&](int j, const double *cur, double *nxt, Regs &fnew, const Regs &fput)
                    __attribute__((always_inline)) {
        // keeps the scheduler from hoisting the next stage's loads above this
        // stage's write to LDS, whose wait would then cover them too
        __builtin_amdgcn_sched_barrier(0);
        arr_fetch(arr, kat(j + 2), fnew);
        body(kfirst + dir * j, cur);
        arr_put(nxt, arr, trash, fput);
        wsync();
    };
    int j = 0;
    for (; j + 1 < cnt; j += 2) {
        step(j, stg, stg + SZ, fa, fb);
        step(j + 1, stg + SZ, stg, fb, fa);
    }
    if (j < cnt) step(j, stg, stg + SZ, fa, fb);
}

// The problem arrays of a value-pass stage: A, c, Q, q, B, R, and with cross
// terms (MR) M, r.
template <int NK, bool MR>
struct ValueStage;
template <int NK>
struct ValueStage<NK, false> {
    static constexpr int NM = 4 * NK - 1, SA = (NM * NM + 63) / 64, SB = (NM * MMAX + 63) / 64;
    using Regs = StageRegs<SA, 1, SA, 1, SB, 1>;
    StageArr a[6];
};
template <int NK>
struct ValueStage<NK, true> {
    static constexpr int NM = 4 * NK - 1, SA = (NM * NM + 63) / 64, SB = (NM * MMAX + 63) / 64;
    using Regs = StageRegs<SA, 1, SA, 1, SB, 1, SB, 1>;
    StageArr a[8];
};
template <int NK, bool MR>
LQK_DEV ValueStage<NK, MR> value_stage(const ProbPtrs &P, const InstDesc &d, const StageLayout &L)
{
    ValueStage<NK, MR> v;
    const int n = d.n, m = d.m;
    v.a[0] = stage_arr(P.A + d.oA, n * n, n * n, L.oA);
    v.a[1] = stage_arr(P.c ? P.c + d.oc : nullptr, n, n, L.oc);
    v.a[2] = stage_arr(P.Q + d.oA, n * n, n * n, L.oQ);
    v.a[3] = stage_arr(P.q ? P.q + d.oc : nullptr, n, n, L.oq);
    v.a[4] = stage_arr(P.B + d.oB, n * m, n * m, L.oB);
    v.a[5] = stage_arr(P.R + d.oR, m * m, m * m, L.oR);
    if constexpr (MR) {
        v.a[6] = stage_arr(P.M ? P.M + d.oB : nullptr, n * m, n * m, L.oM);
        v.a[7] = stage_arr(P.r ? P.r + d.og : nullptr, m, m, L.orr);
    }
    return v;
}

LQK_DEV void stage_consts(double *buf)
{
    if (lane() < 2) buf[lane()] = (double)lane();
}

// Per-lane LDS addresses of a tile's four registers (0 = the 0.0 slot).
struct GMap {
    uint32_t a[4];
};

// A~ = [[A, c], [0, 1]]
LQK_DEV GMap gmap_Ah(const StageLayout &L, int n)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        g.a[r] = (i < n && c < n) ? L.oA + i * n + c : (c == n && i < n) ? L.oc + i : (c == n && i == n) ? 1 : 0;
    }
    return g;
}
// Q~ = [[Q, q], [q', 0]]
LQK_DEV GMap gmap_Qh(const StageLayout &L, int n)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        g.a[r] = (i < n && c < n) ? L.oQ + i * n + c : (c == n && i < n) ? L.oq + i : (i == n && c < n) ? L.oq + c : 0;
    }
    return g;
}
// B~ = [[B], [0]]
LQK_DEV GMap gmap_Bh(const StageLayout &L, int n, int m)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        g.a[r] = (i < n && c < m) ? L.oB + i * m + c : 0;
    }
    return g;
}
// B~' = [B', 0]
LQK_DEV GMap gmap_BhT(const StageLayout &L, int n, int m)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = trow(r);
        g.a[r] = (a < m && c < n) ? L.oB + c * m + a : 0;
    }
    return g;
}
// R
LQK_DEV GMap gmap_R(const StageLayout &L, int m)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        g.a[r] = (i < m && c < m) ? L.oR + i * m + c : 0;
    }
    return g;
}
// M~' = [M', r]
LQK_DEV GMap gmap_MhT(const StageLayout &L, int n, int m)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = trow(r);
        g.a[r] = (a < m && c < n) ? L.oM + c * m + a : (a < m && c == n) ? L.orr + a : 0;
    }
    return g;
}

LQK_DEV Tile gather(const double *buf, const GMap &g)
{
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) t.v[r] = buf[g.a[r]];
    return t;
}

// Tile maps from a function (row, col) -> buffer index (0: the 0.0 slot,
// 1: the 1.0 slot).
template <class F>
LQK_DEV GMap gmap_of(F idx)
{
    GMap g;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) g.a[r] = idx(trow(r), c);
    return g;
}

}  // namespace lqk
