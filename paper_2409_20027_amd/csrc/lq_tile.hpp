// lq_tile.hpp -- wave-level 16x16 FP64 tile algebra for gfx950.
//
// One wave64 owns one tile.  The register layout R(X) of a tile X is the
// accumulator layout of the FP64 16x16x4 matrix instruction on gfx950: lane l
// holds rows 4*r + l/16, r = 0..3, of column l%16 in its register r (rows
// interleaved across the four 16-lane groups; measured with one-hot operands).
// The instruction takes its A operand as A[l%16][l/16] and its B operand as
// B[l/16][l%16], so for the K-slice s of a product P'Q the A operand is
// register s of R(P) and the B operand register s of R(Q): P'Q is formed
// straight from registers (tn below), with no data movement.  Every product of
// the solver is written as P'Q of tiles held in the right form (a matrix, or
// its transpose, loaded transposed from memory or kept transposed across a
// recursion); the few remaining transposes and symmetrisations go through a
// wave-private LDS slot (row stride 17 doubles).
//
// Every small dense object of the solver (an (n+1)x(n+1) homogeneous matrix,
// an (n+1)xm factor, an mxm block) is a zero-padded tile, so n <= 15 and
// m <= 16 fit; the per-lane small factorisations below need m <= MMAX.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define LQK_DEV __device__ __forceinline__

constexpr int TE = 16;            // tile edge
constexpr int LD = 17;            // LDS row stride (doubles)
constexpr int SLOT = TE * LD;     // doubles per LDS tile slot
constexpr int TILE = 256;         // doubles per tile in global memory
constexpr int MMAX = 4;           // largest m for the per-lane small solves

struct Tile {
    d4 v;
};

LQK_DEV int lane() { return threadIdx.x & 63; }
LQK_DEV int tcol() { return threadIdx.x & 15; }
LQK_DEV int tgrp() { return (threadIdx.x >> 4) & 3; }
// Row of register r of this lane.
LQK_DEV int trow(int r) { return 4 * r + tgrp(); }

// Ordering point for LDS hand-offs between the lanes of one wave.  LDS
// instructions of a wave are executed in order, so a wavefront-scope fence
// (which keeps the compiler from moving LDS accesses across it) is enough;
// unlike a workgroup barrier it does not wait for outstanding global loads.
LQK_DEV void wsync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

LQK_DEV Tile tzero()
{
    Tile t;
    t.v = (d4){0.0, 0.0, 0.0, 0.0};
    return t;
}

LQK_DEV Tile tident(int n1)
{
    Tile t;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) t.v[r] = (trow(r) == c && c < n1) ? 1.0 : 0.0;
    return t;
}

LQK_DEV Tile tadd(const Tile &a, const Tile &b)
{
    Tile t;
    t.v = a.v + b.v;
    return t;
}
LQK_DEV Tile tsub(const Tile &a, const Tile &b)
{
    Tile t;
    t.v = a.v - b.v;
    return t;
}
// Global memory, tile-native layout: 64 lanes x 4 doubles, 2 KiB, coalesced.
LQK_DEV Tile gload(const double *p)
{
    Tile t;
    t.v = *reinterpret_cast<const d4 *>(p + 4 * lane());
    return t;
}
LQK_DEV void gstore(double *p, const Tile &t) { *reinterpret_cast<d4 *>(p + 4 * lane()) = t.v; }

// Constants read by lanes whose tile entry is not backed by an input array.
__device__ double kConst01[2] = {0.0, 1.0};   // global address space: loads stay global_load
LQK_DEV const double *zptr() { return &kConst01[0]; }
LQK_DEV const double *optr() { return &kConst01[1]; }

// One global load from a per-lane address that was chosen before the load.
// The address goes through an empty asm so that the compiler sees one load of
// an opaque address: it cannot duplicate the load into the branches of the
// address selection, and nothing depends on a loaded value until it is used.
// Independent loads then issue back to back and a load issued one stage ahead
// is only waited for where it is consumed.
LQK_DEV double ldg(const double *p)
{
    uint64_t a = (uint64_t)p;
    asm("" : "+v"(a));
    return *(const __attribute__((address_space(1))) double *)a;
}
// Last word of a raw (unswizzled, stride 0) buffer resource on gfx9-class
// GPUs: 32-bit data format, the value the ROCm libraries use for raw buffers.
constexpr int kRawBufferWord3 = 0x00020000;

// A raw buffer resource over the first len doubles at p (p null: an empty
// range).  The hardware's range check returns 0 for a load past the end, so a
// masked load needs no per-lane address selection.
LQK_DEV __amdgpu_buffer_rsrc_t brsrc(const double *p, int len)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(p ? p : zptr()), (short)0, p ? len * 8 : 0, kRawBufferWord3);
}
// Element idx of the range (0 past its end).
LQK_DEV double bload(__amdgpu_buffer_rsrc_t r, int idx)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0);
    return __builtin_bit_cast(double, v);
}

// Store to byte offset off of the range; a store at or past its end is
// dropped by the same check, so a masked store needs no branch.
constexpr int BOOB = (int)0x80000000u;   // an offset past any range
LQK_DEV void bstore(__amdgpu_buffer_rsrc_t r, int off, double x)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, x), r, off, 0, 0);
}

// A tile's leading n1 x n1 block stored row-major with row stride n1 at p
// (the start of a TILE slot): only n1^2 doubles move; the rest of the tile
// is zero.
LQK_DEV Tile gload_c(const double *p, int n1)
{
    const __amdgpu_buffer_rsrc_t rs = brsrc(p, n1 * n1);
    const int c = tcol();
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        t.v[r] = bload(rs, (i < n1 && c < n1) ? i * n1 + c : n1 * n1);   // past the end: 0
    }
    return t;
}
LQK_DEV void gstore_c(double *p, const Tile &t, int n1)
{
    const __amdgpu_buffer_rsrc_t rs = brsrc(p, n1 * n1);
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double x = t.v[r];
        bstore(rs, (i < n1 && c < n1) ? 8 * (i * n1 + c) : BOOB, x);
    }
}

// p[idx] if ok, else 0 (from a constant in memory).
LQK_DEV const double *at(const double *p, int64_t idx, bool ok) { return ok ? p + idx : zptr(); }
LQK_DEV double ldz(const double *p, int64_t idx, bool ok) { return ldg(at(p, idx, ok)); }

// Global memory, row-major rows x cols block with leading dimension ld,
// placed at tile offset (i0, j0); everything else zero.
LQK_DEV Tile gload_rm(const double *src, int rows, int cols, int ld, int i0 = 0, int j0 = 0)
{
    Tile t = tzero();
    if (!src) return t;
    const int c = tcol() - j0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r) - i0;
        t.v[r] = ldz(src, (int64_t)i * ld + c, i >= 0 && i < rows && c >= 0 && c < cols);
    }
    return t;
}
// Transposed placement: tile(i0 + i, j0 + j) = src[j * ld + i].
LQK_DEV Tile gload_rm_t(const double *src, int rows, int cols, int ld, int i0 = 0, int j0 = 0)
{
    Tile t = tzero();
    if (!src) return t;
    const int c = tcol() - j0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r) - i0;
        t.v[r] = ldz(src, (int64_t)c * ld + i, i >= 0 && i < rows && c >= 0 && c < cols);
    }
    return t;
}
// Store the rows x cols block at tile offset (i0, j0) to row-major dst.
LQK_DEV void gstore_rm(double *dst, const Tile &t, int rows, int cols, int ld, int i0 = 0, int j0 = 0)
{
    // No early return: an empty block is an empty range, so a sweep's stores
    // stay branch-free and its waits for the loads count them exactly.
    const __amdgpu_buffer_rsrc_t rs = brsrc(dst, (rows > 0 && cols > 0) ? (rows - 1) * ld + cols : 0);
    const int c = tcol() - j0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r) - i0;
        const double x = t.v[r];
        bstore(rs, (i >= 0 && i < rows && c >= 0 && c < cols) ? 8 * (i * ld + c) : BOOB, x);
    }
}

// LDS staging.
LQK_DEV void sput(double *s, const Tile &t)
{
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) s[trow(r) * LD + c] = t.v[r];
}
LQK_DEV Tile sget(const double *s)
{
    Tile t;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) t.v[r] = s[trow(r) * LD + c];
    return t;
}
LQK_DEV Tile sget_t(const double *s)
{
    Tile t;
    const int c = tcol();
#pragma unroll
    for (int r = 0; r < 4; ++r) t.v[r] = s[c * LD + trow(r)];
    return t;
}

// Row permutation that makes the FP32 16x16x4 instruction's accumulator (row
// 4g + r in lane j + 16g, register r) coincide with the FP64 tile layout (row
// 4r + g): feed row pi4(a) of the A operand as its row a.
LQK_DEV int pi4(int a) { return 4 * (a & 3) + (a >> 2); }

// acc + P'Q over the contraction length 4*KS, both operands from registers.
// PR = 0: FP64 products and accumulation.  PR = 1: FP32 products accumulated
// in FP32 (the A operand rows permuted by pi4 with one lane shuffle per
// slice), the result added to the FP64 accumulator in FP64.
template <int KS, int PR>
LQK_DEV d4 tn(const Tile &P, const Tile &Q, d4 acc)
{
    if constexpr (PR == 0) {
#pragma unroll
        for (int k = 0; k < KS; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P.v[k], Q.v[k], acc, 0, 0, 0);
        return acc;
    } else {
        const int src = pi4(tcol()) + 16 * tgrp();
        f4 a4 = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const float a = __shfl((float)P.v[k], src);
            a4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, (float)Q.v[k], a4, 0, 0, 0);
        }
        d4 o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = acc[r] + (double)a4[r];
        return o;
    }
}
// P'Q
template <int KS, int PR>
LQK_DEV Tile tnz(const Tile &P, const Tile &Q)
{
    Tile t;
    t.v = tn<KS, PR>(P, Q, (d4){0.0, 0.0, 0.0, 0.0});
    return t;
}
// acc + P'Q
template <int KS, int PR>
LQK_DEV Tile tna(const Tile &P, const Tile &Q, const Tile &acc)
{
    Tile t;
    t.v = tn<KS, PR>(P, Q, acc.v);
    return t;
}

// A vector v held in column `col` of a tile (v[i] in lane col + 16*(i%4),
// register i/4).  vrows returns v at this lane's four rows, vcol returns
// v at this lane's column; both by lane shuffles, no LDS.
LQK_DEV d4 vrows(const Tile &V, int col)
{
    const int src = col + 16 * tgrp();
    d4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = __shfl(V.v[r], src);
    return o;
}
LQK_DEV double vcol(const Tile &V, int col)
{
    const int c = tcol();
    const int src = col + 16 * (c & 3);
    const double x0 = __shfl(V.v[0], src), x1 = __shfl(V.v[1], src);
    const double x2 = __shfl(V.v[2], src), x3 = __shfl(V.v[3], src);
    const int rr = c >> 2;
    return rr == 0 ? x0 : (rr == 1 ? x1 : (rr == 2 ? x2 : x3));
}

// True on every lane if no entry of the tile is NaN or infinite.
LQK_DEV bool tfinite(const Tile &X)
{
    const bool bad = !(isfinite(X.v[0]) && isfinite(X.v[1]) && isfinite(X.v[2]) && isfinite(X.v[3]));
    return __ballot(bad) == 0;
}

// Symmetric part 1/2 (X + X').
LQK_DEV Tile tsym(const Tile &X, double *s)
{
    wsync();
    sput(s, X);
    wsync();
    Tile t = sget_t(s);
    wsync();
    Tile o;
    o.v = 0.5 * (X.v + t.v);
    return o;
}
LQK_DEV Tile ttrans(const Tile &X, double *s)
{
    wsync();
    sput(s, X);
    wsync();
    Tile t = sget_t(s);
    wsync();
    return t;
}

// ---------------------------------------------------------------------------
// Cross-lane helpers.
// ---------------------------------------------------------------------------

// x of lane l (l uniform), on every lane.
LQK_DEV double rlane(double x, int l)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// x of lane P of this lane's 16-lane row (one 64-bit DPP row broadcast; every
// lane is written, so the old value is irrelevant).
template <int P>
LQK_DEV double rowbcast(double x)
{
    return __builtin_amdgcn_update_dpp(x, x, 0x150 + P, 0xf, 0xf, true);
}

// Register r of a tile for a uniform run-time r.
LQK_DEV double treg(const d4 &v, int r) { return r == 0 ? v[0] : (r == 1 ? v[1] : (r == 2 ? v[2] : v[3])); }

// Exchanges between the four 16-lane rows with the gfx950 lane-swap
// instructions (VALU, no LDS).  permlane16_swap(x, x) returns the even rows'
// content in both rows of each row pair ([0]) and the odd rows' content ([1]);
// permlane32_swap(x, x) returns the low half's content in both halves ([0]) and
// the high half's ([1]).

// max of an unsigned over each pair of rows {0,1}, {2,3} (OFF = 16) or over
// the two halves (OFF = 32), on every lane: one swap leaves one row's values
// in one register and the other row's in the other.
template <int OFF>
LQK_DEV uint32_t rowmax_u(uint32_t x)
{
    const auto sw = OFF == 16 ? __builtin_amdgcn_permlane16_swap(x, x, false, false)
                              : __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return max((uint32_t)sw[0], (uint32_t)sw[1]);
}

// x of row gq (uniform) at this lane's column, on every lane.
LQK_DEV uint32_t rowsel_u(uint32_t x, int gq)
{
    const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    const uint32_t pair = (gq & 1) ? s[1] : s[0];
    const auto t = __builtin_amdgcn_permlane32_swap(pair, pair, false, false);
    return (gq & 2) ? t[1] : t[0];
}
LQK_DEV double rowsel(double x, int gq)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = rowsel_u((uint32_t)b, gq), hi = rowsel_u((uint32_t)(b >> 32), gq);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1/d from the hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - d r) (each squares the relative error).
LQK_DEV double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inverse of the leading n1 x n1 block, in registers.
//
// In-place elimination with partial (row) pivoting: for pivot p the largest
// |X[i][p]|, i >= p, is found over the four lanes holding column p (lane-swap
// reductions), rows p and piv are exchanged by row selects, column p reaches
// every lane of its row by a DPP row broadcast, and the update is one FMA per
// register.  The row exchanges turn into a column permutation of the result,
// undone at the end by one gather.  Rows and columns >= n1 stay zero.  Returns
// false if a pivot is zero or not finite.
// ---------------------------------------------------------------------------
template <int P>
LQK_DEV void gj_step(d4 &v, int n1, bool &ok, int &piv_out)
{
    const int c = tcol(), g = tgrp();
    // Pivot search over rows P..n1-1 of column P with one integer key per
    // candidate: the high word of |x| (sign, exponent and 20 mantissa bits,
    // ordered like |x| for finite and infinite values) with its low 4 bits
    // replaced by 15 - row.  The largest key is a pivot within 2^-16 of the
    // largest |x| (the lowest row among equal keys); a maximum over the lane's
    // registers, then over the column's four lanes (lane swaps), finds it.
    uint32_t key = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = 4 * r + g;
        // through a scalar: a bit cast of the vector element itself has been
        // compiled as a cast of element 0 whatever r is
        const double x = v[r];
        const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32);
        const uint32_t k = (hi & 0x7ffffff0u) | (uint32_t)(15 - i);
        key = (c == P && i >= P && i < n1) ? max(key, k) : key;
    }
    key = rowmax_u<32>(rowmax_u<16>(key));
    const uint32_t kp = (uint32_t)__builtin_amdgcn_readlane((int)key, P);
    const int piv = 15 - (int)(kp & 15u);
    // a pivot column that is zero to the key's resolution, or a pivot that is
    // not finite
    ok = ok && (kp >= 16u) && ((kp & 0x7ff00000u) != 0x7ff00000u);
    constexpr int gp = P & 3, rp = P >> 2;
    // row P (on every lane); it moves to the pivot row's place unless the
    // pivot is already on the diagonal (piv is uniform: the branch is scalar)
    const double rowP = rowsel(v[rp], gp);
    double rowQ = rowP;
    if (piv != P) {
        const int gq = piv & 3, rq = piv >> 2;
        rowQ = rowsel(treg(v, rq), gq);   // pivot row
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r == rq && g == gq) v[r] = rowP;
    }
    const double pinv = recip(rlane(rowQ, P));
    const double prow = rowQ * pinv;
    // v - colp (x) w is the whole elimination step for every row but P: with
    // w[P] = 1 + 1/pivot, column P becomes -colp/pivot.  Row P becomes wP.
    const double w = (c == P) ? 1.0 + pinv : prow;
    const double wP = (c == P) ? pinv : prow;
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = fma(-rowbcast<P>(v[r]), w, v[r]);
    if (g == gp) v[rp] = wP;
    piv_out = piv;
}

template <int P, int PMAX>
LQK_DEV void gj_steps(d4 &v, int n1, int steps, bool &ok, int *perm)
{
    if constexpr (P < PMAX) {
        if (P < steps) {
            gj_step<P>(v, n1, ok, perm[P]);
            gj_steps<P + 1, PMAX>(v, n1, steps, ok, perm);
        }
    }
}

// Inverse of the leading n1 x n1 block of X (n1 <= 4 * NK), zero elsewhere.
// homog: X has the form [[M, 0], [r, 1]] (last column e_n, as I + J~ C~ for a
// homogeneous C~ with zero last row and column); pivots are then taken among
// the first n1 - 1 rows and the last step, a no-op, is skipped.
template <int NK>
LQK_DEV bool gj_inverse(Tile &X, int n1, bool homog = false)
{
    bool ok = true;
    int perm[4 * NK];
#pragma unroll
    for (int p = 0; p < 4 * NK; ++p) perm[p] = p;
    const int rows = homog ? n1 - 1 : n1;
    gj_steps<0, 4 * NK>(X.v, rows, rows, ok, perm);
    // result column j is column src(j) of the eliminated matrix, src being the
    // composition of the row exchanges taken in order
    int x = tcol();
#pragma unroll
    for (int p = 0; p < 4 * NK; ++p) {
        const int q = perm[p];
        x = (x == p) ? q : ((x == q) ? p : x);
    }
    const int src = x + 16 * tgrp();
#pragma unroll
    for (int r = 0; r < 4; ++r) X.v[r] = __shfl(X.v[r], src);
    return ok;
}

// ---------------------------------------------------------------------------
// Small (m <= MMAX) blocks.  The m x m block of a tile lives in register 0 of
// lanes j + 16 i.  The solver's inverses work on it in place across those
// lanes; the element build (not on the hot path) reads it on every lane
// (readlane), factorises it redundantly and writes the result back by a
// per-lane select.
// ---------------------------------------------------------------------------

// The leading m x m block of W on every lane, identity-padded to MMAX.
LQK_DEV void small_from_tile(const Tile &W, int m, double a[MMAX][MMAX])
{
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
            const double v = rlane(W.v[0], j + 16 * i);
            a[i][j] = (i < m && j < m) ? v : (i == j ? 1.0 : 0.0);
        }
}

// Tile holding the leading m x m block of a (TR: of a'), zero elsewhere.  The
// entries are the same on every lane; register 0 of lane j + 16 i takes entry
// (i, j) by a chain of selects on the lane's row and column (two conditions,
// so the chain stays in registers instead of becoming an indexed table).
template <bool TR>
LQK_DEV Tile small_to_tile(const double a[MMAX][MMAX], int m)
{
    const int c = tcol(), g = tgrp();
    double v = 0.0;
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) v = (g == i && c == j) ? (TR ? a[j][i] : a[i][j]) : v;
    Tile t = tzero();
    t.v[0] = (c < m && g < m) ? v : 0.0;
    return t;
}

// One unpivoted Gauss-Jordan step on the leading 4 x 4 block, which lives in
// register 0 (row i in lane group i).  The pivots of the unpivoted elimination
// are the D of W = L D L', so they are all positive iff W is positive definite.
template <int P>
LQK_DEV void small_gj_step(double &v0, bool &ok)
{
    const int c = tcol(), g = tgrp();
    const double piv = rlane(v0, P + 16 * P);
    ok = ok && (piv > 0.0) && (piv < INFINITY);
    const double pinv = recip(piv);
    const double rowP = rowsel(v0, P);     // W[P][c]
    const double cp = rowbcast<P>(v0);     // W[g][P]
    const double prow = (c == P) ? pinv : rowP * pinv;
    v0 = (g == P) ? prow : ((c == P) ? -cp * pinv : fma(-cp, prow, v0));
}

// Inverse of a symmetric positive definite m x m block W (m <= 4) across the
// lanes that hold it (no per-lane copy of the block).  The block is padded to
// 4 x 4 with an identity, so the four steps run without branches and the
// padding steps change nothing.  W^{-1} is symmetric, so the result also
// serves as R(W^{-1}'): tn(WiT, X) = W^{-1} X.  False if W is not positive
// definite.
LQK_DEV bool spd_inverse_t(const Tile &W, int m, Tile &WiT)
{
    const int c = tcol(), g = tgrp();
    const bool in = (c < m) && (g < m);
    double v0 = in ? W.v[0] : ((c == g) ? 1.0 : 0.0);
    bool ok = true;
    small_gj_step<0>(v0, ok);
    small_gj_step<1>(v0, ok);
    small_gj_step<2>(v0, ok);
    small_gj_step<3>(v0, ok);
    WiT = tzero();
    WiT.v[0] = in ? v0 : 0.0;
    return ok;
}

// Pivoted register Gauss-Jordan for an m x m block, kept out of line: it is
// the rare branch of gen_inverse_t.
LQK_DEV bool small_pivoted_inverse(Tile &W, int m) { return gj_inverse<1>(W, m); }

// Same for a symmetric m x m block that may be indefinite: the unpivoted
// elimination when W is positive definite (the usual case), the pivoted
// register Gauss-Jordan otherwise (a uniform branch).  False if W is singular.
LQK_DEV bool gen_inverse_t(const Tile &W, int m, Tile &WiT)
{
    if (spd_inverse_t(W, m, WiT)) return true;
    WiT = W;
    return small_pivoted_inverse(WiT, m);
}

// L^{-1} of the Cholesky factor of an SPD m x m block given on every lane
// (identity-padded), in place.  False if not positive definite.
LQK_DEV bool small_chol_inv(double a[MMAX][MMAX])
{
    bool ok = true;
    double l[MMAX][MMAX];
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        double d = a[j][j];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= l[j][p] * l[j][p];
        ok = ok && (d > 0.0) && (d < INFINITY);
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        l[j][j] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < MMAX; ++i) {
            double v = a[i][j];
#pragma unroll
            for (int p = 0; p < j; ++p) v -= l[i][p] * l[j][p];
            l[i][j] = v * inv;
        }
    }
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
#pragma unroll
        for (int i = 0; i < MMAX; ++i) a[i][j] = 0.0;
        a[j][j] = 1.0 / l[j][j];
#pragma unroll
        for (int i = j + 1; i < MMAX; ++i) {
            double v = 0.0;
#pragma unroll
            for (int p = j; p < i; ++p) v += l[i][p] * a[p][j];
            a[i][j] = -v / l[i][i];
        }
    }
    return ok;
}

// Launch a kernel template <NK, PR> for the run-time slice count and precision.
#define LQK_DISPATCH(nk, pr, CALL)   \
    if (pr) {                        \
        switch (nk) {                \
        case 1: CALL(1, 1); break;   \
        case 2: CALL(2, 1); break;   \
        case 3: CALL(3, 1); break;   \
        default: CALL(4, 1); break;  \
        }                            \
    } else {                         \
        switch (nk) {                \
        case 1: CALL(1, 0); break;   \
        case 2: CALL(2, 0); break;   \
        case 3: CALL(3, 0); break;   \
        default: CALL(4, 0); break;  \
        }                            \
    }

// Horizons the status encoding can report: stages k <= T < 2^23 keep
// (-code) | (k << 8) a positive int32.
constexpr int TMAX_STATUS = 1 << 23;

// Report a failure of an instance: status = (-code) | (k << 8).  Of several
// failures the one at the largest stage index is kept (the first one a
// backward sweep over the stages meets), whatever the order the waves finish in.
LQK_DEV void report(int32_t *status, int inst, int code, int k)
{
    if (status && lane() == 0) atomicMax(&status[inst], (int32_t)((-code) | (k << 8)));
}

}  // namespace lqk
