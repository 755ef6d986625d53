// lq_tile.hpp -- wave-level 16x16 FP64 tile algebra for gfx950.
//
// One wave64 owns one tile.  The register layout is the accumulator layout of
// the FP64 16x16x4 matrix instruction on gfx950: lane l holds rows
// 4*r + l/16, r = 0..3, of column l%16 (rows interleaved across the four
// 16-lane groups; measured with one-hot operands).  The A operand of the
// instruction is A[l%16][l/16] and the B operand B[l/16][l%16].  Products stage both operands through a
// wave-private LDS slot (row-major, padded row stride of 17 doubles so that
// column reads do not collide on the same banks) and issue ceil(K/4) matrix
// instructions, K being the contraction length actually needed.
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
LQK_DEV Tile tneg(const Tile &a)
{
    Tile t;
    t.v = -a.v;
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

// Address of p[idx] if ok, else of a constant zero.  Every tile entry is one
// load from a per-lane address chosen before the load, so nothing depends on a
// loaded value until it is used: independent loads issue back to back and a
// load issued one stage ahead is only waited for where it is consumed.
LQK_DEV const double *at(const double *p, int64_t idx, bool ok) { return ok ? p + idx : zptr(); }
LQK_DEV double ldz(const double *p, int64_t idx, bool ok) { return *at(p, idx, ok); }

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
    const int c = tcol() - j0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r) - i0;
        if (i >= 0 && i < rows && c >= 0 && c < cols) dst[i * ld + c] = t.v[r];
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

// Stage a tile for products of precision PR (0: FP64, 1: FP32 operands).
template <int PR>
LQK_DEV void sputp(double *s, const Tile &t)
{
    if constexpr (PR == 0) {
        sput(s, t);
    } else {
        float *f = reinterpret_cast<float *>(s);
        const int c = tcol();
#pragma unroll
        for (int r = 0; r < 4; ++r) f[trow(r) * LD + c] = (float)t.v[r];
    }
}

// acc + op(X) op(Y) over contraction length 4*KS, operands already staged.
// PR = 0: FP64 products and accumulation.  PR = 1: FP32 products accumulated
// in FP32, the result added to the FP64 accumulator in FP64.
template <int KS, int PR, bool TX, bool TY>
LQK_DEV d4 mfma_k(const double *sx, const double *sy, d4 acc)
{
    const int c = tcol(), g = tgrp();
    if constexpr (PR == 0) {
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int kk = 4 * k + g;
            const double a = TX ? sx[kk * LD + c] : sx[c * LD + kk];
            const double b = TY ? sy[c * LD + kk] : sy[kk * LD + c];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
        }
        return acc;
    } else {
        const float *fx = reinterpret_cast<const float *>(sx);
        const float *fy = reinterpret_cast<const float *>(sy);
        const int pc = pi4(c);
        f4 a4 = (f4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 0; k < KS; ++k) {
            const int kk = 4 * k + g;
            const float a = TX ? fx[kk * LD + pc] : fx[pc * LD + kk];
            const float b = TY ? fy[c * LD + kk] : fy[kk * LD + c];
            a4 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, a4, 0, 0, 0);
        }
        d4 o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = acc[r] + (double)a4[r];
        return o;
    }
}

// Same with a run-time slice count (small auxiliary products only).
template <bool TX, bool TY>
LQK_DEV d4 mfma_staged(const double *sx, const double *sy, int ks, d4 acc)
{
    const int c = tcol(), g = tgrp();
    for (int k = 0; k < ks; ++k) {
        const int kk = 4 * k + g;
        const double a = TX ? sx[kk * LD + c] : sx[c * LD + kk];
        const double b = TY ? sy[c * LD + kk] : sy[kk * LD + c];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Contraction slices for a contraction length K.
LQK_DEV int kslices(int K) { return (K + 3) >> 2; }

// D = op(X) op(Y) (+ acc).  Stages X into sx and Y into sy (two slots).
template <bool TX, bool TY>
LQK_DEV Tile mm(const Tile &X, const Tile &Y, int K, double *sx, double *sy)
{
    wsync();
    sput(sx, X);
    sput(sy, Y);
    wsync();
    Tile d;
    d.v = mfma_staged<TX, TY>(sx, sy, kslices(K), (d4){0.0, 0.0, 0.0, 0.0});
    wsync();
    return d;
}
template <bool TX, bool TY>
LQK_DEV Tile mma(const Tile &X, const Tile &Y, const Tile &acc, int K, double *sx, double *sy)
{
    wsync();
    sput(sx, X);
    sput(sy, Y);
    wsync();
    Tile d;
    d.v = mfma_staged<TX, TY>(sx, sy, kslices(K), acc.v);
    wsync();
    return d;
}

// Compile-time slice-count versions of mm / mma.
template <int KS, int PR, bool TX, bool TY>
LQK_DEV Tile mmk(const Tile &X, const Tile &Y, double *sx, double *sy)
{
    wsync();
    sputp<PR>(sx, X);
    sputp<PR>(sy, Y);
    wsync();
    Tile d;
    d.v = mfma_k<KS, PR, TX, TY>(sx, sy, (d4){0.0, 0.0, 0.0, 0.0});
    return d;
}
template <int KS, int PR, bool TX, bool TY>
LQK_DEV Tile mmak(const Tile &X, const Tile &Y, const Tile &acc, double *sx, double *sy)
{
    wsync();
    sputp<PR>(sx, X);
    sputp<PR>(sy, Y);
    wsync();
    Tile d;
    d.v = mfma_k<KS, PR, TX, TY>(sx, sy, acc.v);
    return d;
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

// Inverse of the leading n1 x n1 block (zero elsewhere) by in-place
// Gauss-Jordan elimination with partial (row) pivoting; the column order is
// restored at the end.  Returns false if a pivot is zero or not finite.
LQK_DEV bool gj_inverse(Tile &X, int n1, double *s)
{
    const int l = lane(), c = tcol(), g = tgrp();
    wsync();
    sput(s, X);
    wsync();
    bool ok = true;
    int perm = 0;
    for (int p = 0; p < n1; ++p) {
        double v = (l >= p && l < n1) ? fabs(s[l * LD + p]) : -1.0;
        int idx = l;
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) {
            const double ov = __shfl_xor(v, off, 16);
            const int oi = __shfl_xor(idx, off, 16);
            if (ov > v || (ov == v && oi < idx)) {
                v = ov;
                idx = oi;
            }
        }
        const int piv = __shfl(idx, 0);
        const double pmax = __shfl(v, 0);
        ok = ok && (pmax > 0.0) && (pmax < INFINITY);
        if (l == p) perm = piv;
        if (piv != p && l < TE) {
            const double a = s[p * LD + l], b = s[piv * LD + l];
            s[p * LD + l] = b;
            s[piv * LD + l] = a;
        }
        wsync();
        const double pinv = 1.0 / s[p * LD + p];
        const double rowp = s[p * LD + c] * pinv;
        double colp[4], cur[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            colp[r] = s[trow(r) * LD + p];
            cur[r] = s[trow(r) * LD + c];
        }
        wsync();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = trow(r);
            double nv;
            if (i == p)
                nv = (c == p) ? pinv : rowp;
            else
                nv = (c == p) ? -colp[r] * pinv : cur[r] - colp[r] * rowp;
            s[i * LD + c] = nv;
        }
        wsync();
    }
    for (int p = n1 - 1; p >= 0; --p) {
        const int q = __shfl(perm, p);
        if (q != p && l < TE) {
            const double a = s[l * LD + p], b = s[l * LD + q];
            s[l * LD + p] = b;
            s[l * LD + q] = a;
        }
        wsync();
    }
    X = sget(s);
    wsync();
    return ok;
}

// ---------------------------------------------------------------------------
// Per-lane small (m <= MMAX) factorisations.  Every lane reads the whole m x m
// block and factorises it redundantly in registers; the result goes back into
// tile layout through lane 0 and the LDS slot.
// ---------------------------------------------------------------------------

// Read the leading m x m block of a staged slot into a register array,
// identity-padded to MMAX.
LQK_DEV void small_read(const double *s, int m, double a[MMAX][MMAX])
{
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
            const double v = s[i * LD + j];  // in the slot for every i, j < MMAX
            a[i][j] = (i < m && j < m) ? v : (i == j ? 1.0 : 0.0);
        }
}

// In-register Cholesky a = L L' (lower, into a).  False if not PD.
LQK_DEV bool small_chol(double a[MMAX][MMAX])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
        double d = a[j][j];
#pragma unroll
        for (int p = 0; p < j; ++p) d -= a[j][p] * a[j][p];
        ok = ok && (d > 0.0) && (d < INFINITY);
        const double ljj = sqrt(d > 0.0 ? d : 1.0);
        a[j][j] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < MMAX; ++i) {
            double v = a[i][j];
#pragma unroll
            for (int p = 0; p < j; ++p) v -= a[i][p] * a[j][p];
            a[i][j] = v * inv;
        }
#pragma unroll
        for (int i = 0; i < j; ++i) a[i][j] = 0.0;
    }
    return ok;
}

// Inverse of a lower-triangular L (in place).
LQK_DEV void small_tri_inv(double a[MMAX][MMAX])
{
    double li[MMAX][MMAX];
#pragma unroll
    for (int j = 0; j < MMAX; ++j) {
#pragma unroll
        for (int i = 0; i < MMAX; ++i) li[i][j] = 0.0;
        li[j][j] = 1.0 / a[j][j];
#pragma unroll
        for (int i = j + 1; i < MMAX; ++i) {
            double v = 0.0;
#pragma unroll
            for (int p = j; p < i; ++p) v += a[i][p] * li[p][j];
            li[i][j] = -v / a[i][i];
        }
    }
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) a[i][j] = li[i][j];
}

// In-register Gauss-Jordan inverse with partial pivoting (general matrix).
LQK_DEV bool small_gj_inv(double a[MMAX][MMAX])
{
    bool ok = true;
    int perm[MMAX];
#pragma unroll
    for (int p = 0; p < MMAX; ++p) {
        int piv = p;
        double best = fabs(a[p][p]);
#pragma unroll
        for (int i = p + 1; i < MMAX; ++i)
            if (fabs(a[i][p]) > best) {
                best = fabs(a[i][p]);
                piv = i;
            }
        ok = ok && (best > 0.0) && (best < INFINITY);
        perm[p] = piv;
#pragma unroll
        for (int i = p + 1; i < MMAX; ++i) {
            const bool sw = (piv == i);
#pragma unroll
            for (int j = 0; j < MMAX; ++j) {
                const double t = a[p][j];
                a[p][j] = sw ? a[i][j] : a[p][j];
                a[i][j] = sw ? t : a[i][j];
            }
        }
        const double pinv = 1.0 / (best > 0.0 ? a[p][p] : 1.0);
        double rowp[MMAX], colp[MMAX];
#pragma unroll
        for (int j = 0; j < MMAX; ++j) rowp[j] = a[p][j] * pinv;
#pragma unroll
        for (int i = 0; i < MMAX; ++i) colp[i] = a[i][p];
#pragma unroll
        for (int i = 0; i < MMAX; ++i)
#pragma unroll
            for (int j = 0; j < MMAX; ++j) {
                if (i == p)
                    a[i][j] = (j == p) ? pinv : rowp[j];
                else
                    a[i][j] = (j == p) ? -colp[i] * pinv : a[i][j] - colp[i] * rowp[j];
            }
    }
#pragma unroll
    for (int p = MMAX - 1; p >= 0; --p) {
#pragma unroll
        for (int q = 0; q < MMAX; ++q) {
            const bool sw = (perm[p] == q) && (q != p);
#pragma unroll
            for (int i = 0; i < MMAX; ++i) {
                const double t = a[i][p];
                a[i][p] = sw ? a[i][q] : a[i][p];
                a[i][q] = sw ? t : a[i][q];
            }
        }
    }
    return ok;
}

// Write the leading m x m block of a (registers, identical on every lane) into
// tile layout (zero elsewhere), through slot s.
LQK_DEV Tile small_to_tile(const double a[MMAX][MMAX], int m, double *s)
{
    const int c = tcol();
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        double v = 0.0;
#pragma unroll
        for (int ii = 0; ii < MMAX; ++ii)
#pragma unroll
            for (int jj = 0; jj < MMAX; ++jj) v = (i == ii && c == jj && ii < m && jj < m) ? a[ii][jj] : v;
        t.v[r] = v;
    }
    (void)s;
    return t;
}

// Inverse of an m x m SPD block through Cholesky (every lane redundantly).
LQK_DEV bool spd_inverse(const Tile &W, int m, Tile &Winv, double *s)
{
    wsync();
    sput(s, W);
    wsync();
    double a[MMAX][MMAX];
    small_read(s, m, a);
    wsync();
    const bool ok = small_chol(a);
    small_tri_inv(a);  // a = L^{-1}
    double w[MMAX][MMAX];
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
            double v = 0.0;
#pragma unroll
            for (int p = 0; p < MMAX; ++p) v += a[p][i] * a[p][j];  // L^{-T} L^{-1}
            w[i][j] = v;
        }
    Winv = small_to_tile(w, m, s);
    return ok;
}

// Inverse of a general m x m block (every lane redundantly, pivoted).
LQK_DEV bool gen_inverse_small(const Tile &W, int m, Tile &Winv, double *s)
{
    wsync();
    sput(s, W);
    wsync();
    double a[MMAX][MMAX];
    small_read(s, m, a);
    wsync();
    const bool ok = small_gj_inv(a);
    Winv = small_to_tile(a, m, s);
    return ok;
}

// Lower Cholesky factor inverse L^{-1} of an m x m SPD block held in global
// memory (row-major, ld = m); every lane redundantly.  Returns false if not PD.
LQK_DEV bool chol_inv_global(const double *R, int m, double li[MMAX][MMAX])
{
#pragma unroll
    for (int i = 0; i < MMAX; ++i)
#pragma unroll
        for (int j = 0; j < MMAX; ++j) {
            // clamped indices keep every load in bounds and unconditional
            const int ii = i < m ? i : 0, jj = j < m ? j : 0;
            const double v = R[ii * m + jj];
            li[i][j] = (i < m && j < m) ? v : (i == j ? 1.0 : 0.0);
        }
    const bool ok = small_chol(li);
    small_tri_inv(li);
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

// Report the first failure of an instance: status = (-code) | (k << 8).
LQK_DEV void report(int32_t *status, int inst, int code, int k)
{
    if (status && lane() == 0) atomicCAS(&status[inst], 0, (int32_t)((-code) | (k << 8)));
}

}  // namespace lqk
