// lq_kernels.hpp -- kernels and host launchers shared by the host plan
// (lq_abi.hip) and the translation units that define them.  NK is the number
// of 4-wide contraction slices of an (n+1)-long product, ceil((n_max+1)/4).
#pragma once
#include "lq_desc.hpp"

namespace lqk {

void launch_build_elements(int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                           const int64_t *elem_start, int batch, double *elems, int32_t *status);
void launch_selftest_inv(hipStream_t st, const double *X, double *Xi, int n1, int homog, int32_t *ok);
void launch_selftest_mm(int pr, hipStream_t st, const double *X, const double *Y, const double *Z, double *D, int tx,
                        int ty);

void launch_value_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *elems, double *X, int prefix,
                       int32_t *status);
void launch_value_ks(int nk, int pr, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                     int batch, int dd, int prefix, const double *Xin, double *Xout, int32_t *status);
void launch_cv_start(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                     const int32_t *seg_start, int batch, const double *Xfin, double *Y, int32_t *status);
void launch_value_riccati(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                          const int32_t *seg_start, int batch, const double *Xfin, ValPtrs V, double *Yroll,
                          double *ckpt, int stride, int32_t *status);
void launch_value_recompute(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                            const int32_t *seg_start, int batch, int stride, const double *ckpt, ValPtrs V,
                            int32_t *status);
void launch_roll_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                      const int32_t *seg_start, int batch, double *Y);
void launch_affine_ks(int nk, int pr, int radix, unsigned grid, hipStream_t st, const InstDesc *inst, const int32_t *x_start, int batch,
                      int dd, int suffix, const double *Yin, double *Yout);
void launch_roll_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                       const int32_t *seg_start, int batch, const double *Yfin, double *x, double *u, double *lam);

void launch_adj_back_fold(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, const InstDesc *inst,
                          const int32_t *seg_start, int batch, double *Y);
void launch_adj_back_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, const InstDesc *inst,
                           const int32_t *seg_start, int batch, const double *Yfin, double *Yfwd, int32_t *status);
void launch_adj_fwd_apply(int nk, int pr, unsigned grid, hipStream_t st, ProbPtrs P, AdjPtrs J, GradPtrs Gr,
                          const InstDesc *inst, const int32_t *seg_start, int batch, const double *Yfin);

// Per-lane path for n <= 4 (lq_small.hip): one lane per segment or scan entry.
void launch_small_value_fold(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                             const int32_t *seg_start, int batch, double *X, int32_t *status);
void launch_small_value_ks(int n, int64_t total, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                           int batch, int dd, const double *Xin, double *Xout, int32_t *status);
// Every level of the per-lane value scan in one workgroup (the entries held in
// LDS); false, launching nothing, when the class has more scan entries than
// 512 at n <= 2, 352 at n = 3, 200 at n = 4 (LQSCAN_SCAN1=0: never).
bool launch_small_value_scan1(int n, int64_t total, hipStream_t st, const InstDesc *inst, const int32_t *x_start,
                              int batch, int max_nseg, double *X, int32_t *status);
// Every level of a per-lane affine-map scan in one workgroup, in place in Y;
// false, launching nothing, when the class has more than 512 scan entries
// (LQSCAN_SCAN1=0: never).
bool launch_small_affine_scan1(int n, int radix, int64_t total, hipStream_t st, const InstDesc *inst,
                               const int32_t *x_start, int batch, int max_nseg, int suffix, double *Y);
void launch_small_value_riccati(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, const InstDesc *inst,
                                const int32_t *seg_start, int batch, const double *Xfin, ValPtrs V, double *Yroll,
                                double *ckpt, int stride, int32_t *status);
void launch_small_affine_ks(int n, int radix, int64_t total, hipStream_t st, const InstDesc *inst,
                            const int32_t *x_start, int batch, int dd, int suffix, const double *Yin, double *Yout);
void launch_small_costate_fold(int n, int64_t total, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                               const int32_t *seg_start, int batch, double *Y);
void launch_small_costate_apply(int n, int64_t total, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                                const int32_t *seg_start, int batch, const double *Yfin);
void launch_small_roll_apply(int n, int m, int64_t total, hipStream_t st, ProbPtrs P, ValPtrs V, const InstDesc *inst,
                             const int32_t *seg_start, int batch, const double *Yfin, double *x, double *u,
                             double *lam);

void launch_nmpc_init(hipStream_t st, NmpcPtrs N, double *x, const double *u);
void launch_nmpc_shift(hipStream_t st, NmpcPtrs N, double *x0, double *u, double *uapp);
void launch_nmpc_linearise(int pr, hipStream_t st, NmpcPtrs N, NmpcWork Wk, const double *x, const double *u);
void launch_costate_fold(int nk, int pr, unsigned grid, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                         const int32_t *seg_start, int batch, double *Y);
void launch_costate_apply(int nk, int pr, unsigned grid, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                          const int32_t *seg_start, int batch, const double *Yfin);
void launch_nmpc_quadraticise(int pr, hipStream_t st, NmpcPtrs N, NmpcWork Wk, const double *x, const double *u,
                              const double *scal);
void launch_admm_update(hipStream_t st, NmpcPtrs N, const double *u, double *scal, int init);
void launch_nmpc_candidate(hipStream_t st, NmpcPtrs N, NmpcWork Wk, double *x, double *u, double *scal);

}  // namespace lqk
