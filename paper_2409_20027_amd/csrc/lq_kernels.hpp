// lq_kernels.hpp -- kernel declarations shared by the host plan (lq_abi.hip)
// and the translation units that define them.
#pragma once
#include "lq_desc.hpp"

namespace lqk {

__global__ void k_build_elements(ProbPtrs P, const InstDesc *inst, const int64_t *elem_start, int batch,
                                 double *elems, int32_t *status);
__global__ void k_value_fold(ProbPtrs P, const InstDesc *inst, const int32_t *seg_start, int batch,
                             const double *elems, double *X, int32_t *status);
__global__ void k_value_terminal(ProbPtrs P, const InstDesc *inst, double *X);
__global__ void k_value_ks(const InstDesc *inst, const int32_t *x_start, int batch, int dd,
                           const double *Xin, double *Xout, int32_t *status);
__global__ void k_value_riccati(ProbPtrs P, const InstDesc *inst, const int32_t *seg_start, int batch,
                                const double *Xfin, ValPtrs V, int32_t *status);
__global__ void k_selftest_mm(const double *X, const double *Y, const double *Z, double *D, int tx, int ty);

__global__ void k_roll_fold(ProbPtrs P, ValPtrs V, const InstDesc *inst, const int32_t *seg_start, int batch,
                            double *Y);
__global__ void k_affine_ks(const InstDesc *inst, const int32_t *x_start, int batch, int dd, int suffix,
                            const double *Yin, double *Yout);
__global__ void k_roll_apply(ProbPtrs P, ValPtrs V, const InstDesc *inst, const int32_t *seg_start, int batch,
                             const double *Yfin, double *x, double *u, double *lam);
__global__ void k_roll_init(ProbPtrs P, const InstDesc *inst, double *Y);

}  // namespace lqk
