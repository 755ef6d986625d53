/*
 * lqscan.h -- C ABI of the MI355X (gfx950) parallel-in-time LQ solver.
 *
 * The library solves the linear-quadratic subproblem that one Newton step of
 * the parallel-in-time method of Iacob, Abdulsamad and Saerkkae (arXiv
 * 2409.20027, Sec. III) reduces to, for one problem or a ragged batch:
 *
 *   min  sum_{k<T} [ 1/2 x_k'Q_k x_k + x_k'M_k u_k + 1/2 u_k'R_k u_k + q_k'x_k + r_k'u_k ]
 *        + 1/2 x_T'Q_T x_T + q_T'x_T
 *   s.t. x_{k+1} = A_k x_k + B_k u_k + c_k,   x_0 = x0.
 *
 * This is the problem eq:linearized-ocp with psi_t of eq:linearized-ocp-param
 * (paper index t = 1..N is k = t-1 here, N = T, P_t = Q_k, R_t + alpha I = R_k,
 * d_t = r_k), generalised by a dynamics offset c_k, a state-linear term q_k
 * and an initial state x0 so that configurations other than the paper's
 * (c = q = 0, x0 = 0) can be posed.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All numeric arrays are IEEE FP64, on the device, stage-major and packed
 *   back to back over the instances of the batch in instance order; matrices
 *   are row-major.  For instance i with sizes (n_i, m_i, T_i) the arrays hold
 *     A, Q: T_i*n_i*n_i   B, M: T_i*n_i*m_i   R: T_i*m_i*m_i
 *     c, q: T_i*n_i       r: T_i*m_i
 *     QT: n_i*n_i         qT, x0: n_i
 *     S: (T_i+1)*n_i*n_i  s, x, lambda: (T_i+1)*n_i
 *     Gamma: T_i*m_i*n_i  gamma, u: T_i*m_i
 *   Pointers documented as nullable may be NULL, meaning "all zero".
 * - The caller owns every buffer: problem data, outputs, the element buffer
 *   and the workspace.  The library never allocates, frees or synchronises
 *   inside a solve call, so every call may be captured into a HIP graph.
 *   Only lq_plan_create / lq_plan_destroy allocate (small descriptor tables).
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *   work is enqueued asynchronously on it.
 * - Argument errors are returned synchronously (LQ_ERR_ARG, LQ_ERR_UNSUPPORTED)
 *   before anything is enqueued.  Numerical failures are reported per
 *   instance through the device array `status` (int32, one per instance,
 *   nullable): 0 means success, otherwise
 *       status[i] = (-code) | (k << 8)
 *   with code one of LQ_ERR_NOT_PD / LQ_ERR_SINGULAR / LQ_ERR_NONFINITE and
 *   k the stage where it was detected (for the scan's operator: the first
 *   stage of the segment whose combination failed).  Of several failures the
 *   one with the largest status value, i.e. at the largest stage, is kept (a
 *   backward sweep over the stages meets it first), independently of the
 *   order in which the device work finishes; status must be zeroed by the
 *   caller before the first call that should report into it.  Results of a
 *   failed instance are unspecified; other instances are unaffected.
 * - Supported sizes: 1 <= n <= 15, 1 <= m <= 4, 1 <= T < 2^23.
 * - Calls that share a workspace must not run concurrently.
 */
#ifndef LQSCAN_H
#define LQSCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LQ_OK = 0,
    LQ_ERR_ARG = -1,          /* bad argument (NULL required pointer, size out of range) */
    LQ_ERR_NOT_PD = -2,       /* R_k or R_k + B'S_{k+1}B not positive definite            */
    LQ_ERR_SINGULAR = -3,     /* (I + C J) of the scan operator not invertible             */
    LQ_ERR_NONFINITE = -4,    /* NaN / Inf produced                                        */
    LQ_ERR_HIP = -5,          /* a HIP runtime call failed                                  */
    LQ_ERR_WORKSPACE = -6,    /* workspace / element buffer NULL or misaligned             */
    LQ_ERR_UNSUPPORTED = -7   /* sizes outside the supported range                         */
} lq_status;

typedef enum {
    LQ_FP64 = 0,   /* every product and factorisation in FP64                               */
    LQ_MIXED = 1   /* products in FP32; the (I + C J)^{-1} and Cholesky factorisations and
                      the symmetrisation of the value matrices in FP64                       */
} lq_precision;

/* Scan strategy of a plan. */
typedef enum {
    LQ_SCAN = 0,        /* segmented associative scan (default)                             */
    LQ_SEQUENTIAL = 1   /* one segment per instance: the plain sequential recursion         */
} lq_mode;

typedef struct lq_plan lq_plan;   /* opaque */

/*
 * Create a plan for a batch of `batch` instances with sizes nx[i], nu[i], T[i]
 * (host arrays).  `seg_len` is the number of stages folded per segment of the
 * scan (0 = choose automatically, ignored in LQ_SEQUENTIAL mode: T/16
 * clamped to 1..16, and at most 4 for the instances of a size class with
 * n <= 4, served by the per-lane kernels, when the class has fewer than 16384
 * stages in all).  Allocates small device descriptor tables on the current
 * device.
 * Errors: LQ_ERR_ARG, LQ_ERR_UNSUPPORTED (nx > 15, nu > 4, or T >= 2^23:
 * the status word (-code) | (k << 8) must stay a positive int32 for every
 * stage k <= T; with nx <= 15 this also keeps (T + 1) nx^2 below 2^31, the
 * 32-bit stage offsets inside one instance's arrays), LQ_ERR_HIP.
 */
lq_status lq_plan_create(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                         int32_t precision, int32_t mode, int32_t seg_len, lq_plan **out);
/*
 * Same with one segment length per instance (host array seg_len[batch]; 0 =
 * automatic, >= T[i] = the sequential recursion for that instance).  Used by
 * the segment-length autotuner, which picks a length per (n, m, T) class.
 */
lq_status lq_plan_create_seg(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                             int32_t precision, const int32_t *seg_len, lq_plan **out);
/*
 * Same with the segment lengths of an autotuner cache (the JSON file that
 * paper_2409_20027_amd/autotune.py writes): each instance takes the length
 * tuned for its class -- key "n<n>_m<m>_T<t>_B<b>_<fp64|mixed>" with t the
 * power of two at or above T[i] and b the one at or above the number of
 * instances of the batch in that (n, m, t) class -- where -1 means the
 * sequential recursion (one segment) and a class absent from the cache
 * gets the automatic length.  cache_path NULL: every length automatic.
 * Errors: LQ_ERR_ARG also for a file that cannot be read or an entry
 * without a readable "L"; otherwise those of lq_plan_create.
 */
lq_status lq_plan_create_tuned(int32_t batch, const int32_t *nx, const int32_t *nu, const int32_t *T,
                               int32_t precision, const char *cache_path, lq_plan **out);
void lq_plan_destroy(lq_plan *plan);

/* Bytes of scratch device memory the solve calls need (256-byte aligned base). */
size_t lq_plan_workspace_bytes(const lq_plan *plan);
/* Bytes of the element buffer written by lq_build_elements (256-byte aligned base). */
size_t lq_plan_elements_bytes(const lq_plan *plan);
/* Segment length the plan uses (the automatic choice if seg_len was 0). */
int32_t lq_plan_seg_len(const lq_plan *plan);
/* Total number of stages sum_i T_i. */
int64_t lq_plan_total_stages(const lq_plan *plan);

/* Device pointers to the problem data, packed as described above. */
typedef struct {
    const double *A, *B, *c;      /* c nullable                 */
    const double *Q, *R, *M;      /* M nullable                 */
    const double *q, *r;          /* nullable                   */
    const double *QT, *qT, *x0;   /* qT nullable                */
} lq_problem;

/* Value functions and affine control law (device pointers). */
typedef struct {
    double *S, *s;                /* V_k(x) = 1/2 x'S_k x + s_k'x + const, k = 0..T  */
    double *Gamma, *gamma;        /* u_k = Gamma_k x_k + gamma_k,          k = 0..T-1 */
} lq_value;

/*
 * lq_build_elements -- the value-function elements nu_t of
 * eq:value-fun-elem-init, one per stage plus the terminal element nu_{N+1}.
 * The stage element minimises the stage cost over u_k for a fixed pair
 * (x_k, x_{k+1}); in the form used here (which never inverts Q_k, unlike the
 * printed q_t, r_t) it is
 *   A_e = A - B R^{-1} M',  b = c - B R^{-1} r,  C = B R^{-1} B' = G G',
 *   J = Q - M R^{-1} M',    eta = -(q - M R^{-1} r),   G = B L^{-T}, R = L L'.
 * The terminal element is zero except J = Q_T, eta = -q_T.
 *
 * Element layout in `elements` (lq_plan_elements_bytes): instance i owns
 * T_i + 1 consecutive elements (stage k = 0..T_i-1, then the terminal).  An
 * element is 4 tiles of 16 x 16 doubles (8 KiB):
 *   tile 0  [[A_e, b], [0, 1]]        (homogeneous (n+1) x (n+1) map)
 *   tile 1  [[C, 0], [0, 0]]
 *   tile 2  [[J, -eta], [-eta', c0]]  (c0: constant term, -r'R^{-1}r)
 *   tile 3  [[G], [0]]                ((n+1) x m factor, C = G G')
 * zero-padded to 16 x 16, entry (i, j) of a tile stored at double offset
 *   4 * (j + 16 * (i % 4)) + (i / 4)
 * within the tile (the register layout of the FP64 16x16x4 matrix
 * instruction's accumulator, lane-major).  Numerical failure: LQ_ERR_NOT_PD if R_k is not positive
 * definite (status, stage k).
 */
lq_status lq_build_elements(const lq_plan *plan, const lq_problem *prob, double *elements,
                            int32_t *status, void *stream);

/*
 * lq_scan_solve -- value functions S_k, s_k (k = 0..T) and the control law of
 * eq:value-fun-feedback (Gamma, gamma) by the parallel value-function pass
 * (Alg. 2): the suffix products V_k = nu_k (x) ... (x) nu_{N+1} under the
 * operator eq:value-fun-param, with S_k = J(V_k), s_k = -eta(V_k).
 * The scan is segmented: each segment of seg_len stages is folded into one
 * element, the segment elements are scanned in log2 depth, and inside each
 * segment the suffix is completed from its right neighbour's value function
 * by the Bellman step (the operator applied to a stage element and a
 * terminal-type element).  The gain of eq:value-fun-feedback is read as
 *   Gamma = -(R + B'S'B)^{-1} (M' + B'S'A),  gamma = -(R + B'S'B)^{-1} (r + B'(S'c + s')).
 * S_k is symmetrised.  `elements` may be NULL: the element build is then
 * fused into the scan and nothing is materialised; otherwise it must hold the
 * output of lq_build_elements for the same problem.
 * Numerical failures: LQ_ERR_NOT_PD (R_k + B'S_{k+1}B not positive definite;
 * with cross terms M or r also R_k, whose inverse forms the Schur complement),
 * LQ_ERR_SINGULAR.  Without cross terms R_k itself is never factorised: it
 * enters the fused fold only through W = R_k + B'J B (J the aggregate's value
 * matrix), so an indefinite R_k is accepted wherever R_k + B'S_{k+1}B is
 * positive definite.  R_k must still be invertible (the stage element's
 * C = B R_k^{-1} B' needs it): a singular R_k can make W singular
 * (LQ_ERR_SINGULAR at that stage).
 */
lq_status lq_scan_solve(const lq_plan *plan, const lq_problem *prob, const double *elements,
                        const lq_value *out, void *workspace, int32_t *status, void *stream);

/*
 * lq_rollout -- state propagation pass (Alg. 3): the closed-loop maps
 *   x_{k+1} = (A + B Gamma) x_k + (B gamma + c)
 * composed by a prefix scan (eq:state-prop-comb-rule; the first element
 * carries x0 as in eq:state-prop-init-elem-init), then u_k = Gamma x_k + gamma
 * and the co-states lambda_k = S_k x_k + s_k.
 * Outputs x ((T+1) n), u (T m), lambda ((T+1) n, nullable).  The pass is
 * products and sums only, so it has no numerical failure: status is not
 * written (it is kept for a signature uniform with the other solve calls).
 */
lq_status lq_rollout(const lq_plan *plan, const lq_problem *prob, const lq_value *val,
                     double *x, double *u, double *lambda, void *workspace, int32_t *status,
                     void *stream);

/*
 * lq_rollout_cv -- the same outputs as lq_rollout from the conditional value
 * functions instead of the closed-loop maps (eq:value-fun-prefix-sum): with
 * the prefix element V(x_0, x_k) = nu_0 (x) ... (x) nu_{k-1} of eq:value-fun-def
 * (dual form eq:value-fun-elements, parameters A, b, C) and the value function
 * (S_k, s_k) of val, the optimal state minimises V(x_0, x_k) + V_k(x_k):
 *   (I + C S_k) x_k = A x_0 + b - C s_k.
 * Segmented: the prefix elements are formed at the segment starts (fold of
 * each segment with the fused element build, then a log-depth prefix scan
 * under eq:value-fun-param), the formula gives the segment-start states, and
 * inside each segment the states follow the closed-loop recursion
 * x_{k+1} = (A + B Gamma) x_k + B gamma + c (the formula with the one-stage
 * prefix), u_k = Gamma x_k + gamma, lambda_k = S_k x_k + s_k.
 * Arguments, layouts and ownership are those of lq_rollout; val must hold the
 * lq_scan_solve (or lq_solve) output for the same problem.  The workspace's
 * scan buffers are overwritten.  Numerical failures: LQ_ERR_NOT_PD (R_k not
 * positive definite where cross terms need its inverse), LQ_ERR_SINGULAR (a
 * singular I + C S_k or fold matrix).
 */
lq_status lq_rollout_cv(const lq_plan *plan, const lq_problem *prob, const lq_value *val,
                        double *x, double *u, double *lambda, void *workspace, int32_t *status,
                        void *stream);

/* Gradients (device pointers, same packing as lq_problem; NULL = not wanted). */
typedef struct {
    double *A, *B, *c, *Q, *R, *M, *q, *r, *QT, *qT, *x0;
} lq_grads;

/*
 * lq_solve -- lq_scan_solve followed by lq_rollout, as one call: the same
 * value pass and state propagation (Alg. 2 then Alg. 3), with the rollout's
 * segment fold done inside the value pass's Bellman sweep, where the gains
 * Gamma_k, gamma_k are formed (the closed-loop map F_k = A_k + B_k Gamma_k of
 * eq:state-prop-comb-rule needs nothing else), so the stage data is read once
 * less.  Arguments, layouts, ownership and errors are those of lq_scan_solve
 * (elements, out) and lq_rollout (x, u, lambda); the results are the same up to
 * rounding order.
 */
lq_status lq_solve(const lq_plan *plan, const lq_problem *prob, const double *elements, const lq_value *out,
                   double *x, double *u, double *lambda, void *workspace, int32_t *status, void *stream);

/*
 * lq_solve_static -- lq_solve for callers that cannot allocate device memory
 * (code under HIP graph capture that must not see an allocation, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with the scan buffers in a scratch array that the library holds
 * in device memory (LQ_STATIC_SCRATCH_BYTES per GPU, for the life of the
 * process) instead of a caller workspace.  The call allocates nothing and
 * makes no allocating library call; its first call on a device looks up that
 * device's copy of the array (once per device).
 * Arguments, layouts, ownership and numerical failures are those of lq_solve
 * without `workspace`.  Errors: those of lq_solve, and LQ_ERR_WORKSPACE
 * (synchronously, nothing enqueued) if the plan's scan buffers exceed
 * LQ_STATIC_SCRATCH_BYTES (lq_plan_static_bytes tells what a plan needs), or
 * LQ_ERR_HIP if the array's address cannot be found.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap in time on one GPU (concurrent streams, host
 * threads) race and must be serialised by the caller.  The solve reads no
 * scratch entry before writing it, so nothing needs clearing between calls.
 */
#define LQ_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
size_t lq_plan_static_bytes(const lq_plan *plan);
lq_status lq_solve_static(const lq_plan *plan, const lq_problem *prob, const double *elements, const lq_value *out,
                          double *x, double *u, double *lambda, int32_t *status, void *stream);

/*
 * lq_adjoint -- reverse-mode derivative of the LQ solution (not in the
 * paper; implicit differentiation of the KKT system).  Given the loss
 * gradients gx = dL/dx_k (k = 0..T, (T+1) n) and gu = dL/du_k (T m), the
 * adjoint is the same LQ with linear terms (gx, gu), c = 0 and x0 = 0; it
 * reuses S and Gamma: a suffix scan of the affine maps
 *   s~_k = gx_k + Gamma'gu_k + (A + B Gamma)' s~_{k+1},   s~_T = gx_T,
 * then gamma~_k = -(R + B'S_{k+1}B)^{-1}(gu_k + B's~_{k+1}), a prefix scan of
 *   dx_{k+1} = (A + B Gamma) dx_k + B gamma~_k,  dx_0 = 0,
 * du = Gamma dx + gamma~, dlam = S dx + s~, and per-stage outer products
 *   dL/dA_k = lam_{k+1} dx_k' + dlam_{k+1} x_k'    dL/dB_k = lam_{k+1} du_k' + dlam_{k+1} u_k'
 *   dL/dc_k = dlam_{k+1}                           dL/dx0 = dlam_0
 *   dL/dQ_k = sym(dx_k x_k')   dL/dR_k = sym(du_k u_k')   dL/dM_k = dx_k u_k' + x_k du_k'
 *   dL/dq_k = dx_k   dL/dr_k = du_k   dL/dQ_T = sym(dx_T x_T')   dL/dq_T = dx_T.
 * Inputs: the forward solution val (S, s, Gamma, gamma), x, u, lambda.
 * val may be NULL: the value functions are then recomputed by rerunning the
 * value pass from the problem data, exactly as lq_adjoint_ckpt with
 * ckpt == NULL, and the workspace must hold
 * lq_plan_adjoint_ckpt_workspace_bytes (LQ_ERR_WORKSPACE if NULL or
 * misaligned).
 */
lq_status lq_adjoint(const lq_plan *plan, const lq_problem *prob, const lq_value *val,
                     const double *x, const double *u, const double *lambda,
                     const double *gx, const double *gu, const lq_grads *grads,
                     void *workspace, int32_t *status, void *stream);

/*
 * Level checkpointing of the differentiated solve (not in the paper): the
 * forward keeps only the scan's segment carries, and the adjoint recomputes
 * S_k, s_k, Gamma_k, gamma_k from them instead of reading them back, so that
 * between forward and backward a caller holds one (n+1) x (n+1) carry per
 * `stride` segments instead of the (T+1) n^2 + T m n + ... value arrays.
 *
 * The checkpoint of a plan for a stride (>= 1) is lq_plan_checkpoint_bytes
 * of device memory (caller-owned, 256-byte aligned): one 16 x 16-double slot
 * per group of `stride` consecutive segments of an instance, holding the
 * value function S~ = [[S, s], [s', const]] at the group's right end (the
 * terminal element for the instance's last group) as an (n+1) x (n+1)
 * row-major block at the start of the slot; instance i's first slot is
 * seg0_i / stride + i (seg0_i: the instance's first segment in the plan).
 *
 * lq_solve_ckpt -- lq_solve that also writes the checkpoint for `stride`.
 * Arguments, layouts, ownership and errors are those of lq_solve, plus
 * LQ_ERR_ARG for stride < 1 and LQ_ERR_WORKSPACE for a NULL or misaligned
 * ckpt.  The value outputs `out` are still written (the rollout's co-states
 * need S_k and s_k); a caller that differentiates later may release them once
 * the call has completed and keep only ckpt, x, u and lambda.
 *
 * lq_adjoint_ckpt -- lq_adjoint without the value functions: with ckpt
 * (written by lq_solve_ckpt for the same problem, plan and stride) one wave
 * per group reruns the Bellman steps of eq:value-fun-param (with the gain of
 * eq:value-fun-feedback) from the group's carry, right to left over its
 * stride * seg_len stages; with ckpt == NULL the whole value pass (Alg. 2)
 * is rerun from the problem data (nothing kept from the forward but x, u,
 * lambda).  The recomputed S, s, Gamma, gamma go to the workspace, which
 * must hold lq_plan_adjoint_ckpt_workspace_bytes (more than
 * lq_plan_workspace_bytes); the rest is lq_adjoint.  With stride 1 the
 * recomputed arrays equal the forward's bit for bit; larger strides trade
 * checkpoint memory (about 1/stride) for a longer sequential sweep per wave,
 * and agree with the forward up to rounding order.  Numerical failures are
 * those of the forward's Bellman steps (LQ_ERR_NOT_PD, LQ_ERR_NONFINITE), then
 * of lq_adjoint.
 */
size_t lq_plan_checkpoint_bytes(const lq_plan *plan, int32_t stride);
size_t lq_plan_adjoint_ckpt_workspace_bytes(const lq_plan *plan);
lq_status lq_solve_ckpt(const lq_plan *plan, const lq_problem *prob, const double *elements, const lq_value *out,
                        double *x, double *u, double *lambda, double *ckpt, int32_t stride, void *workspace,
                        int32_t *status, void *stream);
lq_status lq_adjoint_ckpt(const lq_plan *plan, const lq_problem *prob, const double *ckpt, int32_t stride,
                          const double *x, const double *u, const double *lambda,
                          const double *gx, const double *gu, const lq_grads *grads,
                          void *workspace, int32_t *status, void *stream);

/*
 * ---------------------------------------------------------------------------
 * Newton / interior-point step (Alg. 4 inside the log-barrier method of
 * Sec. II-B) for x_{k+1} = x_k + h f(x_k, u_k) (one explicit Euler step) with
 * l_k = 1/2 (x - ref_k)'Q(x - ref_k) + 1/2 u'R u, l_T = 1/2 (x - ref_T)'Q_T(x - ref_T),
 * and the control box umin < u < umax as 2 nu inequalities with the barrier
 * -mu sum [log(umax - u) + log(u - umin)].  Models f:
 *   NMPC_TANH      f = tanh(W x) + B u (any nx <= 15, nu <= 4);
 *   NMPC_PENDULUM  the torque-limited pendulum of Sec. V, nx = 2, nu = 1,
 *                  x = (theta, omega), param = (g, l, m, b);
 *   NMPC_CARTPOLE  the force-limited cart-pole of Sec. V, nx = 4, nu = 1,
 *                  x = (p, theta, v, omega), param = (g, l, m_c, m_p), with
 *                  omega^2 in the cart acceleration (textbook cart-pole).
 * For the pendulum and cart-pole the second derivatives of f enter P, the
 * cross term M and R of the expansion (eq:linearized-ocp-param).
 * ---------------------------------------------------------------------------
 */
typedef enum { NMPC_TANH = 0, NMPC_PENDULUM = 1, NMPC_CARTPOLE = 2 } nmpc_model;

/* A plan with batch B >= 1 instances, all of sizes (nx, nu, T), solves B
 * problems at once that share the model, costs, bounds and reference and
 * differ in x0 ([B][nx]) and their trajectories: nmpc_state.x is
 * [B][(T+1) nx], u [B][T nu], scal [B][NMPC_NSCAL], admm_z / admm_v
 * [B][T][2 nu]; every decision is taken per instance. */
typedef struct {
    int32_t nx, nu, T;
    double h;
    const double *W, *Bm;          /* nx*nx, nx*nu (device; NMPC_TANH only, else ignored) */
    const double *Q, *R, *QT;      /* nx*nx, nu*nu, nx*nx             (device) */
    const double *xref, *x0;       /* (T+1)*nx, batch*nx              (device) */
    double umin, umax;
    int32_t model;                 /* nmpc_model                                */
    double param[4];               /* model constants (host values)             */
    /* ADMM (Sec. II-C): with admm_rho > 0 the augmentation
     * admm_rho/2 |h(u_k) - z_k + v_k/admm_rho|^2, h(u) = [u - umax; umin - u],
     * replaces the barrier (mu is then unused and u may leave the box).
     * admm_z, admm_v: T*2*nu device arrays, rows u - umax then umin - u per
     * stage, written by nmpc_admm_update.  admm_rho is the weight of each
     * stage's term (fold any time step into it). */
    double admm_rho;
    double *admm_z, *admm_v;
} nmpc_problem;

/* Indices of the device scalar array nmpc_state.scal (NMPC_NSCAL doubles). */
enum {
    NMPC_MU = 0,          /* barrier weight (set by the caller)                      */
    NMPC_ALPHA = 1,       /* Levenberg-Marquardt weight alpha (updated by the step)   */
    NMPC_NU = 2,          /* growth factor of alpha after a rejection                 */
    NMPC_COST = 3,        /* J_mu of the nominal after the step                       */
    NMPC_PRED = 4,        /* predicted decrease of the step                           */
    NMPC_RHO = 5,         /* gain ratio (-inf if rejected before it could be formed)  */
    NMPC_ACCEPTED = 6,    /* 1.0 if the step was accepted                             */
    NMPC_COST_NEW = 7,    /* J_mu of the candidate                                    */
    NMPC_GRAD = 8,        /* |dJ_mu/du|_inf at the nominal the step started from      */
    NMPC_RP = 9,          /* ADMM primal residual |h(u) - z|_inf (nmpc_admm_update)   */
    NMPC_RD = 10,         /* ADMM dual residual |z - z_prev|_inf (nmpc_admm_update)   */
    /* Barrier levels ended on the device, so that a caller can enqueue several
     * newton_step calls (or replay a graph of them) between read-backs: with
     * LEVEL_TOL > 0 each step counts the level's iterations in LEVEL_ITERS and,
     * after the iteration that starts from |dJ_mu/du|_inf <= LEVEL_TOL or that
     * reaches LEVEL_MAX iterations, sets LEVEL_DONE to 0.5; the next step turns
     * it to 1 and, while it is 1, newton_step leaves the instance unchanged.
     * The caller sets LEVEL_TOL and LEVEL_MAX and zeroes LEVEL_ITERS and
     * LEVEL_DONE when it starts a level.  LEVEL_TOL <= 0: no level control. */
    NMPC_LEVEL_TOL = 11,
    NMPC_LEVEL_MAX = 12,
    NMPC_LEVEL_ITERS = 13,
    NMPC_LEVEL_DONE = 14,
    NMPC_NSCAL = 15
};

typedef struct {
    double *x, *u;   /* nominal trajectory (T+1)*nx and T*nu (device), replaced on acceptance */
    double *scal;    /* NMPC_NSCAL device scalars                                             */
} nmpc_state;

/* Workspace of newton_step / nmpc_init for a plan whose instances all have
 * the problem's (nx, nu, T) (the plan's segment length is used by every scan). */
size_t nmpc_workspace_bytes(const lq_plan *plan);

/* x <- nonlinear rollout of u from x0 (call once before the first step). */
lq_status nmpc_init(const lq_plan *plan, const nmpc_problem *prob, const nmpc_state *state, void *workspace,
                    void *stream);

/*
 * One Newton iteration at the barrier weight scal[NMPC_MU]:
 * linearisation and co-states (parallel co-state pass, Alg. 1), second-order
 * expansion, the LQ step (lq_scan_solve + lq_rollout, value pass and state
 * propagation of Alg. 2-3), the nonlinear rollout of u + du and the
 * acceptance test with the damping update (see lq_newton.hip): the nominal is
 * replaced by (rollout(u + du), u + du) if the gain ratio is positive.  A
 * rejected step (including an LQ step whose R + B'S'B is not positive
 * definite) leaves the nominal unchanged and increases alpha.  Everything is
 * enqueued on `stream`; decisions are taken on the device.  `status` is not
 * written (rejections are part of the method).  Errors: LQ_ERR_ARG if the
 * plan does not match the problem or the model its sizes.
 */
lq_status newton_step(const lq_plan *plan, const nmpc_problem *prob, const nmpc_state *state, void *workspace,
                      int32_t *status, void *stream);

/*
 * ADMM consensus and multiplier steps (eq:admm-step-4 and eq:admm-step-5 of
 * Sec. II-C) for the control box, from the nominal controls state->u, with
 * w = h(u) = [u - umax; umin - u] per stage and C = {w <= 0}:
 *   init != 0:  z = min(0, w), v = 0 (the start of the ADMM loop);
 *   init == 0:  z <- min(0, w + v/rho), v <- v + rho (w - z), and
 *               scal[NMPC_RP] = |w - z|_inf, scal[NMPC_RD] = |z - z_prev|_inf.
 * One block on `stream`.  Errors: LQ_ERR_ARG if the plan does not match the
 * problem or prob->admm_rho <= 0 or admm_z / admm_v is null.
 */
lq_status nmpc_admm_update(const lq_plan *plan, const nmpc_problem *prob, const nmpc_state *state, int32_t init,
                           void *stream);

/*
 * Receding horizon (Sec. V, model predictive control): for every instance the
 * plant takes one step with the first control, x0 <- x0 + h f(x0, u_0) (x0 is
 * the device array prob->x0 points to, updated in place; u_0 is written to
 * u_applied [batch][nu]), and state->u shifts by one stage for the next
 * solve's warm start (the last control is kept).  Call nmpc_init before the
 * next solve's first newton_step (it re-rolls the nominal from the new x0).
 * Errors: LQ_ERR_ARG if the plan does not match the problem or a pointer is
 * null.
 */
lq_status nmpc_shift(const lq_plan *plan, const nmpc_problem *prob, const nmpc_state *state, double *x0,
                     double *u_applied, void *stream);

/*
 * Diagnostic: one 16 x 16 tile product D = op(X) op(Y) (+ Z) through the
 * library's matrix-core tile primitive (P'Q of register tiles, with the LDS
 * transpose the solver uses where op needs it), with FP64 products (precision
 * LQ_FP64) or FP32 products added to Z in FP64 (LQ_MIXED).  X, Y, Z, D are
 * device pointers to row-major 16 x 16 FP64 arrays (Z nullable).  Used by the
 * test suite to pin the operand and accumulator layouts of the matrix
 * instructions.
 */
lq_status lq_selftest_tile_mm(const double *X, const double *Y, const double *Z, double *D,
                              int32_t transpose_x, int32_t transpose_y, int32_t precision, void *stream);

/*
 * Diagnostic: the solver's register Gauss-Jordan inverse (partial pivoting)
 * of the leading n1 x n1 block of X (1 <= n1 <= 16).  homog != 0 declares X
 * of the form [[M, 0], [r, 1]] (last column e_{n1-1}; n1 >= 2), as the value
 * operator's I + J~C~; pivots are then taken among the first n1 - 1 rows.  X
 * and Xinv are device pointers to row-major 16 x 16 FP64 arrays (entries
 * outside the block are ignored; on success Xinv is zero there); *ok (device
 * int32) receives 1, or 0 for a zero or non-finite pivot.  Used by the test
 * suite to pin the pivot search.
 */
lq_status lq_selftest_tile_inverse(const double *X, double *Xinv, int32_t n1, int32_t homog, int32_t *ok,
                                   void *stream);

/*
 * Diagnostic phase timing.  Phases of the solve calls, in enqueue order (a
 * phase is one kernel launch, except the scans: one launch per level):
 */
enum {
    LQ_PH_BUILD = 0,         /* lq_build_elements                                  */
    LQ_PH_VALUE_FOLD = 1,    /* value pass: fold of each segment (fused element build) */
    LQ_PH_VALUE_SCAN = 2,    /* value pass: log-depth scan of the segment elements  */
    LQ_PH_VALUE_BELLMAN = 3, /* value pass: Bellman steps inside segments + control law */
    LQ_PH_ROLL_FOLD = 4,     /* rollout: composition of each segment's maps         */
    LQ_PH_ROLL_SCAN = 5,     /* rollout: log-depth prefix scan                      */
    LQ_PH_ROLL_APPLY = 6,    /* rollout: states, controls, co-states                */
    LQ_PH_ADJ_BACK_FOLD = 7,  /* adjoint: composition of each segment's backward maps */
    LQ_PH_ADJ_BACK_SCAN = 8,  /* adjoint: log-depth suffix scan                      */
    LQ_PH_ADJ_BACK_APPLY = 9, /* adjoint: s~ and gamma~ inside segments              */
    LQ_PH_ADJ_FWD_FOLD = 10,  /* adjoint: composition of each segment's forward maps  */
    LQ_PH_ADJ_FWD_SCAN = 11,  /* adjoint: log-depth prefix scan                      */
    LQ_PH_ADJ_FWD_APPLY = 12, /* adjoint: dx, du, dlambda and the gradients          */
    LQ_PH_CV_FOLD = 13,       /* conditional-value rollout: fold of each segment    */
    LQ_PH_CV_SCAN = 14,       /* conditional-value rollout: log-depth prefix scan   */
    LQ_PH_CV_START = 15,      /* conditional-value rollout: segment-start states    */
    LQ_PH_ADJ_RECOMPUTE = 16, /* checkpointed adjoint: S, Gamma from the checkpoint  */
    LQ_NPHASE = 17
};
/*
 * lq_plan_set_timing enables event recording around the phases whose bit is
 * set in `mask` (bit p = phase p; 0 disables) for at most `capacity` phase
 * launches; it creates the HIP events (this call may allocate).  While
 * enabled, each solve call records a start and a stop event on its own stream
 * around every selected phase.  lq_plan_phase_times waits for the recorded
 * events, writes the summed milliseconds and the number of recorded launches
 * per phase (arrays of LQ_NPHASE, either nullable) and resets the counters.
 * Not for use inside HIP graph capture.
 */
lq_status lq_plan_set_timing(lq_plan *plan, uint32_t mask, int32_t capacity);
lq_status lq_plan_phase_times(lq_plan *plan, double *ms, int64_t *count);

/* Library version string. */
const char *lq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LQSCAN_H */
