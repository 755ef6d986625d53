// lq_newton.hip -- one iteration of the parallel-in-time Newton method (Alg. 4)
// inside the primal log-barrier method (Sec. II-B), for the dynamics
//   x_{k+1} = x_k + h f(x_k, u_k),
// f = tanh(W x) + B u (synthetic network) or the pendulum / cart-pole of
// Sec. V (lq_models.hpp; their derivatives by forward-mode jets),
// tracking costs l_k = 1/2 (x - ref_k)'Q(x - ref_k) + 1/2 u'R u,
// l_T = 1/2 (x - ref_T)'Q_T(x - ref_T), and the box |u| bounds written as
// 2 nu inequalities u - umax <= 0, umin - u <= 0 with the barrier
//   c(u) = -mu sum_i [log(umax - u_i) + log(u_i - umin)].
//
// Steps (all enqueued on the caller's stream, decisions taken on the device):
//   1. k_nmpc_linearise      A_k = I + h df/dx, B_k = h df/du (tanh model:
//                            df/dx = diag(1 - tanh^2 z) W, z = W x_k), g_k = Q (x_k - ref_k);
//                            its stage-0 lane also clears the step's LQ status
//                            and zero initial state and copies Q_T
//   2. co-state suffix scan  lambda_T = Q_T(x_T - ref_T),
//                            lambda_k = g_k + A_k' lambda_{k+1}   (eq:co-state-eq;
//                            homogeneous maps [[A_k', g_k], [0, 1]], Alg. 1)
//   3. k_nmpc_quadraticise   P_k = Q + h lambda_{k+1}' d2f/dx2, M_k = h lambda_{k+1}' d2f/dxdu,
//                            R~_k = R + d2c/du2 + h lambda_{k+1}' d2f/du2 + alpha I,
//                            d_k = R u + dc/du + B_k' lambda_{k+1}
//                            (tanh model: lambda' d2f/dx2 = sum_i lambda_i tanh''(z_i) w_i w_i',
//                            no mixed or control second derivatives)
//   4. the LQ step           eq:linearized-ocp with psi_t of eq:linearized-ocp-param
//                            (delta x_0 = 0) by lq_scan_solve + lq_rollout
//   5. k_nmpc_rollout        candidate u + du and its nonlinear rollout (sequential
//                            in k on one wave, controls staged through LDS)
//   6. k_nmpc_reduce         predicted decrease of the expansion (without alpha),
//                            |d|_inf, J_mu of the nominal and of the candidate
//                            (block reductions), gain ratio rho = (J_mu(u) -
//                            J_mu(u + du)) / pred; accept if pred > 0 and rho > 0:
//                            alpha *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; else
//                            alpha *= nu, nu *= 2; on acceptance the candidate
//                            then replaces the nominal (the same block, after
//                            the decision).
#include <algorithm>
#include <cfloat>
#include <cstdlib>

#include "lq_kernels.hpp"
#include "lq_models.hpp"

namespace lqk {

// Largest state and control dimensions of the Newton kernels' per-lane arrays.
constexpr int NXMAX = 15;
constexpr int NUMAX = MMAX;

// Nonlinear step x' = x + h f(x, u).
LQK_DEV void f_step(const NmpcPtrs &N, int n, int m, const double *x, const double *u, double *xn)
{
    if (N.model == MODEL_TANH) {
        for (int i = 0; i < n; ++i) {
            double z = 0.0, bu = 0.0;
            for (int j = 0; j < n; ++j) z += N.W[i * n + j] * x[j];
            for (int j = 0; j < m; ++j) bu += N.Bm[i * m + j] * u[j];
            xn[i] = x[i] + N.h * (tanh_em1(z) + bu);
        }
    } else if (N.model == MODEL_PENDULUM) {
        const double z[3] = {x[0], x[1], u[0]};
        double f[2];
        pendulum_f<double, double>(N.prm, z, f);
        for (int i = 0; i < 2; ++i) xn[i] = x[i] + N.h * f[i];
    } else {
        const double z[5] = {x[0], x[1], x[2], x[3], u[0]};
        double f[4];
        cartpole_f<double, double>(N.prm, z, f);
        for (int i = 0; i < 4; ++i) xn[i] = x[i] + N.h * f[i];
    }
}

// Jets of f at z = (x_k, u_k) for the pendulum (NZ = 3) or cart-pole (NZ = 5).
template <int NZ, typename RT>
LQK_DEV void model_jets(const NmpcPtrs &N, const double *xk, const double *uk, Jet<NZ, RT> *f)
{
    constexpr int n = NZ - 1;
    Jet<NZ, RT> z[NZ];
#pragma unroll
    for (int i = 0; i < n; ++i) z[i] = jvar<NZ, RT>((RT)xk[i], i);
    z[n] = jvar<NZ, RT>((RT)uk[0], n);
    RT prm[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) prm[i] = (RT)N.prm[i];
    if constexpr (NZ == 3)
        pendulum_f<Jet<NZ, RT>, RT>(prm, z, f);
    else
        cartpole_f<Jet<NZ, RT>, RT>(prm, z, f);
}

// A_k = I + h df/dx, B_k = h df/du from the jets (pendulum / cart-pole);
// gk = instance * T + stage indexes the packed workspace.
template <int NZ>
LQK_DEV void linearise_model(const NmpcPtrs &N, const NmpcWork &Wk, int64_t gk, const double *xk, const double *uk)
{
    constexpr int n = NZ - 1;
    Jet<NZ, double> f[n];
    model_jets<NZ, double>(N, xk, uk, f);
    double *A = Wk.A + gk * n * n, *B = Wk.B + gk * n;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) A[i * n + j] = (i == j ? 1.0 : 0.0) + N.h * f[i].g[j];
        B[i] = N.h * f[i].g[n];
    }
}

// P_k = Q + h S_xx, M_k = h S_xu and h S_uu (added to R~ and Rh) of
// S = lambda_{k+1}' f, in arithmetic type RT.
template <int NZ, typename RT>
LQK_DEV RT quadraticise_model(const NmpcPtrs &N, const NmpcWork &Wk, int64_t gk, const double *xk, const double *uk,
                              const double *l1)
{
    constexpr int n = NZ - 1;
    Jet<NZ, RT> f[n];
    model_jets<NZ, RT>(N, xk, uk, f);
    Jet<NZ, RT> S = (RT)l1[0] * f[0];
    for (int i = 1; i < n; ++i) S = S + (RT)l1[i] * f[i];
    const RT h = (RT)N.h;
    double *P = Wk.P + gk * n * n, *M = Wk.M + gk * n;
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) P[a * n + b] = (double)((RT)N.Q[a * n + b] + h * S.H[a][b]);
        M[a] = (double)(h * S.H[a][n]);
    }
    return h * S.H[n][n];
}

// ADMM residual of global stage gk (instance * T + stage), input i:
// (a, b) = h(u) - z + v / rho for the rows u_i - umax <= 0 and umin - u_i <= 0.
LQK_DEV void admm_ab(const NmpcPtrs &N, int64_t gk, int i, double ui, double &a, double &b)
{
    const int m = N.nu;
    const double *zk = N.z + gk * 2 * m, *vk = N.v + gk * 2 * m;
    a = (ui - N.umax) - zk[i] + vk[i] / N.rho;
    b = (N.umin - ui) - zk[m + i] + vk[m + i] / N.rho;
}

// Stage cost plus the barrier (+inf if u is infeasible), or plus the ADMM
// augmentation when N.rho > 0; k is the stage (reference row), gk the global
// stage of the instance.
LQK_DEV double stage_cost(const NmpcPtrs &N, int n, int m, int k, int64_t gk, const double *xk, const double *uk,
                          double mu)
{
    const double *rk = N.xref + (int64_t)k * n;
    double J = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) J += 0.5 * (xk[i] - rk[i]) * N.Q[i * n + j] * (xk[j] - rk[j]);
    for (int i = 0; i < m; ++i) {
        for (int j = 0; j < m; ++j) J += 0.5 * uk[i] * N.R[i * m + j] * uk[j];
        if (N.rho > 0.0) {
            double a, b;
            admm_ab(N, gk, i, uk[i], a, b);
            J += 0.5 * N.rho * (a * a + b * b);
            continue;
        }
        const double a = N.umax - uk[i], b = uk[i] - N.umin;
        if (!(a > 0.0 && b > 0.0)) return INFINITY;
        J += -mu * (log(a) + log(b));
    }
    return J;
}

LQK_DEV double terminal_cost(const NmpcPtrs &N, int n, int T, const double *xT)
{
    const double *rT = N.xref + (int64_t)T * n;
    double J = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) J += 0.5 * (xT[i] - rT[i]) * N.QT[i * n + j] * (xT[j] - rT[j]);
    return J;
}

// The nonlinear rollouts below are sequential in time.  Each block has four
// waves: wave 0 runs the recursion reading the controls from LDS, while waves
// 1-3 stage the next chunk of controls u + du (du may be null) into the other
// of two LDS buffers (and write the sums to uout), so no step of the recursion
// waits for a global load, and the only wait on memory is the barrier
// between chunks.
// A chunk is ROLL_SLOTS doubles: R rows (instances) of 2^lg slots each.
constexpr int ROLL_THREADS = 256;
constexpr int ROLL_SLOTS = 4096;

// Stage one chunk: row r (instance inst0 + r, skipped unless bit r of `act`
// is set) copies cnt doubles from global offset (inst0 + r) * rstride + g0
// into LDS at r * (2^lg + 1) (the padding keeps lanes reading different rows
// at the same slot in different banks).  Threads tp = 0 .. np-1 take part;
// each issues U loads before it stores the first value.
template <bool DU>
LQK_DEV void stage_controls(double *__restrict__ buf, int lg, int cnt, uint64_t act, int64_t inst0, int64_t rstride,
                            int64_t g0, const double *__restrict__ u, const double *__restrict__ du,
                            double *__restrict__ uout, int tp, int np)
{
    constexpr int U = 8;
    const int cap = 1 << lg;
    for (int base = tp; base < ROLL_SLOTS; base += np * U) {
        double v[U];
        int64_t o[U];
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int idx = base + j * np;
            const int r = idx >> lg, k = idx & (cap - 1);
            ok[j] = idx < ROLL_SLOTS && k < cnt && ((act >> r) & 1);
            o[j] = (inst0 + r) * rstride + g0 + k;
            v[j] = 0.0;
            if (ok[j]) v[j] = (DU && du) ? u[o[j]] + du[o[j]] : u[o[j]];
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (!ok[j]) continue;
            const int idx = base + j * np;
            buf[(idx >> lg) * (cap + 1) + (idx & (cap - 1))] = v[j];
            if (uout) uout[o[j]] = v[j];
        }
    }
}

// Pendulum and cart-pole (nu = 1): x_{k+1} = x_k + h f(x_k, u_k + du_k) from
// x0 (du may be null), lane r of wave 0 for instance blockIdx.x * R + r,
// R = 2^(12 - lg) instances per block, chunks of 2^lg stages.  Writes x
// (T + 1 rows) and, if uout is set, the controls used.
template <int MODEL, bool DU>
__global__ __launch_bounds__(ROLL_THREADS) void k_nmpc_rollout(NmpcPtrs N, const double *__restrict__ u,
                                                               const double *__restrict__ du,
                                                               double *__restrict__ xout, double *__restrict__ uout,
                                                               const double *lvl, int lg)
{
    constexpr int n = (MODEL == MODEL_PENDULUM) ? 2 : 4;
    __shared__ double su[2][ROLL_SLOTS + 64];
    const int T = N.T, R = ROLL_SLOTS >> lg, CH = 1 << lg;
    const int t = threadIdx.x, lane = t & 63;
    const int64_t inst0 = (int64_t)blockIdx.x * R;
    const int64_t b = inst0 + lane;
    const bool mine = lane < R && b < N.batch && !level_done(lvl, b);
    const uint64_t act = __ballot(mine);   // the same in every wave
    if (act == 0) return;                  // uniform over the block
    if (!DU) du = nullptr;
    const int nch = (T + CH - 1) / CH;
    double x[n];
    if (t < 64 && mine) {
#pragma unroll
        for (int i = 0; i < n; ++i) {
            x[i] = N.x0[b * n + i];
            xout[b * (T + 1) * n + i] = x[i];
        }
    }
    if (nch == 0) return;
    stage_controls<DU>(su[0], lg, min(CH, T), act, inst0, T, 0, u, du, uout, t, ROLL_THREADS);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int c0 = c * CH, len = min(CH, T - c0);
        if (t < 64) {
            if (mine) {
                const double *row = su[c & 1] + lane * (CH + 1);
                double *xo = xout + b * (T + 1) * n + (int64_t)(c0 + 1) * n;
                double un = row[0];
                for (int k = 0; k < len; ++k) {
                    const double uk = un;
                    un = row[min(k + 1, len - 1)];   // next control read while this step runs
                    double f[n];
                    if constexpr (MODEL == MODEL_PENDULUM) {
                        const double z[3] = {x[0], x[1], uk};
                        pendulum_f<double, double>(N.prm, z, f);
                    } else {
                        const double z[5] = {x[0], x[1], x[2], x[3], uk};
                        cartpole_f<double, double>(N.prm, z, f);
                    }
#pragma unroll
                    for (int i = 0; i < n; ++i) {
                        x[i] = x[i] + N.h * f[i];
                        xo[(int64_t)k * n + i] = x[i];
                    }
                }
            }
        } else if (c + 1 < nch) {
            const int n0 = c0 + CH;
            stage_controls<DU>(su[(c + 1) & 1], lg, min(CH, T - n0), act, inst0, T, n0, u, du, uout, t - 64,
                               ROLL_THREADS - 64);
        }
        __syncthreads();
    }
}

// Value of a double held by lane `src` of the wave, in every lane.
LQK_DEV double wave_bcast(double v, int src)
{
    const uint64_t b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The tanh model: one block per instance, chunks of 1024 stages (m <= 4
// controls each) staged as above.  Lane i < nx of wave 0 computes row i of
// every step, x_i <- x_i + h (tanh(w_i'x) + b_i'u), and the state is
// broadcast from those lanes after each step, so the nx tanh evaluations of
// a step run side by side.  Each row is the same arithmetic in the same
// order as a one-lane loop.  NX > 0: compile-time sizes (nx = NX <= 4,
// nu = NU); NX = 0: any nx <= 15, nu <= 4.
template <int NX, int NU>
__global__ __launch_bounds__(ROLL_THREADS) void k_nmpc_rollout_tanh(NmpcPtrs N, const double *__restrict__ u,
                                                                    const double *__restrict__ du,
                                                                    double *__restrict__ xout,
                                                                    double *__restrict__ uout, const double *lvl)
{
    if (level_done(lvl, blockIdx.x)) return;   // uniform over the block
    constexpr bool FIXED = NX > 0;
    constexpr int XM = FIXED ? NX : NXMAX, UM = FIXED ? NU : NUMAX;
    constexpr int CH = 1024, LG = 12;   // CH * m <= 2^LG = ROLL_SLOTS
    __shared__ double su[2][ROLL_SLOTS + 64];
    const int n = FIXED ? NX : N.nx, m = FIXED ? NU : N.nu, T = N.T;
    const int64_t b = blockIdx.x;   // one instance per block
    const int t = threadIdx.x;
    const bool row = t < n;
    const int ti = row ? t : 0;
    const int nch = (T + CH - 1) / CH;
    xout += b * (T + 1) * n;
    // this lane's row of W and B, and the initial state
    double Wr[XM], Br[UM], x[XM], xi = 0.0;
    if (t < 64) {
#pragma unroll
        for (int j = 0; j < XM; ++j) Wr[j] = (j < n) ? N.W[ti * n + (j < n ? j : 0)] : 0.0;
#pragma unroll
        for (int j = 0; j < UM; ++j) Br[j] = (j < m) ? N.Bm[ti * m + (j < m ? j : 0)] : 0.0;
        xi = N.x0[b * n + ti];
        if (row) xout[t] = xi;
#pragma unroll
        for (int j = 0; j < XM; ++j) x[j] = (j < n) ? wave_bcast(xi, j) : 0.0;
    }
    if (nch == 0) return;
    stage_controls<true>(su[0], LG, min(CH, T) * m, 1, b, (int64_t)T * m, 0, u, du, uout, t, ROLL_THREADS);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int c0 = c * CH, len = min(CH, T - c0);
        if (t < 64) {
            const double *sc = su[c & 1];
            for (int k = 0; k < len; ++k) {
                double uk[UM];
#pragma unroll
                for (int j = 0; j < UM; ++j) uk[j] = (j < m) ? sc[k * m + (j < m ? j : 0)] : 0.0;
                double z = 0.0, bu = 0.0;
#pragma unroll
                for (int j = 0; j < XM; ++j)
                    if (j < n) z += Wr[j] * x[j];
#pragma unroll
                for (int j = 0; j < UM; ++j)
                    if (j < m) bu += Br[j] * uk[j];
                xi = xi + N.h * (tanh_em1(z) + bu);
                if (row) xout[(int64_t)(c0 + k + 1) * n + t] = xi;
#pragma unroll
                for (int j = 0; j < XM; ++j) x[j] = (j < n) ? wave_bcast(xi, j) : 0.0;
            }
        } else if (c + 1 < nch) {
            const int n0 = c0 + CH;
            stage_controls<true>(su[(c + 1) & 1], LG, min(CH, T - n0) * m, 1, b, (int64_t)T * m, (int64_t)n0 * m, u,
                                 du, uout, t - 64, ROLL_THREADS - 64);
        }
        __syncthreads();
    }
}

// One step of the discretised dynamics, x+ = x + h f(x, u), in the arithmetic
// of the sequential rollouts above, and its Jacobian F = I + h df/dx (the
// pendulum and cart-pole by first-order forward mode).
template <int MODEL, int NX, int NU>
LQK_DEV void step_jac(const NmpcPtrs &N, const double (&x)[NX], const double (&u)[NU], double (&xn)[NX],
                      double (&F)[NX][NX])
{
    if constexpr (MODEL == MODEL_TANH) {
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double z = 0.0, bu = 0.0;
#pragma unroll
            for (int j = 0; j < NX; ++j) z += N.W[i * NX + j] * x[j];
#pragma unroll
            for (int j = 0; j < NU; ++j) bu += N.Bm[i * NU + j] * u[j];
            const double th = tanh_em1(z);
            xn[i] = x[i] + N.h * (th + bu);
            const double dth = 1.0 - th * th;
#pragma unroll
            for (int j = 0; j < NX; ++j) F[i][j] = ((i == j) ? 1.0 : 0.0) + N.h * (dth * N.W[i * NX + j]);
        }
    } else {
        double z[NX + 1], f[NX];
        Dual<NX> zd[NX + 1], fd[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            z[i] = x[i];
            zd[i] = dvar<NX>(x[i], i);
        }
        z[NX] = u[0];
        zd[NX] = dvar<NX>(u[0], -1);
        if constexpr (MODEL == MODEL_PENDULUM) {
            pendulum_f<double, double>(N.prm, z, f);
            pendulum_f<Dual<NX>, double>(N.prm, zd, fd);
        } else {
            cartpole_f<double, double>(N.prm, z, f);
            cartpole_f<Dual<NX>, double>(N.prm, zd, fd);
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            xn[i] = x[i] + N.h * f[i];
#pragma unroll
            for (int j = 0; j < NX; ++j) F[i][j] = ((i == j) ? 1.0 : 0.0) + N.h * fd[i].g[j];
        }
    }
}

// Maximum of v over the block (PAR_NT threads; NaN-free inputs).
constexpr int PAR_NT = 256, PAR_SMAX = 4, PAR_ITMAX = 12;
LQK_DEV double block_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int t = threadIdx.x;
    __syncthreads();   // red is free (its previous use has been read)
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < PAR_NT / 64; ++w) r = fmax(r, red[w]);
    return r;
}

// The candidate's nonlinear rollout in parallel over time (not in the paper,
// which takes the LQ step's states): Newton's method on the defects
// d_k = x_k + h f(x_k, u_k) - x_{k+1} of a trajectory, started from the LQ
// step's prediction x + dx.  An iteration solves the linearised recursion
// delta_{k+1} = F_k delta_k + d_k, delta_0 = 0, with an affine-map scan over
// the block's threads and sets x_{k+1} += delta_{k+1}.  It stops once every
// defect is within 8 ulps of the trajectory's largest entry (the sequential
// recursion's own rounding); without that after PAR_ITMAX iterations, or with
// a defect that is not finite, thread 0 runs the sequential recursion
// instead.  One block of PAR_NT threads per instance, each thread
// S = ceil(T / PAR_NT) <= PAR_SMAX consecutive stages whose controls,
// Jacobians and defects stay in its registers.
template <int MODEL, int NX, int NU>
__global__ __launch_bounds__(PAR_NT) void k_nmpc_rollout_par(NmpcPtrs N, const double *__restrict__ u,
                                                             const double *__restrict__ du,
                                                             const double *__restrict__ xnom,
                                                             const double *__restrict__ dx, double *xout,
                                                             double *uout, const double *lvl)
{
    constexpr int NM = NX * NX + NX;
    __shared__ double sm[PAR_NT * NM];
    __shared__ double red[PAR_NT / 64];
    const int b = blockIdx.x;
    if (level_done(lvl, b)) return;   // uniform over the block
    const int T = N.T, t = threadIdx.x;
    const int S = (T + PAR_NT - 1) / PAR_NT;
    const int k0 = min(t * S, T), k1 = min(k0 + S, T);
    u += (int64_t)b * T * NU;
    du += (int64_t)b * T * NU;
    uout += (int64_t)b * T * NU;
    xout += (int64_t)b * (T + 1) * NX;
    xnom += (int64_t)b * (T + 1) * NX;
    dx += (int64_t)b * (T + 1) * NX;
    double uk[PAR_SMAX][NU];
#pragma unroll
    for (int s = 0; s < PAR_SMAX; ++s) {
        const int k = k0 + s;
        if (k >= k1) break;
#pragma unroll
        for (int a = 0; a < NU; ++a) {
            const double v = u[k * NU + a] + du[k * NU + a];
            uk[s][a] = v;
            uout[k * NU + a] = v;
        }
        // the start trajectory x + dx, rows k0 + 1 .. k1
#pragma unroll
        for (int i = 0; i < NX; ++i) xout[(k + 1) * NX + i] = xnom[(k + 1) * NX + i] + dx[(k + 1) * NX + i];
    }
    if (t == 0) {
#pragma unroll
        for (int i = 0; i < NX; ++i) xout[i] = N.x0[(int64_t)b * NX + i];
    }
    __syncthreads();
    bool done = false, bad = false;
    for (int it = 0; it < PAR_ITMAX; ++it) {
        double F[PAR_SMAX][NX][NX], dd[PAR_SMAX][NX], xo[PAR_SMAX][NX];
        double dmax = 0.0, xmax = 0.0;
        bool fin = true;
#pragma unroll
        for (int s = 0; s < PAR_SMAX; ++s) {
            const int k = k0 + s;
            if (k >= k1) break;
            double xk[NX], xn[NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                xk[i] = xout[k * NX + i];
                xo[s][i] = xout[(k + 1) * NX + i];
            }
            step_jac<MODEL, NX, NU>(N, xk, uk[s], xn, F[s]);
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                dd[s][i] = xn[i] - xo[s][i];
                fin = fin && isfinite(dd[s][i]);
                dmax = fmax(dmax, fabs(dd[s][i]));
                xmax = fmax(xmax, fabs(xn[i]));
            }
        }
        if (block_max(fin ? 0.0 : 1.0, red) > 0.0) {
            bad = true;
            break;
        }
        const double dall = block_max(dmax, red), xall = block_max(xmax, red);
        if (dall <= 8.0 * DBL_EPSILON * xall) {
            done = true;
            break;
        }
        // this thread's stages composed: delta_{k1} = Ph delta_{k0} + ph
        double Ph[NX][NX], ph[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            ph[i] = 0.0;
#pragma unroll
            for (int j = 0; j < NX; ++j) Ph[i][j] = (i == j) ? 1.0 : 0.0;
        }
#pragma unroll
        for (int s = 0; s < PAR_SMAX; ++s) {
            if (k0 + s >= k1) break;
            double nP[NX][NX], np[NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                double v = dd[s][i];
#pragma unroll
                for (int j = 0; j < NX; ++j) v += F[s][i][j] * ph[j];
                np[i] = v;
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    double w = 0.0;
#pragma unroll
                    for (int q = 0; q < NX; ++q) w += F[s][i][q] * Ph[q][j];
                    nP[i][j] = w;
                }
            }
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                ph[i] = np[i];
#pragma unroll
                for (int j = 0; j < NX; ++j) Ph[i][j] = nP[i][j];
            }
        }
        // inclusive prefix over threads (Kogge-Stone through LDS):
        // (Ph, ph) <- (Ph, ph) o (prefix of the threads before)
        for (int off = 1; off < PAR_NT; off <<= 1) {
            double *me = sm + t * NM;
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                me[NX * NX + i] = ph[i];
#pragma unroll
                for (int j = 0; j < NX; ++j) me[i * NX + j] = Ph[i][j];
            }
            __syncthreads();
            if (t >= off) {
                const double *o = sm + (t - off) * NM;
                double nP[NX][NX], np[NX];
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    double v = ph[i];
#pragma unroll
                    for (int j = 0; j < NX; ++j) v += Ph[i][j] * o[NX * NX + j];
                    np[i] = v;
#pragma unroll
                    for (int j = 0; j < NX; ++j) {
                        double w = 0.0;
#pragma unroll
                        for (int q = 0; q < NX; ++q) w += Ph[i][q] * o[q * NX + j];
                        nP[i][j] = w;
                    }
                }
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    ph[i] = np[i];
#pragma unroll
                    for (int j = 0; j < NX; ++j) Ph[i][j] = nP[i][j];
                }
            }
            __syncthreads();
        }
        // delta at this thread's first stage: the prefix of the threads before
        // (delta_0 = 0, so only its translation part)
#pragma unroll
        for (int i = 0; i < NX; ++i) sm[t * NM + NX * NX + i] = ph[i];
        __syncthreads();
        double de[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) de[i] = (t > 0) ? sm[(t - 1) * NM + NX * NX + i] : 0.0;
#pragma unroll
        for (int s = 0; s < PAR_SMAX; ++s) {
            const int k = k0 + s;
            if (k >= k1) break;
            double nd[NX];
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                double v = dd[s][i];
#pragma unroll
                for (int j = 0; j < NX; ++j) v += F[s][i][j] * de[j];
                nd[i] = v;
            }
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                de[i] = nd[i];
                xout[(k + 1) * NX + i] = xo[s][i] + de[i];
            }
        }
        __syncthreads();   // the updated trajectory is visible to every thread
    }
    if (done) return;
    (void)bad;
    // not converged (or not finite): the sequential recursion on thread 0
    __syncthreads();
    if (t != 0) return;
    double x[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) x[i] = N.x0[(int64_t)b * NX + i];
    for (int k = 0; k < T; ++k) {
        double ukk[NU], xn[NX], Fd[NX][NX];
#pragma unroll
        for (int a = 0; a < NU; ++a) ukk[a] = uout[k * NU + a];
        step_jac<MODEL, NX, NU>(N, x, ukk, xn, Fd);
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            x[i] = xn[i];
            xout[(k + 1) * NX + i] = x[i];
        }
    }
}

// Step 1 (one lane per stage of every instance), arithmetic type RT, results
// stored in FP64.  NX > 0: compile-time sizes nx = NX, nu = NU (the tanh
// model's per-stage arrays then stay in registers).
template <typename RT, int NX, int NU>
__global__ __launch_bounds__(256) void k_nmpc_linearise(NmpcPtrs N, NmpcWork Wk, const double *x, const double *u)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int n = NX > 0 ? NX : N.nx, m = NX > 0 ? NU : N.nu, T = N.T;
    if (idx >= (int64_t)N.batch * (T + 1)) return;
    const int b = (int)(idx / (T + 1)), k = (int)(idx - (int64_t)b * (T + 1));
    if (k == 0 && Wk.scal) {
        // the step after a level's last iteration: the level is over (0.5 ->
        // 1; the instance's other lanes read 0.5 or 1 and return too)
        double *sc = Wk.scal + (int64_t)b * NMPC_NSCAL;
        if (sc[NMPC_LEVEL_DONE] >= 0.5) {
            sc[NMPC_LEVEL_DONE] = 1.0;
            return;
        }
    }
    if (level_done(Wk.scal, b)) return;
    if (k == 0) {   // the instance's internal LQ status, zero initial state and copy of Q_T, read later in the step
        Wk.status[b] = 0;
        for (int i = 0; i < n; ++i) Wk.zero[(int64_t)b * n + i] = 0.0;
        for (int i = 0; i < n * n; ++i) Wk.QTb[(int64_t)b * n * n + i] = N.QT[i];
    }
    const int64_t gk = (int64_t)b * T + k;   // packed stage index (k < T)
    const double *xk = x + ((int64_t)b * (T + 1) + k) * n;
    const double *rk = N.xref + (int64_t)k * n;
    if (k == T) {   // terminal co-state lambda_T = Q_T (x_T - ref_T)
        for (int i = 0; i < n; ++i) {
            RT v = 0;
            for (int j = 0; j < n; ++j) v += (RT)N.QT[i * n + j] * ((RT)xk[j] - (RT)rk[j]);
            Wk.lamT[(int64_t)b * n + i] = (double)v;
        }
        return;
    }
    const double *uk = u + gk * m;
    if (N.model == MODEL_PENDULUM) {
        linearise_model<3>(N, Wk, gk, xk, uk);
    } else if (N.model == MODEL_CARTPOLE) {
        linearise_model<5>(N, Wk, gk, xk, uk);
    } else {
        RT th[NX > 0 ? NX : NXMAX];
        const RT h = (RT)N.h;
        for (int i = 0; i < n; ++i) {
            RT z = 0;
            for (int j = 0; j < n; ++j) z += (RT)N.W[i * n + j] * (RT)xk[j];
            th[i] = tanh(z);
            Wk.th[gk * n + i] = (double)th[i];
        }
        double *A = Wk.A + gk * n * n;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j)
                A[i * n + j] = (double)((i == j ? (RT)1 : (RT)0) + h * ((RT)1 - th[i] * th[i]) * (RT)N.W[i * n + j]);
        double *B = Wk.B + gk * n * m;
        for (int i = 0; i < n * m; ++i) B[i] = (double)(h * (RT)N.Bm[i]);
    }
    for (int i = 0; i < n; ++i) {
        RT v = 0;
        for (int j = 0; j < n; ++j) v += (RT)N.Q[i * n + j] * ((RT)xk[j] - (RT)rk[j]);
        Wk.g[gk * n + i] = (double)v;
    }
}

// Co-state map M_k = [[A_k', g_k], [0, 1]] from the linearisation: R(M_k)
// (the workspace is packed like the LQ arrays: instance offsets d.oA, d.oc).
LQK_DEV Tile costate_map(const NmpcWork &Wk, const InstDesc &d, int k)
{
    const int n = d.n, c = tcol();
    const double *A = Wk.A + d.oA + (int64_t)k * n * n, *g = Wk.g + d.oc + (int64_t)k * n;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *p = zptr();
        if (i < n && c < n)
            p = A + c * n + i;
        else if (i < n && c == n)
            p = g + i;
        else if (i == n && c == n)
            p = optr();
        t.v[r] = ldg(p);
    }
    return t;
}

// R(M_k') = [[A_k, 0], [g_k', 1]].
LQK_DEV Tile costate_map_t(const NmpcWork &Wk, const InstDesc &d, int k)
{
    const int n = d.n, c = tcol();
    const double *A = Wk.A + d.oA + (int64_t)k * n * n, *g = Wk.g + d.oc + (int64_t)k * n;
    Tile t;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = trow(r);
        const double *p = zptr();
        if (i < n && c < n)
            p = A + i * n + c;
        else if (i == n && c < n)
            p = g + c;
        else if (i == n && c == n)
            p = optr();
        t.v[r] = ldg(p);
    }
    return t;
}

// Step 2a: segment fold of the co-state maps (suffix), Psi_s = M_{k0} ...
// M_{k1-1} kept as Psi'; the block of the last segment writes the terminal
// element [[0, lambda_T], [0, 1]].
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_costate_fold(NmpcWork Wk, const InstDesc *__restrict__ inst,
                                                     const int32_t *__restrict__ seg_start, int batch, double *Y)
{
    __shared__ double lds[SLOT];
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    if (level_done(Wk.scal, i)) return;
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    if (s == d.nseg - 1) gstore_c(Y + (int64_t)(d.xbase + d.nseg) * TILE, load_vec(Wk.lamT + d.on, d.n, d.n, d.n), d.n + 1);
    if (s == 0) return;
    Tile PsiT = tident(d.n + 1);
    for (int k = k0; k < k1; ++k) PsiT = tnz<NK, PR>(costate_map(Wk, d, k), PsiT);   // (Psi M_k)'
    gstore_c(Y + (int64_t)(d.xbase + s) * TILE, ttrans(PsiT, lds), d.n + 1);
}

// Step 2c: co-states inside each segment from lambda at its right end.
template <int NK, int PR>
__global__ __launch_bounds__(64) void k_costate_apply(NmpcWork Wk, const InstDesc *__restrict__ inst,
                                                      const int32_t *__restrict__ seg_start, int batch,
                                                      const double *__restrict__ Yfin)
{
    const int gs = blockIdx.x;
    const int i = find_inst(seg_start, batch, gs);
    if (level_done(Wk.scal, i)) return;
    const InstDesc d = inst[i];
    const int s = gs - d.seg0;
    const int k0 = s * d.L, k1 = min(k0 + d.L, d.T);
    const int n = d.n;
    double *lam = Wk.lam + d.os;
    Tile L = gload_c(Yfin + (int64_t)(d.xbase + s + 1) * TILE, d.n + 1);
    if (s == d.nseg - 1) store_vec(lam + (int64_t)d.T * n, L, n, n);
    for (int k = k1 - 1; k >= k0; --k) {
        L = tnz<NK, PR>(costate_map_t(Wk, d, k), L);   // M_k L
        store_vec(lam + (int64_t)k * n, L, n, n);
    }
}

// Step 3 (one lane per stage): second-order terms of the Hamiltonian.  In
// mixed precision the lambda' d2f contractions (P, M and their R part) are
// formed in RT = float; the gradient d, the barrier terms and alpha stay FP64.
// NX > 0: compile-time sizes as in k_nmpc_linearise.
template <typename RT, int NX, int NU>
__global__ __launch_bounds__(256) void k_nmpc_quadraticise(NmpcPtrs N, NmpcWork Wk, const double *x, const double *u,
                                                           const double *scal)
{
    const int64_t gk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // instance * T + stage
    const int n = NX > 0 ? NX : N.nx, m = NX > 0 ? NU : N.nu, T = N.T;
    if (gk >= (int64_t)N.batch * T) return;
    const int b = (int)(gk / T);
    if (level_done(Wk.scal, b)) return;
    scal += (int64_t)b * NMPC_NSCAL;
    const double mu = scal[NMPC_MU], alpha = scal[NMPC_ALPHA];
    const double *l1 = Wk.lam + (gk + b + 1) * n;   // lambda_{k+1}; T + 1 rows per instance
    const double *uk = u + gk * m;
    const double *xk = x + (gk + b) * n;
    double huu = 0.0;   // h lambda' d2f/du2 (m = 1 for the pendulum and cart-pole)
    if (N.model == MODEL_PENDULUM) {
        huu = (double)quadraticise_model<3, RT>(N, Wk, gk, xk, uk, l1);
    } else if (N.model == MODEL_CARTPOLE) {
        huu = (double)quadraticise_model<5, RT>(N, Wk, gk, xk, uk, l1);
    } else {
        const double *th = Wk.th + gk * n;
        double *P = Wk.P + gk * n * n;
        RT Pl[NX > 0 ? NX * NX : NXMAX * NXMAX];
        for (int i = 0; i < n * n; ++i) Pl[i] = (RT)N.Q[i];
        for (int i = 0; i < n; ++i) {
            const RT t = (RT)th[i];
            const RT w = (RT)l1[i] * (RT)N.h * ((RT)-2 * t * ((RT)1 - t * t));
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) Pl[a * n + b] += w * (RT)N.W[i * n + a] * (RT)N.W[i * n + b];
        }
        for (int i = 0; i < n * n; ++i) P[i] = (double)Pl[i];
    }
    double *Rt = Wk.Rt + gk * m * m;
    double *Rh = Wk.Rh + gk * m * m;
    for (int i = 0; i < m * m; ++i) Rh[i] = N.R[i];
    for (int i = 0; i < m; ++i) {
        const double a = N.umax - uk[i], b = uk[i] - N.umin;
        Rh[i * m + i] += (N.rho > 0.0) ? 2.0 * N.rho : mu * (1.0 / (a * a) + 1.0 / (b * b));
    }
    if (N.model != MODEL_TANH) Rh[0] += huu;
    for (int i = 0; i < m * m; ++i) Rt[i] = Rh[i];
    for (int i = 0; i < m; ++i) Rt[i * m + i] += alpha;
    // the gradient d_k stays FP64 (mixed precision only approximates the Hessian)
    const double *B = Wk.B + gk * n * m;
    for (int i = 0; i < m; ++i) {
        double v = 0.0;
        for (int j = 0; j < m; ++j) v += N.R[i * m + j] * uk[j];
        const double uu = uk[i];
        if (N.rho > 0.0) {
            double ra, rb;
            admm_ab(N, gk, i, uu, ra, rb);
            v += N.rho * (ra - rb);
        } else {
            v += mu * (1.0 / (N.umax - uu) - 1.0 / (uu - N.umin));
        }
        for (int j = 0; j < n; ++j) v += B[j * m + i] * l1[j];
        Wk.d[gk * m + i] = v;
    }
}

// Step 5b (one block per instance): data-parallel sums over the stages with a fixed
// reduction tree -- the predicted decrease of the expansion (alpha excluded),
// |d|_inf, J_mu of the nominal and of the candidate -- then the decision
// (step 6): gain ratio rho = (J_mu(u) - J_mu(u + du)) / pred, accept if
// pred > 0 and rho > 0: alpha *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; else
// alpha *= nu, nu *= 2.  An LQ step that failed counts as pred = 0.
constexpr int RED = 256;
// RB threads per instance, chosen from the horizon (about one to four stages
// per thread).  NX > 0: the sizes nx = NX, nu = NU are compile-time (the
// pendulum, and the cart-pole and tanh model at n = 4, m = 1), so each
// thread's loads of a stage are issued together instead of one loop trip
// at a time.
template <int RB, int NX, int NU>
__global__ __launch_bounds__(RB) void k_nmpc_reduce(NmpcPtrs N, NmpcWork Wk, double *x, double *u, double *scal)
{
    __shared__ double sp[RB], s0[RB], s1[RB], sg[RB];
    __shared__ int s_acc;
    const int t = threadIdx.x, b = blockIdx.x;
    const int n = NX > 0 ? NX : N.nx, m = NX > 0 ? NU : N.nu, T = N.T;
    if (level_done(scal, b)) return;   // uniform over the block
    scal += (int64_t)b * NMPC_NSCAL;
    const int64_t s0k = (int64_t)b * T;              // first packed stage of the instance
    const int64_t xo = (int64_t)b * (T + 1) * n;    // its trajectory rows
    x += xo;
    u += s0k * m;
    const double *xc = Wk.xc + xo, *uc = Wk.uc + s0k * m, *dx = Wk.dx + xo;
    const double mu = scal[NMPC_MU];
    double pred = 0.0, J0 = 0.0, J1 = 0.0, gmax = 0.0;
    for (int k = t; k < T; k += RB) {
        const int64_t gk = s0k + k;
        const double *dxk = dx + (int64_t)k * n, *duk = Wk.du + gk * m;
        double lin = 0.0, qf = 0.0;
        for (int i = 0; i < m; ++i) {
            lin += Wk.d[gk * m + i] * duk[i];
            gmax = fmax(gmax, fabs(Wk.d[gk * m + i]));
        }
        const double *P = Wk.P + gk * n * n, *Rh = Wk.Rh + gk * m * m;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) qf += dxk[i] * P[i * n + j] * dxk[j];
        if (N.model != MODEL_TANH) {
            const double *Mk = Wk.M + gk * n * m;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < m; ++j) qf += 2.0 * dxk[i] * Mk[i * m + j] * duk[j];
        }
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) qf += duk[i] * Rh[i * m + j] * duk[j];
        pred += lin + 0.5 * qf;
        J0 += stage_cost(N, n, m, k, gk, x + (int64_t)k * n, u + (int64_t)k * m, mu);
        J1 += stage_cost(N, n, m, k, gk, xc + (int64_t)k * n, uc + (int64_t)k * m, mu);
    }
    sp[t] = pred;
    s0[t] = J0;
    s1[t] = J1;
    sg[t] = gmax;
    for (int h = RB / 2; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) {
            sp[t] += sp[t + h];
            s0[t] += s0[t + h];
            s1[t] += s1[t + h];
            sg[t] = fmax(sg[t], sg[t + h]);
        }
    }
    if (t == 0) {
        pred = sp[0];
        {
            const double *dxT = dx + (int64_t)T * n;
            double qf = 0.0;
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) qf += dxT[i] * N.QT[i * n + j] * dxT[j];
            pred += 0.5 * qf;
        }
        pred = -pred;
        J0 = s0[0] + terminal_cost(N, n, T, x + (int64_t)T * n);
        J1 = s1[0] + terminal_cost(N, n, T, xc + (int64_t)T * n);
        const bool lq_ok = (Wk.status[b] == 0);
        if (!lq_ok) {
            pred = 0.0;
            J1 = INFINITY;
        }
        double alpha = scal[NMPC_ALPHA], nu = scal[NMPC_NU];
        double rho = -INFINITY;
        bool acc = false;
        if (pred > 0.0 && isfinite(J1)) {
            rho = (J0 - J1) / pred;
            acc = rho > 0.0;
        }
        if (acc) {
            const double tt = 2.0 * rho - 1.0;
            const double f = 1.0 - tt * tt * tt;
            alpha *= (f > 1.0 / 3.0 ? f : 1.0 / 3.0);
            nu = 2.0;
        } else {
            alpha *= nu;
            nu *= 2.0;
        }
        scal[NMPC_PRED] = pred;
        scal[NMPC_GRAD] = sg[0];
        scal[NMPC_COST] = acc ? J1 : J0;
        scal[NMPC_COST_NEW] = J1;
        scal[NMPC_ALPHA] = alpha;
        scal[NMPC_NU] = nu;
        scal[NMPC_RHO] = rho;
        scal[NMPC_ACCEPTED] = acc ? 1.0 : 0.0;
        s_acc = acc;
        // level control: the level ends after the iteration that started from
        // |d|_inf <= LEVEL_TOL or that used up LEVEL_MAX iterations
        const double tol = scal[NMPC_LEVEL_TOL];
        if (tol > 0.0) {
            const double it = scal[NMPC_LEVEL_ITERS] + 1.0;
            scal[NMPC_LEVEL_ITERS] = it;
            if (sg[0] <= tol || it >= scal[NMPC_LEVEL_MAX]) scal[NMPC_LEVEL_DONE] = 0.5;
        }
    }
    // commit: every thread's reads of x, u are behind the reduction's barriers
    __syncthreads();
    if (!s_acc) return;
    for (int i = t; i < (T + 1) * n; i += RB) x[i] = xc[i];
    for (int i = t; i < T * m; i += RB) u[i] = uc[i];
}

// ADMM consensus and multiplier steps of Sec. II-C (eq:admm-step-4, -5) for
// the control box, w = h(u) = [u - umax; umin - u] per stage, C = {w <= 0}:
// z <- min(0, w + v / rho), v <- v + rho (w - z), with |r_p|_inf = |w - z|_inf
// and |r_d|_inf = |z - z_prev|_inf reduced over the block (init: z = min(0, w),
// v = 0, residuals not formed).
__global__ __launch_bounds__(RED) void k_admm_update(NmpcPtrs N, const double *u, double *scal, int init)
{
    __shared__ double sp[RED], sd[RED];
    const int t = threadIdx.x, m = N.nu, b = blockIdx.x;   // one block per instance
    const int64_t cnt = (int64_t)N.T * 2 * m;
    u += (int64_t)b * N.T * m;
    double *z = N.z + (int64_t)b * cnt, *v = N.v + (int64_t)b * cnt;
    scal += (int64_t)b * NMPC_NSCAL;
    double rp = 0.0, rd = 0.0;
    for (int64_t o = t; o < cnt; o += RED) {
        const int64_t k = o / (2 * m);
        const int i = (int)(o - k * 2 * m);
        const double ui = u[k * m + (i < m ? i : i - m)];
        const double w = (i < m) ? ui - N.umax : N.umin - ui;
        if (init) {
            z[o] = fmin(0.0, w);
            v[o] = 0.0;
            continue;
        }
        const double zn = fmin(0.0, w + v[o] / N.rho);
        rd = fmax(rd, fabs(zn - z[o]));
        rp = fmax(rp, fabs(w - zn));
        z[o] = zn;
        v[o] += N.rho * (w - zn);
    }
    sp[t] = rp;
    sd[t] = rd;
    for (int h = RED / 2; h > 0; h >>= 1) {
        __syncthreads();
        if (t < h) {
            sp[t] = fmax(sp[t], sp[t + h]);
            sd[t] = fmax(sd[t], sd[t + h]);
        }
    }
    if (t == 0 && !init) {
        scal[NMPC_RP] = sp[0];
        scal[NMPC_RD] = sd[0];
    }
}

// Receding horizon (one lane per instance): the plant takes one step with the
// first control, x0 <- x0 + h f(x0, u_0) (u_0 is also written to uapp), and
// the controls shift by one stage for the next solve's warm start (the last
// one is kept).
__global__ __launch_bounds__(64) void k_nmpc_shift(NmpcPtrs N, double *x0, double *u, double *uapp)
{
    const int b = blockIdx.x * 64 + threadIdx.x;
    if (b >= N.batch) return;
    const int n = N.nx, m = N.nu, T = N.T;
    double *xb = x0 + (int64_t)b * n, *ub = u + (int64_t)b * T * m;
    double xc[NXMAX], u0[NUMAX], xn[NXMAX];
    for (int i = 0; i < n; ++i) xc[i] = xb[i];
    for (int i = 0; i < m; ++i) {
        u0[i] = ub[i];
        uapp[(int64_t)b * m + i] = u0[i];
    }
    f_step(N, n, m, xc, u0, xn);
    for (int i = 0; i < n; ++i) xb[i] = xn[i];
    for (int k = 0; k + 1 < T; ++k)
        for (int i = 0; i < m; ++i) ub[(int64_t)k * m + i] = ub[(int64_t)(k + 1) * m + i];
}


static void launch_rollout(hipStream_t st, const NmpcPtrs &N, const double *u, const double *du, double *xout,
                           double *uout, const double *lvl)
{
    // pendulum / cart-pole: R = 2^(12 - lg) instances per block, the smallest
    // power of two >= batch, at most 64 (one lane of wave 0 each)
    int lg = 12;
    while (lg > 6 && (int64_t)(ROLL_SLOTS >> lg) < N.batch) --lg;
    const unsigned blocks = (unsigned)((N.batch + (ROLL_SLOTS >> lg) - 1) / (ROLL_SLOTS >> lg));
#define RL(M, D) \
    hipLaunchKernelGGL((k_nmpc_rollout<M, D>), dim3(blocks), dim3(ROLL_THREADS), 0, st, N, u, du, xout, uout, lvl, lg)
    if (N.model == MODEL_PENDULUM) {
        if (du) RL(MODEL_PENDULUM, true); else RL(MODEL_PENDULUM, false);
    } else if (N.model == MODEL_CARTPOLE) {
        if (du) RL(MODEL_CARTPOLE, true); else RL(MODEL_CARTPOLE, false);
    } else {
#define RT(X, U) \
    hipLaunchKernelGGL((k_nmpc_rollout_tanh<X, U>), dim3(N.batch), dim3(ROLL_THREADS), 0, st, N, u, du, xout, uout, lvl)
        if (N.nx <= 4) {
            switch (N.nx * 8 + N.nu) {
            case 9: RT(1, 1); break;  case 10: RT(1, 2); break; case 11: RT(1, 3); break; case 12: RT(1, 4); break;
            case 17: RT(2, 1); break; case 18: RT(2, 2); break; case 19: RT(2, 3); break; case 20: RT(2, 4); break;
            case 25: RT(3, 1); break; case 26: RT(3, 2); break; case 27: RT(3, 3); break; case 28: RT(3, 4); break;
            case 33: RT(4, 1); break; case 34: RT(4, 2); break; case 35: RT(4, 3); break; default: RT(4, 4); break;
            }
        } else {
            RT(0, 0);
        }
#undef RT
    }
#undef RL
}
void launch_nmpc_init(hipStream_t st, NmpcPtrs N, double *x, const double *u)
{
    launch_rollout(st, N, u, nullptr, x, nullptr, nullptr);
}
void launch_nmpc_shift(hipStream_t st, NmpcPtrs N, double *x0, double *u, double *uapp)
{
    hipLaunchKernelGGL(k_nmpc_shift, dim3((N.batch + 63) / 64), dim3(64), 0, st, N, x0, u, uapp);
}
void launch_nmpc_linearise(int pr, hipStream_t st, NmpcPtrs N, NmpcWork Wk, const double *x, const double *u)
{
    // The Jacobians define the co-states and hence the gradient, which sets
    // the point Newton converges to: FP64 in every precision mode.
    (void)pr;
    const int64_t cnt = (int64_t)N.batch * (N.T + 1);
    const dim3 g((unsigned)((cnt + 255) / 256));
    if (N.nx == 2 && N.nu == 1)
        hipLaunchKernelGGL((k_nmpc_linearise<double, 2, 1>), g, dim3(256), 0, st, N, Wk, x, u);
    else if (N.nx == 4 && N.nu == 1)
        hipLaunchKernelGGL((k_nmpc_linearise<double, 4, 1>), g, dim3(256), 0, st, N, Wk, x, u);
    else
        hipLaunchKernelGGL((k_nmpc_linearise<double, 0, 0>), g, dim3(256), 0, st, N, Wk, x, u);
}
void launch_costate_fold(int nk, int pr, unsigned grid, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                         const int32_t *seg_start, int batch, double *Y)
{
#define CALL(K, R) hipLaunchKernelGGL((k_costate_fold<K, R>), dim3(grid), dim3(64), 0, st, Wk, inst, seg_start, batch, Y)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
void launch_costate_apply(int nk, int pr, unsigned grid, hipStream_t st, NmpcWork Wk, const InstDesc *inst,
                          const int32_t *seg_start, int batch, const double *Yfin)
{
#define CALL(K, R) \
    hipLaunchKernelGGL((k_costate_apply<K, R>), dim3(grid), dim3(64), 0, st, Wk, inst, seg_start, batch, Yfin)
    LQK_DISPATCH(nk, pr, CALL)
#undef CALL
}
void launch_nmpc_quadraticise(int pr, hipStream_t st, NmpcPtrs N, NmpcWork Wk, const double *x, const double *u,
                              const double *scal)
{
    const unsigned g = (unsigned)(((int64_t)N.batch * N.T + 255) / 256);
#define QC(R, X, U) hipLaunchKernelGGL((k_nmpc_quadraticise<R, X, U>), dim3(g), dim3(256), 0, st, N, Wk, x, u, scal)
    if (N.nx == 2 && N.nu == 1) {
        if (pr) QC(float, 2, 1); else QC(double, 2, 1);
    } else if (N.nx == 4 && N.nu == 1) {
        if (pr) QC(float, 4, 1); else QC(double, 4, 1);
    } else {
        if (pr) QC(float, 0, 0); else QC(double, 0, 0);
    }
#undef QC
}
template <int RB>
static void launch_reduce(hipStream_t st, const NmpcPtrs &N, const NmpcWork &Wk, double *x, double *u, double *scal)
{
    if (N.nx == 2 && N.nu == 1)
        hipLaunchKernelGGL((k_nmpc_reduce<RB, 2, 1>), dim3(N.batch), dim3(RB), 0, st, N, Wk, x, u, scal);
    else if (N.nx == 4 && N.nu == 1)
        hipLaunchKernelGGL((k_nmpc_reduce<RB, 4, 1>), dim3(N.batch), dim3(RB), 0, st, N, Wk, x, u, scal);
    else
        hipLaunchKernelGGL((k_nmpc_reduce<RB, 0, 0>), dim3(N.batch), dim3(RB), 0, st, N, Wk, x, u, scal);
}
// The parallel rollout where it applies: horizons of 64 .. PAR_NT * PAR_SMAX
// stages for the pendulum, the cart-pole and the tanh model with nx <= 4,
// nu = 1 (LQSCAN_PAR_ROLLOUT=0: always the sequential kernels).
static bool launch_rollout_par(hipStream_t st, const NmpcPtrs &N, const NmpcWork &Wk, const double *x,
                               const double *u)
{
    const char *e = getenv("LQSCAN_PAR_ROLLOUT");
    const bool on = !(e && e[0] == '0' && e[1] == 0);
    if (!on || N.T < 64 || N.T > PAR_NT * PAR_SMAX || N.nu != 1) return false;
#define RP(M, X) \
    hipLaunchKernelGGL((k_nmpc_rollout_par<M, X, 1>), dim3(N.batch), dim3(PAR_NT), 0, st, N, u, Wk.du, x, Wk.dx, \
                       Wk.xc, Wk.uc, Wk.scal)
    if (N.model == MODEL_PENDULUM) {
        RP(MODEL_PENDULUM, 2);
    } else if (N.model == MODEL_CARTPOLE) {
        RP(MODEL_CARTPOLE, 4);
    } else {
        switch (N.nx) {
        case 1: RP(MODEL_TANH, 1); break;
        case 2: RP(MODEL_TANH, 2); break;
        case 3: RP(MODEL_TANH, 3); break;
        case 4: RP(MODEL_TANH, 4); break;
        default: return false;
        }
    }
#undef RP
    return true;
}

void launch_nmpc_candidate(hipStream_t st, NmpcPtrs N, NmpcWork Wk, double *x, double *u, double *scal)
{
    if (!launch_rollout_par(st, N, Wk, x, u)) launch_rollout(st, N, u, Wk.du, Wk.xc, Wk.uc, Wk.scal);
    if (N.T <= 96)
        launch_reduce<64>(st, N, Wk, x, u, scal);
    else if (N.T <= 384)
        launch_reduce<256>(st, N, Wk, x, u, scal);
    else
        launch_reduce<1024>(st, N, Wk, x, u, scal);
}
void launch_admm_update(hipStream_t st, NmpcPtrs N, const double *u, double *scal, int init)
{
    hipLaunchKernelGGL(k_admm_update, dim3(N.batch), dim3(RED), 0, st, N, u, scal, init);
}

}  // namespace lqk
