"""Pins of the oracle's pendulum and cart-pole models (Sec. V) and of the
interior-point loop with converged inner Newton iterations (Sec. II-B, Alg. 4).

The dynamics are pinned by mechanics (the power balance of each system, which
a wrong sign, a dropped term or a wrong power of omega breaks), the
hand-derived Jacobians and second derivatives by finite differences of the
dynamics, the co-state gradient by finite differences of J_mu, and the Newton
step by the regularised Newton system it must solve.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W


def rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


MODELS = {"pendulum": W.pendulum_problem, "cartpole": W.cartpole_problem}


def random_states(p, rng, count=20):
    n = p.nx
    xs = rng.uniform(-3, 3, (count, n))
    us = rng.uniform(0.9 * p.umin, 0.9 * p.umax, (count, p.nu))
    return xs, us


def test_pendulum_power_balance():
    """E = m l^2 omega^2 / 2 + m g l (1 - cos theta) changes at the rate
    tau omega - b omega^2 along f."""
    p = W.pendulum_problem(10)
    g, l, m, b = p.param
    rng = np.random.default_rng(0)
    for x, u in zip(*random_states(p, rng)):
        f = oracle.nmpc_f(p, x, u)
        th, om = x
        dE = m * l * l * om * f[1] + m * g * l * np.sin(th) * f[0]
        assert f[0] == om
        assert abs(dE - (u[0] * om - b * om * om)) <= 1e-12 * (1 + abs(dE))


def test_cartpole_power_balance():
    """With the pole at (p + l sin theta, -l cos theta):
    E = (m_c + m_p) v^2 / 2 + m_p l v omega cos theta + m_p l^2 omega^2 / 2 - m_p g l cos theta
    changes at the rate F v (no friction).  The omega^2 in p'' is needed for this."""
    p = W.cartpole_problem(10)
    g, l, mc, mp = p.param
    rng = np.random.default_rng(1)
    for x, u in zip(*random_states(p, rng)):
        f = oracle.nmpc_f(p, x, u)
        _, th, v, om = x
        a, al = f[2], f[3]
        assert f[0] == v and f[1] == om
        # dE/dt by the chain rule
        dE = ((mc + mp) * v * a + mp * l * (a * om * np.cos(th) + v * al * np.cos(th) - v * om * om * np.sin(th))
              + mp * l * l * om * al + mp * g * l * np.sin(th) * om)
        assert abs(dE - u[0] * v) <= 1e-11 * (1 + abs(u[0] * v) + mp * g * l * abs(om))


def test_pendulum_equilibria():
    """Hanging and upright rest states with zero torque are equilibria."""
    p = W.pendulum_problem(10)
    for th in (0.0, np.pi):
        f = oracle.nmpc_f(p, np.array([th, 0.0]), np.array([0.0]))
        assert np.max(np.abs(f)) < 1e-14   # sin(pi) rounds to 1.2e-16


@pytest.mark.parametrize("name", sorted(MODELS))
def test_jacobians_match_fd(name):
    """A = I + h df/dx and B = h df/du of the expansion against central differences of f."""
    p = MODELS[name](12)
    rng = np.random.default_rng(2)
    x = rng.uniform(-2, 2, (p.T + 1, p.nx))
    u = rng.uniform(0.5 * p.umin, 0.5 * p.umax, (p.T, p.nu))
    e = oracle.nmpc_expand(p, x, u, 1e-2)
    eps = 1e-6
    for k in (0, 5, 11):
        A = np.zeros((p.nx, p.nx))
        B = np.zeros((p.nx, p.nu))
        for j in range(p.nx):
            d = np.eye(p.nx)[j] * eps
            A[:, j] = (oracle.nmpc_f(p, x[k] + d, u[k]) - oracle.nmpc_f(p, x[k] - d, u[k])) / (2 * eps)
        for j in range(p.nu):
            d = np.eye(p.nu)[j] * eps
            B[:, j] = (oracle.nmpc_f(p, x[k], u[k] + d) - oracle.nmpc_f(p, x[k], u[k] - d)) / (2 * eps)
        assert rel(e["A"][k], np.eye(p.nx) + p.h * A) < 1e-9
        assert rel(e["B"][k], p.h * B) < 1e-8


@pytest.mark.parametrize("name", sorted(MODELS))
def test_second_derivatives_match_fd(name):
    """P = Q + h lam' d2f/dx2, M = h lam' d2f/dxdu and the lam' d2f/du2 part of Rh
    against central second differences of lam_{k+1}' f."""
    p = MODELS[name](12)
    rng = np.random.default_rng(3)
    x = rng.uniform(-2, 2, (p.T + 1, p.nx))
    u = rng.uniform(0.5 * p.umin, 0.5 * p.umax, (p.T, p.nu))
    mu = 1e-2
    e = oracle.nmpc_expand(p, x, u, mu)
    n, m = p.nx, p.nu
    for k in (1, 7):
        lam = e["lam"][k + 1]

        def s(z):
            return lam @ oracle.nmpc_f(p, z[:n], z[n:])

        z0 = np.concatenate([x[k], u[k]])
        H = np.zeros((n + m, n + m))
        eps = 1e-4
        for i in range(n + m):
            for j in range(n + m):
                di, dj = np.eye(n + m)[i] * eps, np.eye(n + m)[j] * eps
                H[i, j] = (s(z0 + di + dj) - s(z0 + di - dj) - s(z0 - di + dj) + s(z0 - di - dj)) / (4 * eps * eps)
        scale = np.max(np.abs(H)) + 1e-300
        assert np.max(np.abs((e["P"][k] - p.Q) - p.h * H[:n, :n])) < 1e-6 * p.h * scale
        assert np.max(np.abs(e["M"][k] - p.h * H[:n, n:])) < 1e-6 * p.h * scale
        ub = u[k, 0]
        barrier = mu * (1 / (p.umax - ub) ** 2 + 1 / (ub - p.umin) ** 2)
        assert abs((e["Rh"][k, 0, 0] - p.R[0, 0] - barrier) - p.h * H[n, n]) < 1e-6 * p.h * scale


def grad_fd(p, u, mu, eps=1e-6):
    g = np.zeros_like(u)
    for k in range(u.shape[0]):
        for i in range(u.shape[1]):
            up, um = u.copy(), u.copy()
            up[k, i] += eps
            um[k, i] -= eps
            g[k, i] = (oracle.nmpc_cost(p, up, mu) - oracle.nmpc_cost(p, um, mu)) / (2 * eps)
    return g


@pytest.mark.parametrize("name", sorted(MODELS))
def test_costate_gradient_is_fd_gradient(name):
    """d_k from the co-state pass (eq:co-state-eq) is the gradient of J_mu(u) of the nonlinear rollout."""
    p = MODELS[name](25)
    p = dataclasses.replace(p, Q=np.eye(p.nx) * 0.3)   # a running state cost too
    u = p.u0 * 5.0
    x = oracle.nmpc_rollout(p, u)
    e = oracle.nmpc_expand(p, x, u, 1e-2)
    g = grad_fd(p, u, 1e-2)
    assert rel(e["d"], g) < 1e-6


@pytest.mark.parametrize("name", sorted(MODELS))
def test_newton_step_solves_regularised_newton_system(name):
    """The LQ step with the cross term M satisfies (Hess J_mu + alpha I) du = -grad J_mu,
    the Hessian-vector product taken by central differences of the co-state gradient."""
    p = MODELS[name](20)
    p = dataclasses.replace(p, Q=np.eye(p.nx) * 0.3)
    mu, alpha = 1e-2, 0.5
    u = p.u0 * 5.0
    x = oracle.nmpc_rollout(p, u)
    e = oracle.nmpc_expand(p, x, u, mu)
    Ra = e["Rh"] + alpha * np.eye(p.nu)[None]
    o = oracle.lq_solve(e["A"], e["B"], None, e["P"], Ra, p.QT, np.zeros(p.nx), M=e["M"], r=e["d"])
    du = o["u"]

    def grad(uu):
        return oracle.nmpc_expand(p, oracle.nmpc_rollout(p, uu), uu, mu)["d"]

    eps = 1e-5
    Hv = (grad(u + eps * du) - grad(u - eps * du)) / (2 * eps)
    resid = Hv + alpha * du + e["d"]
    assert np.max(np.abs(resid)) < 1e-5 * np.max(np.abs(e["d"]))


@pytest.mark.parametrize("name,N", [("pendulum", 40), ("cartpole", 40), ("pendulum", 200)])
def test_interior_point_swing_up(name, N):
    """The IP loop keeps every iterate strictly feasible, ends every barrier level at
    |dJ_mu/du|_inf <= tol or the iteration cap, lowers mu by zeta from mu0 while above
    mu_min, and swings the pole up (final angle within 0.1 rad of upright)."""
    p = MODELS[name](N)
    o = oracle.nmpc_ip_solve(p, mu0=W.IP_MU0, zeta=W.IP_ZETA, mu_min=W.IP_MU_MIN, tol=W.IP_TOL,
                             max_iter=W.IP_MAX_ITER, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    assert np.all(o["u"] < p.umax) and np.all(o["u"] > p.umin)
    mus = W.IP_MU0 * W.IP_ZETA ** np.arange(len(o["level_iters"]))
    assert len(mus) == 5 and mus[-1] > W.IP_MU_MIN and mus[-1] * W.IP_ZETA <= W.IP_MU_MIN
    ends = np.cumsum(o["level_iters"]) - 1
    for lv, e in enumerate(ends):
        assert o["mu"][e] == pytest.approx(mus[lv])
        assert o["grad"][e] <= W.IP_TOL or o["level_iters"][lv] == W.IP_MAX_ITER
    theta = o["x"][-1][0 if name == "pendulum" else 1]
    assert abs(theta - np.pi) < 0.1
    # the rollout of the result is the returned trajectory
    assert rel(oracle.nmpc_rollout(p, o["u"]), o["x"]) < 1e-14


def test_tanh_model_unchanged_by_default():
    """A problem without model fields is the tanh network; its expansion has M = 0."""
    p = W.nmpc_problem(seed=1, T=8)
    x = oracle.nmpc_rollout(p, p.u0)
    e = oracle.nmpc_expand(p, x, p.u0, 1e-2)
    assert np.all(e["M"] == 0.0)
    xn = x[0] + p.h * (np.tanh(p.W @ x[0]) + p.Bm @ p.u0[0])
    assert rel(x[1], xn) < 1e-15


# --------------------------------------------------------------------------
# ADMM (Sec. II-C) on the control box
# --------------------------------------------------------------------------

def random_admm(p, rng, rho=0.7):
    z = -np.abs(rng.standard_normal((p.T, 2 * p.nu)))
    v = np.abs(rng.standard_normal((p.T, 2 * p.nu)))
    return {"rho": rho, "z": z, "v": v}


@pytest.mark.parametrize("name", sorted(MODELS))
def test_admm_gradient_is_fd_gradient(name):
    """With the augmentation rho/2 |h(u) - z + v/rho|^2 in place of the barrier, d_k is the
    gradient of J_AD(u) of the nonlinear rollout (u may leave the box)."""
    p = MODELS[name](25)
    rng = np.random.default_rng(5)
    admm = random_admm(p, rng)
    u = p.u0 * 5.0
    u[3, 0] = 1.2 * p.umax   # outside the box: allowed for ADMM
    e = oracle.nmpc_expand(p, oracle.nmpc_rollout(p, u), u, 0.0, admm=admm)
    g = np.zeros_like(u)
    eps = 1e-6
    for k in range(p.T):
        up, um = u.copy(), u.copy()
        up[k, 0] += eps
        um[k, 0] -= eps
        g[k, 0] = (oracle.nmpc_cost(p, up, 0.0, admm=admm) - oracle.nmpc_cost(p, um, 0.0, admm=admm)) / (2 * eps)
    assert np.isfinite(oracle.nmpc_cost(p, u, 0.0, admm=admm))
    assert rel(e["d"], g) < 1e-6


@pytest.mark.parametrize("name", sorted(MODELS))
def test_admm_newton_step_solves_regularised_newton_system(name):
    """The Newton step of J_AD (R + 2 rho I in the expansion) solves (Hess J_AD + alpha I) du = -grad J_AD."""
    p = MODELS[name](20)
    rng = np.random.default_rng(6)
    admm = random_admm(p, rng)
    alpha = 0.5
    u = p.u0 * 5.0
    e = oracle.nmpc_expand(p, oracle.nmpc_rollout(p, u), u, 0.0, admm=admm)
    Ra = e["Rh"] + alpha * np.eye(p.nu)[None]
    du = oracle.lq_solve(e["A"], e["B"], None, e["P"], Ra, p.QT, np.zeros(p.nx), M=e["M"], r=e["d"])["u"]

    def grad(uu):
        return oracle.nmpc_expand(p, oracle.nmpc_rollout(p, uu), uu, 0.0, admm=admm)["d"]

    eps = 1e-5
    Hv = (grad(u + eps * du) - grad(u - eps * du)) / (2 * eps)
    assert np.max(np.abs(Hv + alpha * du + e["d"])) < 1e-5 * np.max(np.abs(e["d"]))


@pytest.mark.parametrize("name,N", [("pendulum", 40), ("cartpole", 20)])
def test_admm_solve_invariants_and_convergence(name, N):
    """z stays in C = {z <= 0}, the multipliers stay non-negative and complementary to z
    (v_i > 0 only where z_i = 0), the loop stops at |r_p|, |r_d| <= eps, the final controls
    violate the box by at most eps, and the swing-up still reaches the top."""
    p = MODELS[name](N)
    rho = W.ADMM_RHO[name] * p.h
    o = oracle.nmpc_admm_solve(p, rho=rho, eps=W.ADMM_EPS, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                               max_admm=W.ADMM_MAX_ITER, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    assert o["admm_iters"] < W.ADMM_MAX_ITER
    assert o["rp"][-1] <= W.ADMM_EPS and o["rd"][-1] <= W.ADMM_EPS
    assert np.all(o["z"] <= 0.0) and np.all(o["v"] >= 0.0)
    assert np.all((o["v"] == 0.0) | (o["z"] == 0.0))
    viol = max(np.max(o["u"] - p.umax), np.max(p.umin - o["u"]))
    assert viol <= W.ADMM_EPS
    theta = o["x"][-1][0 if name == "pendulum" else 1]
    assert abs(theta - np.pi) < 0.15
    assert rel(oracle.nmpc_rollout(p, o["u"]), o["x"]) < 1e-14


# --------------------------------------------------------------------------
# Receding-horizon MPC (Sec. V)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", sorted(MODELS))
def test_mpc_closed_loop_stabilises(name):
    """The closed loop follows the plant model step by step, keeps every applied control
    inside the bounds and ends at the upright equilibrium (cart at 0) after 4 s."""
    xs = W.mpc_initial_states(name, 6)
    for xi in xs:
        p = W.mpc_problem(name, xi)
        o = oracle.nmpc_mpc_simulate(p, xi, steps=W.MPC_STEPS, mu_levels=W.MPC_MU_LEVELS, iters=W.MPC_ITERS,
                                     alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
        x, u = o["x"], o["u"]
        assert np.all(np.abs(u) < p.umax)
        for t in (0, 7, 150, W.MPC_STEPS - 1):
            f = oracle.nmpc_f(p, x[t], u[t])
            assert rel(x[t + 1], x[t] + p.h * f) < 1e-15
        target = p.xref[0]
        assert np.max(np.abs(x[-1] - target)) < 0.05, x[-1]
