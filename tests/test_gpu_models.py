"""GPU parity of the Newton / interior-point step for the pendulum and cart-pole
models of Sec. V (newton_step with model selector) against the FP64 oracle.

Single steps: accept decision identical, predicted decrease, costs, alpha,
gradient norm and the new trajectory within 1e-10 (normwise relative).

Whole interior-point solves (mu from 0.1 times 0.2 while above 1e-4, inner
loops to |dJ_mu/du|_inf <= 1e-6): an accept decision taken where the
predicted decrease is below 1e-9 |J_mu| compares rounding errors and is not
determined by the arithmetic; it can change the damping and from there on
the two runs may follow different (equally valid) paths.  Up to the first such
iteration the traces take the same decisions (a step whose LQ solve fails has
pred = 0 on both sides and is rejected by both) and their costs agree to 2e-7:
the oracle's own loop with u perturbed by 1e-15 (relative) after every step
moves its cost trace by up to 3.8e-8 there (pendulum, N = 400: up to a
hundred iterations of a nonconvex descent amplify round-off).  At the end
both runs are stationary to the tolerance in the last barrier level (or at
its iteration cap) and reach the same local minimum: final J_mu within 1e-7,
controls and states within 1e-5 (the perturbed oracle runs end up to 4e-7
apart).
"""
import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MODELS = {"pendulum": W.pendulum_problem, "cartpole": W.cartpole_problem}


@pytest.fixture(scope="module")
def lq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_20027_amd import lqscan
    return lqscan


def rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


@pytest.mark.parametrize("name", sorted(MODELS))
@pytest.mark.parametrize("seg_len,mode", [(0, "scan"), (5, "scan"), (1, "scan"), (0, "sequential")])
def test_single_newton_step(lq, name, seg_len, mode):
    p = MODELS[name](97)
    u0 = p.u0 * 5.0   # away from zero so that every term is exercised
    import dataclasses
    p = dataclasses.replace(p, u0=u0, Q=np.eye(p.nx) * 0.2)
    mu, alpha, nu = 0.1, 0.05, 2.0
    x0 = oracle.nmpc_rollout(p, p.u0)
    acc, x1, u1, a1, nu1, cost, pred, rho, grad = oracle.nmpc_newton_step(p, x0, p.u0, mu, alpha, nu,
                                                                          with_grad=True)
    s = lq.NewtonMPC(p, seg_len=seg_len, mode=mode)
    s.init(alpha, nu)
    s.step(mu)
    torch.cuda.synchronize()
    sc = s.scal.cpu().numpy()
    assert bool(sc[lq.NMPC_ACCEPTED] > 0.5) == acc
    assert abs(sc[lq.NMPC_PRED] - pred) <= 1e-10 * abs(pred)
    assert abs(sc[lq.NMPC_COST] - cost) <= 1e-10 * abs(cost)
    assert abs(sc[lq.NMPC_GRAD] - grad) <= 1e-10 * abs(grad)
    assert abs(sc[lq.NMPC_ALPHA] - a1) <= 1e-10 * abs(a1) and sc[lq.NMPC_NU] == nu1
    assert rel(s.u.cpu().numpy().reshape(p.T, p.nu), u1) < 1e-10
    assert rel(s.x.cpu().numpy().reshape(p.T + 1, p.nx), x1) < 1e-10


def ip(lq, p, **kw):
    args = dict(mu0=W.IP_MU0, zeta=W.IP_ZETA, mu_min=W.IP_MU_MIN, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    ref = oracle.nmpc_ip_solve(p, **args)
    got = lq.NewtonMPC(p, **kw).ip_solve(**args)
    return got, ref


@pytest.mark.parametrize("name,N", [("pendulum", 40), ("cartpole", 40), ("pendulum", 400), ("cartpole", 1000)])
def test_interior_point_solve_matches_oracle(lq, name, N):
    p = MODELS[name](N)
    got, ref = ip(lq, p)
    check_ip(p, got, ref)


def check_ip(p, got, ref):
    n = min(len(got["cost"]), len(ref["cost"]))
    # pred = 0 exactly: the LQ step failed (R + B'S'B not positive definite) and
    # both runs reject; a positive pred below 1e-9 |J| is a round-off decision
    soft = (ref["pred"][:n] != 0.0) & (np.abs(ref["pred"][:n]) <= 1e-9 * np.abs(ref["cost"][:n]))
    first = int(np.argmax(soft)) if soft.any() else n
    assert first >= 5
    assert np.array_equal(got["accept"][:first], ref["accept"][:first])
    assert rel(got["cost"][:first], ref["cost"][:first]) < 2e-7
    last_level = np.sum(got["level_iters"]) - got["level_iters"][-1]
    assert got["grad"][-1] <= W.IP_TOL or got["level_iters"][-1] == W.IP_MAX_ITER
    eJ = abs(got["cost"][-1] - ref["cost"][-1]) / max(1.0, abs(ref["cost"][-1]))
    eu, ex = rel(got["u"], ref["u"]), rel(got["x"], ref["x"])
    print(f"first round-off decision at {first} of {len(ref['cost'])}; levels {got['level_iters']} vs "
          f"{ref['level_iters']}; final J rel {eJ:.1e}, u {eu:.1e}, x {ex:.1e}")
    assert last_level >= 0
    assert eJ < 1e-7
    assert eu < 1e-5 and ex < 1e-5
    assert np.all(got["u"] < p.umax) and np.all(got["u"] > p.umin)


@pytest.mark.parametrize("name", sorted(MODELS))
def test_interior_point_sequential_mode_matches_oracle(lq, name):
    """The sequential-in-time path (one segment per instance) on the same solve."""
    p = MODELS[name](100)
    got, ref = ip(lq, p, mode="sequential")
    check_ip(p, got, ref)


# --------------------------------------------------------------------------
# ADMM (Sec. II-C)
# --------------------------------------------------------------------------

def admm_state(p, seed, rho=0.7):
    rng = np.random.default_rng(seed)
    z = -np.abs(rng.standard_normal((p.T, 2 * p.nu)))
    v = np.abs(rng.standard_normal((p.T, 2 * p.nu)))
    return {"rho": rho, "z": z, "v": v}


def gpu_with_admm(lq, p, admm, **kw):
    s = lq.NewtonMPC(p, **kw)
    z = torch.as_tensor(admm["z"].reshape(-1), dtype=torch.float64, device="cuda").contiguous()
    v = torch.as_tensor(admm["v"].reshape(-1), dtype=torch.float64, device="cuda").contiguous()
    s.prob_c.admm_rho = admm["rho"]
    s.prob_c.admm_z = z.data_ptr()
    s.prob_c.admm_v = v.data_ptr()
    return s, z, v


@pytest.mark.parametrize("name", sorted(MODELS))
@pytest.mark.parametrize("seg_len", [0, 3])
def test_admm_newton_step(lq, name, seg_len):
    """One Newton step on J_AD (augmentation instead of barrier; a control outside the box)."""
    import dataclasses
    p = MODELS[name](61)
    u0 = p.u0 * 5.0
    u0[7, 0] = 1.1 * p.umax
    p = dataclasses.replace(p, u0=u0, Q=np.eye(p.nx) * 0.2)
    admm = admm_state(p, 3)
    alpha, nu = 0.05, 2.0
    x0 = oracle.nmpc_rollout(p, p.u0)
    acc, x1, u1, a1, nu1, cost, pred, rho, grad = oracle.nmpc_newton_step(p, x0, p.u0, 0.0, alpha, nu,
                                                                          with_grad=True, admm=admm)
    s, z, v = gpu_with_admm(lq, p, admm, seg_len=seg_len)
    s.init(alpha, nu)
    s.step(0.0)
    torch.cuda.synchronize()
    sc = s.scal.cpu().numpy()
    assert bool(sc[lq.NMPC_ACCEPTED] > 0.5) == acc
    assert abs(sc[lq.NMPC_PRED] - pred) <= 1e-10 * abs(pred)
    assert abs(sc[lq.NMPC_COST] - cost) <= 1e-10 * abs(cost)
    assert abs(sc[lq.NMPC_GRAD] - grad) <= 1e-10 * abs(grad)
    assert rel(s.u.cpu().numpy().reshape(p.T, p.nu), u1) < 1e-10
    assert rel(s.x.cpu().numpy().reshape(p.T + 1, p.nx), x1) < 1e-10


@pytest.mark.parametrize("init", [1, 0])
def test_admm_update_matches_oracle(lq, init):
    """The consensus / multiplier step: z bit for bit (a projection of the same sums), v and
    both residual norms to round-off (the GPU contracts v + rho (w - z) into one fused
    multiply-add, the oracle rounds twice; for inactive rows v is the cancellation
    v + rho (w - (w + v / rho)) of a few ulp of rho |w|), with controls inside, on and
    outside the box."""
    p = W.cartpole_problem(300)
    rng = np.random.default_rng(9)
    u = rng.uniform(-1.3 * p.umax, 1.3 * p.umax, (p.T, p.nu))
    u[5, 0] = p.umax
    admm = admm_state(p, 10, rho=0.37)
    zr, vr, rp, rd = oracle.nmpc_admm_update(p, u, admm["z"], admm["v"], admm["rho"], init)
    s, z, v = gpu_with_admm(lq, p, admm)
    s.u.copy_(torch.as_tensor(u.reshape(-1), dtype=torch.float64))
    lq.nmpc_admm_update(s.plan, s.prob_c, s.state_c, init)
    torch.cuda.synchronize()
    assert np.array_equal(z.cpu().numpy().reshape(p.T, -1), zr)
    vg = v.cpu().numpy().reshape(p.T, -1)
    w = np.concatenate([u - p.umax, p.umin - u], axis=1)
    scale = admm["rho"] * np.abs(w) + np.abs(admm["v"])
    assert np.all(np.abs(vg - vr) <= 8 * np.finfo(float).eps * scale)
    if not init:
        sc = s.scal.cpu().numpy()
        assert abs(sc[lq.NMPC_RP] - rp) <= 1e-14 * max(rp, 1.0) and abs(sc[lq.NMPC_RD] - rd) <= 1e-14 * max(rd, 1.0)


@pytest.mark.parametrize("name,N", [("pendulum", 40), ("pendulum", 400), ("cartpole", 20)])
def test_admm_solve_matches_oracle(lq, name, N):
    """Whole ADMM solves: the same number of ADMM iterations and the same final
    trajectory (ADMM's inner loops end far above round-off, see the IP tests), the
    invariants z <= 0, v >= 0, v z = 0, and residuals within eps."""
    p = MODELS[name](N)
    args = dict(rho=W.ADMM_RHO[name] * p.h, eps=W.ADMM_EPS, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                max_admm=W.ADMM_MAX_ITER, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    ref = oracle.nmpc_admm_solve(p, **args)
    got = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN).admm_solve(**args)
    print(f"{name} N={N}: ADMM {got['admm_iters']} vs {ref['admm_iters']}, Newton {got['newton_iters']} vs "
          f"{ref['newton_iters']}, u {rel(got['u'], ref['u']):.1e}")
    assert got["admm_iters"] == ref["admm_iters"]
    assert rel(got["u"], ref["u"]) < 1e-5 and rel(got["x"], ref["x"]) < 1e-5
    assert np.all(got["z"] <= 0.0) and np.all(got["v"] >= 0.0) and np.all((got["v"] == 0) | (got["z"] == 0))
    assert got["rp"][-1] <= W.ADMM_EPS and got["rd"][-1] <= W.ADMM_EPS


@pytest.mark.parametrize("name", sorted(MODELS))
def test_graph_replayed_solves_equal_eager(lq, name):
    """ip_solve and admm_solve replaying captured newton_step graphs (with the host's
    eager writes and readbacks between replays; ADMM's inner levels ended by the host
    or, in chunks of 2 to 4 steps, on the device) give the eager results bit for bit."""
    p = MODELS[name](60)
    args = dict(mu0=W.IP_MU0, zeta=W.IP_ZETA, mu_min=W.IP_MU_MIN, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    s = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN)
    e = s.ip_solve(**args, graph=False)
    g = s.ip_solve(**args, graph=True)
    assert np.array_equal(e["level_iters"], g["level_iters"])
    assert np.array_equal(e["cost"], g["cost"]) and np.array_equal(e["grad"], g["grad"])
    assert np.array_equal(e["u"], g["u"]) and np.array_equal(e["x"], g["x"])
    aargs = dict(rho=W.ADMM_RHO[name] * p.h, eps=W.ADMM_EPS, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                 max_admm=40, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    ea = s.admm_solve(**aargs, graph=False)
    for chunk in ("auto", 1, 3):
        ga = s.admm_solve(**aargs, graph=True, chunk=chunk)
        assert ea["admm_iters"] == ga["admm_iters"] and np.array_equal(ea["inner"], ga["inner"])
        assert np.array_equal(ea["rp"], ga["rp"]) and np.array_equal(ea["u"], ga["u"])


def test_solves_keep_their_graphs_while_the_problem_is_unchanged(lq):
    """ip_solve captures its chunk graph on the first solve and replays that graph
    on later solves of the same problem, bit for bit equal, also after an
    admm_solve that changes the problem struct and restores it; admm_solve keeps
    its single-step graph the same way.  A changed problem struct (a model
    parameter here) is captured again, and its solve equals that of a fresh
    solver built with the new parameter."""
    import dataclasses
    p = MODELS["pendulum"](60)
    args = dict(mu0=W.IP_MU0, zeta=W.IP_ZETA, mu_min=W.IP_MU_MIN, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    aargs = dict(rho=W.ADMM_RHO["pendulum"] * p.h, eps=W.ADMM_EPS, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                 max_admm=40, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)

    def same(a, b):
        assert np.array_equal(a["level_iters"], b["level_iters"]) and np.array_equal(a["cost"], b["cost"])
        assert np.array_equal(a["u"], b["u"]) and np.array_equal(a["x"], b["x"])

    s = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN)
    a = s.ip_solve(**args)
    g1 = s._chunk_graph
    same(a, s.ip_solve(**args))
    assert s._chunk_graph is g1
    aa = s.admm_solve(**aargs)
    same(a, s.ip_solve(**args))
    assert s._chunk_graph is g1
    kept = dict(s._step_graphs)
    ab = s.admm_solve(**aargs)
    assert s._step_graphs.keys() == kept.keys() and all(s._step_graphs[k] is g for k, g in kept.items())
    assert np.array_equal(aa["inner"], ab["inner"]) and np.array_equal(aa["rp"], ab["rp"])
    assert np.array_equal(aa["u"], ab["u"]) and np.array_equal(aa["z"], ab["z"]) and np.array_equal(aa["v"], ab["v"])
    prm = np.array(p.param, dtype=np.float64)
    prm[0] *= 1.05
    s.prob_c.param[0] = float(prm[0])
    d = s.ip_solve(**args)
    assert s._chunk_graph is not g1
    same(d, lq.NewtonMPC(dataclasses.replace(p, param=prm), seg_len=W.IP_SEG_LEN).ip_solve(**args))


# --------------------------------------------------------------------------
# Batches and receding-horizon MPC (Sec. V)
# --------------------------------------------------------------------------

def test_batched_newton_matches_single_instances(lq):
    """A batch of pendulum problems that differ in x0 and u0, fixed Newton iterations per
    barrier level: every instance ends where the oracle's single-instance loop does."""
    import dataclasses
    B = 4
    base = W.pendulum_problem(80)
    rng = np.random.default_rng(12)
    x0 = np.stack([rng.uniform(-0.5, 0.5, B), rng.uniform(-0.5, 0.5, B)], axis=1)
    u0 = 0.1 * rng.standard_normal((B, base.T, 1))
    p = dataclasses.replace(base, x0=x0, u0=u0)
    levels, iters = W.MPC_MU_LEVELS[:3], 3
    got = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN).run(levels, iters, W.NMPC_ALPHA0, W.NMPC_NU0)
    for b in range(B):
        pb = dataclasses.replace(base, x0=x0[b], u0=u0[b])
        ref = oracle.nmpc_solve(pb, levels, iters, W.NMPC_ALPHA0, W.NMPC_NU0)
        assert rel(got["u"][b], ref["u"]) < 1e-10
        assert rel(got["x"][b], ref["x"]) < 1e-10


@pytest.mark.parametrize("name,B,steps", [("pendulum", 5, 40), ("cartpole", 3, 30)])
def test_mpc_simulation_matches_oracle(lq, name, B, steps):
    """Batched receding-horizon simulation (one launch sequence for all instances, warm
    start by nmpc_shift): each instance's closed-loop states and applied controls against
    the oracle's sequential simulation, to 1e-6.  Near the upright equilibrium the last
    Newton steps of a barrier level predict decreases at round-off of the cost, where the
    accept decision compares rounding errors; the oracle's own loop with u perturbed by
    1e-15 (relative) after every Newton step spreads the pendulum's closed loop by up to
    4.7e-8 (cart-pole 2e-13) over these cases."""
    xs = W.mpc_initial_states(name, B, seed=21)
    p = W.mpc_problem(name, xs)
    got = lq.NewtonMPC(p).mpc_simulate(steps, mu_levels=W.MPC_MU_LEVELS, iters=W.MPC_ITERS,
                                       alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    worst = 0.0
    for b in range(B):
        ref = oracle.nmpc_mpc_simulate(W.mpc_problem(name, xs[b]), xs[b], steps=steps, mu_levels=W.MPC_MU_LEVELS,
                                       iters=W.MPC_ITERS, alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
        worst = max(worst, rel(got["x"][b], ref["x"]), rel(got["u"][b], ref["u"]))
    print(f"{name}: closed-loop rel diff {worst:.1e}")
    assert worst < 1e-6


@pytest.mark.parametrize("chunk", [2, 3, 7])
def test_device_level_control_equals_host_levels(lq, chunk):
    """ip_solve with the barrier levels ended on the device (graph chunks of 2, 3
    and 7 newton_step calls per read-back, so that levels end inside, at the end
    of and well before the end of a chunk) equals the eager solve, whose levels
    the host ends after every step, bit for bit: the steps past a level's end
    leave the instance unchanged."""
    p = MODELS["pendulum"](60)
    args = dict(mu0=W.IP_MU0, zeta=W.IP_ZETA, mu_min=W.IP_MU_MIN, tol=W.IP_TOL, max_iter=W.IP_MAX_ITER,
                alpha0=W.NMPC_ALPHA0, nu0=W.NMPC_NU0)
    e = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN).ip_solve(**args, graph=False)
    g = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN, level_chunk=chunk).ip_solve(**args, graph=True)
    assert np.array_equal(e["level_iters"], g["level_iters"])
    assert np.array_equal(e["cost"], g["cost"]) and np.array_equal(e["accept"], g["accept"])
    assert np.array_equal(e["u"], g["u"]) and np.array_equal(e["x"], g["x"])


def test_step_after_a_finished_level_is_a_no_op(lq):
    """newton_step with level control: a tolerance every nominal meets ends the
    level after one iteration (LEVEL_DONE = 0.5, LEVEL_ITERS = 1); the next two
    steps change neither the trajectory nor any scalar but LEVEL_DONE (0.5 -> 1)."""
    p = MODELS["cartpole"](50)
    s = lq.NewtonMPC(p, seg_len=W.IP_SEG_LEN)
    s.init(W.NMPC_ALPHA0, W.NMPC_NU0)
    s._sc[:, lq.NMPC_MU] = W.IP_MU0
    s._sc[:, lq.NMPC_LEVEL_TOL] = 1e300
    s._sc[:, lq.NMPC_LEVEL_MAX] = 100.0
    lq.newton_step(s.plan, s.prob_c, s.state_c, s.ws)
    torch.cuda.synchronize()
    sc1, x1, u1 = s.scal.cpu().numpy().copy(), s.x.cpu().numpy().copy(), s.u.cpu().numpy().copy()
    assert sc1[lq.NMPC_LEVEL_DONE] == 0.5 and sc1[lq.NMPC_LEVEL_ITERS] == 1.0
    for _ in range(2):
        lq.newton_step(s.plan, s.prob_c, s.state_c, s.ws)
    torch.cuda.synchronize()
    sc2 = s.scal.cpu().numpy()
    assert sc2[lq.NMPC_LEVEL_DONE] == 1.0
    keep = [i for i in range(lq.NMPC_NSCAL) if i != lq.NMPC_LEVEL_DONE]
    assert np.array_equal(sc1[keep], sc2[keep])
    assert np.array_equal(s.x.cpu().numpy(), x1) and np.array_equal(s.u.cpu().numpy(), u1)


@pytest.mark.parametrize("case,T", [("tanh", 512), ("tanh", 1024), ("pendulum", 100), ("pendulum", 400),
                                    ("pendulum", 1000), ("cartpole", 1000)])
def test_parallel_rollout_matches_sequential(lq, monkeypatch, case, T):
    """One Newton step whose candidate rollout runs in parallel over time
    (Newton on the defects from the LQ step's prediction, T >= 64) against the
    same step with the sequential recursion (LQSCAN_PAR_ROLLOUT=0), from the
    same state after three sequential steps: the same decision, the
    candidate's cost within 1e-12 and the new trajectory within 1e-12
    relative.  (The two differ at rounding level: each satisfies the recursion
    to a few ulps per stage, which unstable dynamics amplify along the horizon,
    and over many Newton steps the decisions of a barrier run may then part at
    a round-off decision, as for any rounding change.)"""
    if case == "tanh":
        p = W.nmpc_problem(seed=3 if T == 512 else 1, T=T)
        mu, seg = 0.1, 0
    else:
        p = MODELS[case](T)
        mu, seg = W.IP_MU0, W.IP_SEG_LEN

    def state(mode):
        monkeypatch.setenv("LQSCAN_PAR_ROLLOUT", "0")
        s = lq.NewtonMPC(p, seg_len=seg)
        s.init(W.NMPC_ALPHA0, W.NMPC_NU0)
        for _ in range(3):
            s.step(mu)
        monkeypatch.setenv("LQSCAN_PAR_ROLLOUT", mode)
        s.step(mu)
        torch.cuda.synchronize()
        return s.scal.cpu().numpy(), s.x.cpu().numpy(), s.u.cpu().numpy()

    sp, xp, up = state("1")
    ss, xs, us = state("0")
    assert sp[lq.NMPC_ACCEPTED] == ss[lq.NMPC_ACCEPTED]
    cp, cs = sp[lq.NMPC_COST_NEW], ss[lq.NMPC_COST_NEW]   # +inf for a candidate outside the box
    assert (cp == cs) if np.isinf(cs) else abs(cp - cs) <= 1e-12 * abs(cs)
    assert rel(xp, xs) < 1e-12 and rel(up, us) < 1e-12
