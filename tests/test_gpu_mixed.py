"""Mixed precision (FP32 products; FP64 inverses, Cholesky factors and
symmetrisation) against the FP64 oracle, at the stated bounds:
x, u, S <= 1e-4 and gradients <= 1e-3 (normwise relative); Newton/IP final
cost within the spread FP32-sized perturbations give the oracle's own run on
the tanh benchmark (the proposed 1e-5 is below that spread, see
test_mixed_newton) and stationarity of the final iterate on a converging
instance.  The measured errors are printed."""
import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_20027_amd import lqscan
    return lqscan


def rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


@pytest.mark.parametrize("T", [64, 16384])
def test_mixed_long_horizon(lq, T):
    inst = W.cfg2_long(T=T) if T > 64 else W.cfg0_small()
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([inst.n], [inst.m], [inst.T], precision="mixed")
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    n, m = inst.n, inst.m
    ex = rel(out["x"].cpu().numpy().reshape(T + 1, n), ref["x"])
    eu = rel(out["u"].cpu().numpy().reshape(T, m), ref["u"])
    eS = rel(out["S"].cpu().numpy().reshape(T + 1, n, n), ref["S"])
    print(f"mixed T={T}: x {ex:.2e} u {eu:.2e} S {eS:.2e}")
    assert ex <= 1e-4 and eu <= 1e-4 and eS <= 1e-4
    S = out["S"].cpu().numpy().reshape(T + 1, n, n)
    assert np.array_equal(S, np.transpose(S, (0, 2, 1)))   # symmetrised in FP64


def test_mixed_adjoint(lq):
    inst = W.cfg2_long(T=2048)
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([inst.n], [inst.m], [inst.T], precision="mixed")
    out = lq.solve(plan, prob)
    names = ("A", "B", "c", "Q", "R", "QT", "x0")
    g = lq.grad_buffers(plan, names)
    ws = plan.new_workspace()
    lq.lq_adjoint(plan, prob, {k: out[k] for k in ("S", "s", "Gamma", "gamma")}, out["x"], out["u"], out["lam"],
                  2 * out["x"], 2 * out["u"], g, ws, out["status"])
    torch.cuda.synchronize()
    o = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    ref = oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * o["x"], 2 * o["u"])
    errs = {f: rel(g[f].cpu().numpy().reshape(ref[f].shape), ref[f]) for f in names}
    print("mixed adjoint errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-3


def test_mixed_newton(lq):
    """Benchmark tanh problem (unstable, saturating; 60 iterations do not
    converge it) with FP32 LQ steps, against the FP64 oracle.  The proposed
    final-cost bound of 1e-5 cannot hold for any FP32 path: from iteration 36
    on the candidates lie within 1e-7 of the control box, their feasibility is
    decided at rounding level, and the oracle's own run with FP32-sized
    perturbations of its LQ steps ends up to 4.5e-3 away
    (test_mixed_bound.py).  Asserted: the final cost within that spread
    (perturbed_newton.MIXED_NEWTON_BOUND), and the first decision that differs
    from the oracle's taken where the oracle's candidate is within 1e-6 of
    the box; every differing decision is printed with the oracle's predicted
    decrease, gain ratio and box margin."""
    import perturbed_newton as PN
    p = W.nmpc_problem(seed=1, T=1024)
    args = (W.NMPC_MU_LEVELS, W.NMPC_ITERS_PER_LEVEL, W.NMPC_ALPHA0, W.NMPC_NU0)
    ref = PN.run(p, *args)
    got = lq.NewtonMPC(p, precision="mixed").run(*args)
    mism = np.nonzero(got["accept"] != ref["accepted"])[0]
    for it in mism:
        print(f"iteration {it}: oracle {'accept' if ref['accepted'][it] else 'reject'} "
              f"(pred/|J| {ref['pred'][it] / abs(ref['cost'][it]):.2e}, rho {ref['rho'][it]:.4g}, "
              f"box margin {ref['margin'][it]:.2e}), mixed GPU pred {got['pred'][it]:.3e} rho {got['rho'][it]:.4g}")
    ec = abs(got["cost"][-1] - ref["cost"][-1]) / abs(ref["cost"][-1])
    first = int(mism[0]) if len(mism) else len(ref["cost"])
    pre = np.max(np.abs(got["cost"][:first] - ref["cost"][:first]) / np.abs(ref["cost"][:first])) if first else 0.0
    print(f"mixed newton: final cost rel err {ec:.2e}, decision mismatches {len(mism)}/{len(ref['cost'])}, "
          f"cost trace before the first mismatch within {pre:.2e}")
    assert np.all(np.abs(got["u"]) < 1.0)
    assert ec <= PN.MIXED_NEWTON_BOUND
    if len(mism):
        assert ref["margin"][first] < 1e-6


def test_mixed_newton_converges_to_fp64_optimum(lq):
    """On an instance the loop converges, FP32 Hessian products with FP64
    gradients head for the FP64 optimum: the fixed point of the iteration is
    dJ_mu/du = 0 evaluated in FP64.  The final iterate depends on rounding
    through the accept/reject decisions taken at round-off (the FP64 test of
    the same instance gives the spread: stationarity up to 1.1e-5 of its value
    at u0, u up to 7.9e-5 apart).  Asserted: stationarity of the final iterate
    (measured by the oracle's FP64 expansion) below 1e-4 of its value at u0,
    and agreement with the FP64 run to 1e-3."""
    from test_gpu_newton import barrier_gradient, benign_problem
    p = benign_problem()
    ref = oracle.nmpc_solve(p, W.NMPC_MU_LEVELS, W.NMPC_ITERS_PER_LEVEL, W.NMPC_ALPHA0, W.NMPC_NU0)
    got = lq.NewtonMPC(p, precision="mixed").run(W.NMPC_MU_LEVELS, W.NMPC_ITERS_PER_LEVEL, W.NMPC_ALPHA0,
                                                 W.NMPC_NU0)
    mu = W.NMPC_MU_LEVELS[-1]
    g0 = barrier_gradient(p, p.u0, mu)
    g_got = barrier_gradient(p, got["u"].reshape(p.T, p.nu), mu)
    eu = rel(got["u"], ref["u"])
    print(f"mixed newton (converging instance): |dJ/du| {g_got:.2e} (u0: {g0:.2e}), final u rel err {eu:.2e}")
    assert g_got <= 1e-4 * g0
    assert eu <= 1e-3


@pytest.mark.parametrize("seed", range(6))
def test_mixed_random_configurations(lq, seed):
    """The mixed-precision plan on seeded random sizes, segment lengths and
    optional terms, to the mixed bound 1e-4 (a sweep of 100 such
    configurations peaks at 9e-7)."""
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location("_lqtests", os.path.join(os.path.dirname(__file__), "test_gpu_lq.py"))
    t = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(t)
    inst, L = t.random_config(np.random.default_rng(90000 + seed))
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([inst.n], [inst.m], [inst.T], seg_lens=[L], precision="mixed")
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0,
                          M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
    n, m, T = inst.n, inst.m, inst.T
    assert rel(out["x"].cpu().numpy().reshape(T + 1, n), ref["x"]) <= 1e-4
    assert rel(out["u"].cpu().numpy().reshape(T, m), ref["u"]) <= 1e-4
    assert rel(out["S"].cpu().numpy().reshape(T + 1, n, n), ref["S"]) <= 1e-4
