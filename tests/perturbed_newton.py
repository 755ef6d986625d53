"""The oracle's Newton/IP iteration (Alg. 4 inside the barrier loop of
Sec. II-B, with the damping reading of Sec. III-F) composed in Python from the
oracle's own pieces -- expansion, LQ solve, nonlinear rollout and cost -- so
that the data of each LQ step can be perturbed.

With eps = 0 it takes the same decisions and reaches the same iterates as the
oracle's C loop (pinned by test_mixed_bound.py).  With eps > 0 every entry of
the step's A, B, P and R (and of the resulting du) is multiplied by
1 + eps U(-1, 1): perturbations of the size FP32 arithmetic makes in the
step when eps = 2^-24.  Test infrastructure: it calls only the oracle.
"""
import numpy as np

import oracle

FP32_EPS = 2.0 ** -24


def newton_step(p, x, u, mu, alpha, nu, eps=0.0, rng=None):
    """One iteration from the nominal (x, u); returns a dict with the new
    nominal and damping, the decision, the predicted decrease, the gain ratio
    and the candidate's distance to the box (1 - max |u + du| for |u| <= 1)."""
    J0 = oracle.nmpc_cost(p, u, mu)
    e = oracle.nmpc_expand(p, x, u, mu)
    A, B, P, Rh, d = e["A"], e["B"], e["P"], e["Rh"], e["d"]
    if eps:
        pert = lambda a: a * (1.0 + eps * rng.uniform(-1.0, 1.0, a.shape))
        A, B, P, Rh = pert(A), pert(B), pert(P), pert(Rh)
    reject = dict(accepted=False, x=x, u=u, alpha=alpha * nu, nu=2.0 * nu, cost=J0)
    try:
        o = oracle.lq_solve(A, B, None, P, Rh + alpha * np.eye(p.nu)[None], p.QT, np.zeros(p.nx), r=d)
    except oracle.OracleError:
        return dict(reject, pred=0.0, rho=-np.inf, margin=np.nan)
    dx, du = o["x"], o["u"]
    if eps:
        du = du * (1.0 + eps * rng.uniform(-1.0, 1.0, du.shape))
    pred = -((d * du).sum() + 0.5 * (np.einsum("ki,kij,kj->", dx[:-1], P, dx[:-1])
                                     + np.einsum("ki,kij,kj->", du, Rh, du) + dx[-1] @ p.QT @ dx[-1]))
    un = u + du
    half = 0.5 * (p.umax - p.umin)
    margin = 1.0 - np.max(np.abs(un - 0.5 * (p.umax + p.umin))) / half
    J1 = oracle.nmpc_cost(p, un, mu)
    if pred > 0 and np.isfinite(J1):
        rho = (J0 - J1) / pred
        if rho > 0:
            t = 2.0 * rho - 1.0
            f = 1.0 - t ** 3
            return dict(accepted=True, x=oracle.nmpc_rollout(p, un), u=un, alpha=alpha * max(f, 1.0 / 3.0), nu=2.0,
                        cost=J1, pred=pred, rho=rho, margin=margin)
        return dict(reject, pred=pred, rho=rho, margin=margin)
    return dict(reject, pred=pred, rho=-np.inf, margin=margin)


def run(p, mu_levels, iters, alpha0, nu0, eps=0.0, seed=0):
    """Fixed iterations per barrier level; per-iteration traces and the final u."""
    rng = np.random.default_rng(seed)
    u = np.array(p.u0, dtype=np.float64).reshape(p.T, p.nu)
    x = oracle.nmpc_rollout(p, u)
    alpha, nu = alpha0, nu0
    keys = ("accepted", "cost", "pred", "rho", "margin")
    tr = {k: [] for k in keys}
    for mu in mu_levels:
        for _ in range(iters):
            s = newton_step(p, x, u, mu, alpha, nu, eps, rng)
            x, u, alpha, nu = s["x"], s["u"], s["alpha"], s["nu"]
            for k in keys:
                tr[k].append(s[k])
    out = {k: np.array(v) for k, v in tr.items()}
    out["u"], out["x"] = u, x
    return out


# Final-cost bound of the mixed-precision Newton/IP run on the tanh benchmark
# (60 iterations, T = 1024), relative to the FP64 oracle.  Derived from the
# spread of runs(): 24 runs with FP32-sized perturbations (eps = 2^-24) of every
# LQ step end up to 4.52e-3 from the unperturbed run (three clusters: below
# 5e-8 with no or late flips, 4e-6 to 1.08e-5 with four or five flipped
# decisions from iteration 36, 4.52e-3 with ten flips from iteration 40).
# The flips are feasibility decisions: at those iterations the FP64
# candidate u + du lies 6e-11 to 1.2e-7 from the box, inside what the step's
# rounding moves it.  The bound is that maximum, rounded up.
MIXED_NEWTON_BOUND = 5e-3
