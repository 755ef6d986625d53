"""GPU parity: the conditional-value rollout (lq_rollout_cv) against the FP64 oracle.

The states are compared with the oracle's states from the prefix conditional
value functions (eq:value-fun-prefix-sum), the controls and co-states with the
oracle's Riccati solution.  Tolerance: normwise relative error <= 1e-10 per
output array and instance (the FP64 bar of the other LQ parity tests).
"""
import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def lq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_20027_amd import lqscan
    return lqscan


def rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def split(flat, shapes):
    out, o = [], 0
    for shp in shapes:
        k = int(np.prod(shp))
        out.append(flat[o:o + k].reshape(shp))
        o += k
    return out


def run(lq, insts, rollout="cv", **plan_kw):
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], **plan_kw)
    out = lq.solve(plan, prob, rollout=rollout)
    torch.cuda.synchronize()
    x = split(out["x"].cpu().numpy(), [(i.T + 1, i.n) for i in insts])
    u = split(out["u"].cpu().numpy(), [(i.T, i.m) for i in insts])
    lam = split(out["lam"].cpu().numpy(), [(i.T + 1, i.n) for i in insts])
    return x, u, lam, out["status"].cpu().numpy(), plan


def check(insts, x, u, lam, tol=TOL):
    worst = 0.0
    for inst, xi, ui, li in zip(insts, x, u, lam):
        args = (inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
        kw = dict(M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
        xc = oracle.lq_states_cv(*args, **kw)
        ref = oracle.lq_solve(*args, **kw)
        for name, got, want in (("x", xi, xc), ("u", ui, ref["u"]), ("lam", li, ref["lam"])):
            e = rel(got, want)
            worst = max(worst, e)
            assert e <= tol, f"{name}: rel err {e:.3e} (n={inst.n}, m={inst.m}, T={inst.T})"
    return worst


@pytest.mark.parametrize("n,m,T,L", [(3, 2, 37, 5), (4, 4, 50, 8), (1, 1, 9, 2), (15, 4, 40, 6),
                                     (5, 2, 64, 1), (6, 3, 33, 32), (2, 1, 1, 1)])
def test_cv_general_all_terms(lq, n, m, T, L):
    """Every optional term present; segment lengths from one stage to nearly T,
    ragged last segments, n up to 15 (four contraction slices)."""
    inst = W.lq_instance_general(np.random.default_rng(2000 + 10 * n + m), n, m, T)
    x, u, lam, status, _ = run(lq, [inst], seg_len=L)
    assert int(np.abs(status).sum()) == 0
    check([inst], x, u, lam)
    assert np.array_equal(x[0][0], inst.x0)


def test_cv_ragged_batch_per_instance_segments(lq):
    """Instances of mixed sizes in one plan, with the scan at several segment
    lengths and the sequential recursion (one segment)."""
    rng = np.random.default_rng(21)
    dims = [(12, 4, 300), (4, 1, 77), (2, 1, 50), (12, 4, 64), (7, 3, 129), (1, 1, 3)]
    insts = [W.lq_instance(rng, n, m, T) for n, m, T in dims]
    insts.append(W.lq_instance_general(rng, 5, 2, 41))
    seg = [7, 77, 1, 0, 16, 2, 4]
    x, u, lam, status, _ = run(lq, insts, seg_lens=seg)
    assert int(np.abs(status).sum()) == 0
    check(insts, x, u, lam)


def test_cv_equals_affine_rollout(lq):
    """The two rollouts of the same value pass agree to round-off."""
    inst = W.lq_instance_general(np.random.default_rng(22), 8, 3, 500)
    xa, ua, la, _, _ = run(lq, [inst], rollout="affine", seg_len=9)
    xc, uc, lc, status, _ = run(lq, [inst], rollout="cv", seg_len=9)
    assert int(np.abs(status).sum()) == 0
    assert rel(xc[0], xa[0]) < TOL and rel(uc[0], ua[0]) < TOL and rel(lc[0], la[0]) < TOL


def test_cv_full_horizon(lq):
    """n=12, m=4, T=16384 at the default segment length, every stage compared."""
    inst = W.cfg2_long()
    x, u, lam, status, plan = run(lq, [inst])
    assert int(np.abs(status).sum()) == 0
    worst = check([inst], x, u, lam)
    print(f"cv full horizon worst rel err {worst:.3e}, seg_len {plan.seg_len()}")


def test_cv_mixed_precision(lq):
    """The mixed-precision plan on the same path, to the mixed-precision bound
    of the affine rollout (1e-4)."""
    inst = W.lq_instance(np.random.default_rng(23), 12, 4, 1000)
    x, u, lam, status, _ = run(lq, [inst], precision="mixed")
    assert int(np.abs(status).sum()) == 0
    check([inst], x, u, lam, tol=1e-4)
