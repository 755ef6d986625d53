"""Failure injection through the C ABI: host-built inputs whose solve must
report a numerical failure in the per-instance status word
(-code) | (stage << 8), with the other instances of a ragged batch unaffected.
None of these inputs makes a kernel fault: the kernels run to completion and
only the status (and the failed instance's results) change.

* A NaN in one entry of any stage array (A, B, c, Q, R, M, q, r) gives
  LQ_ERR_NONFINITE at that stage; in Q_T at stage T.  The Bellman sweep visits
  every stage and every entry of a stage's data reaches S~_k there, so the
  stage is exact whatever segment it falls in.
* A scan combination with a singular I + C J: n = m = 1, A = B = R = 1, so the
  stage element has C = 1, and Q_6 = -1, so that with one stage per segment the
  first scan level combines entry 5 (C = 1) with entry 6 (J = -1) into
  X = 1 + 1 * (-1) = 0 exactly: LQ_ERR_SINGULAR at stage 5.  The sequential
  recursion of the same problem has R + B'S'B > 0 at every stage (S_6 lies in
  (-1, 0)), so it reports nothing: the failure belongs to the association
  order of the scan, not to the problem.
"""
import numpy as np
import pytest

from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NOT_PD, SINGULAR, NONFINITE = 2, 3, 4


@pytest.fixture(scope="module")
def lq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_20027_amd import lqscan
    return lqscan


def code_of(word):
    return (int(word) & 0xFF, int(word) >> 8)


def solve_status(lq, insts, _fused=True, **plan_kw):
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], **plan_kw)
    out = lq.solve(plan, prob, fused=_fused)
    torch.cuda.synchronize()
    return out


def general(seed, n=4, m=2, T=200):
    return W.lq_instance_general(np.random.default_rng(seed), n, m, T)


@pytest.mark.parametrize("k", [0, 5, 15, 16, 37, 199])
@pytest.mark.parametrize("plan_kw", [dict(seg_len=16), dict(seg_len=16, precision="mixed"), dict(mode="sequential")],
                         ids=["scan", "mixed", "sequential"])
def test_nan_in_A_reports_nonfinite_at_its_stage(lq, k, plan_kw):
    """k covers segment 0 (whose element the scan never forms), the last and
    first stage of a segment, the middle of one, and the last stage."""
    inst = general(300)
    inst.A = inst.A.copy()
    inst.A[k, 1, 2] = np.nan
    out = solve_status(lq, [inst], **plan_kw)
    assert code_of(out["status"][0]) == (NONFINITE, k)


@pytest.mark.parametrize("field", ["A", "B", "c", "Q", "R", "M", "q", "r"])
def test_nan_in_any_stage_array(lq, field):
    inst = general(301)
    k = 77
    arr = getattr(inst, field).copy()
    arr[k].reshape(-1)[-1] = np.nan
    setattr(inst, field, arr)
    out = solve_status(lq, [inst], seg_len=8)
    assert code_of(out["status"][0]) == (NONFINITE, k), field


@pytest.mark.parametrize("value", [np.nan, np.inf])
def test_nonfinite_terminal_cost(lq, value):
    inst = general(302)
    inst.QT = inst.QT.copy()
    inst.QT[0, 0] = value
    out = solve_status(lq, [inst], seg_len=16)
    assert code_of(out["status"][0]) == (NONFINITE, inst.T)


def singular_instance(T=40):
    """n = m = 1: A = B = R = Q_T = 1, Q = 1 except Q_6 = -1, c = 0, x0 = 1."""
    one = np.ones((T, 1, 1))
    Q = one.copy()
    Q[6] = -1.0
    return W.LQInstance(1, 1, T, one.copy(), one.copy(), np.zeros((T, 1)), Q, one.copy(), np.eye(1), np.ones(1))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("fused", [False, True], ids=["lq_scan_solve", "lq_solve"])
def test_singular_scan_combination(lq, precision, fused):
    inst = singular_instance()
    out = solve_status(lq, [inst], seg_len=1, precision=precision, _fused=fused)
    assert code_of(out["status"][0]) == (SINGULAR, 5)


def test_singular_combination_is_absent_from_the_sequential_recursion(lq):
    """The same problem solved sequentially: no failure, and the solution is
    the oracle's (the stage-6 value matrix is negative, the problem convex in u)."""
    import oracle
    inst = singular_instance()
    out = solve_status(lq, [inst], mode="sequential")
    assert int(out["status"][0]) == 0
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    assert ref["S"][6, 0, 0] < 0
    x = out["x"].cpu().numpy().reshape(inst.T + 1, 1)
    assert np.max(np.abs(x - ref["x"])) <= 1e-12 * np.max(np.abs(ref["x"]))


def test_failed_instances_leave_the_rest_of_a_ragged_batch_unchanged(lq):
    """A ragged batch with a NaN instance and a singular-combination instance
    among healthy ones: the two report their failures, every other instance
    has status 0 and results bit-identical to the batch without the two."""
    rng = np.random.default_rng(303)
    healthy = [W.lq_instance(rng, n, max(1, n // 3), T) for n, T in
               ((2, 64), (12, 300), (4, 33), (1, 40), (12, 1000), (4, 129))]
    bad_nan = general(304, 4, 1, 150)
    bad_nan.c = bad_nan.c.copy()
    bad_nan.c[90, 3] = np.nan
    bad_sing = singular_instance()
    mixed_batch = healthy[:2] + [bad_nan] + healthy[2:4] + [bad_sing] + healthy[4:]
    # one stage per segment for every instance, so the singular combination is formed
    out_bad = solve_status(lq, mixed_batch, seg_lens=[1] * len(mixed_batch))
    out_ok = solve_status(lq, healthy, seg_lens=[1] * len(healthy))
    st = out_bad["status"].cpu().numpy()
    assert code_of(st[2]) == (NONFINITE, 90)
    assert code_of(st[5]) == (SINGULAR, 5)
    assert int(np.abs(np.delete(st, [2, 5])).sum()) == 0
    assert int(out_ok["status"].abs().sum()) == 0

    def pieces(out, insts, key, shape):
        flat, o, res = out[key].cpu().numpy(), 0, []
        for i in insts:
            k = int(np.prod(shape(i)))
            res.append(flat[o:o + k])
            o += k
        return res

    shapes = {"x": lambda i: (i.T + 1) * i.n, "u": lambda i: i.T * i.m, "S": lambda i: (i.T + 1) * i.n * i.n,
              "Gamma": lambda i: i.T * i.m * i.n}
    keep = [j for j in range(len(mixed_batch)) if j not in (2, 5)]
    for key, shp in shapes.items():
        got = pieces(out_bad, mixed_batch, key, shp)
        ref = pieces(out_ok, healthy, key, shp)
        for j, r in zip(keep, ref):
            assert np.array_equal(got[j], r), (key, j)
