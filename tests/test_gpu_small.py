"""GPU parity of the per-lane path for small state dimensions (n <= 4, every
m <= 4): the value fold, value-scan levels, Bellman sweep with the rollout's
segment maps, affine-scan levels and rollout apply of lq_small.hip, against
the FP64 oracle (1e-10 normwise relative per output array and instance), and
against the matrix-core tile path (LQSCAN_SMALL=0) on the same inputs.

Plans whose instances span several size classes are split into one sub-plan
per class; the mixed ragged batches here check that every instance is solved
by its class's kernels into the caller's packing and status words.
"""
import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
KEYS = ("S", "s", "Gamma", "gamma", "x", "u", "lam")
SHAPES = {"S": lambda i: (i.T + 1, i.n, i.n), "s": lambda i: (i.T + 1, i.n), "Gamma": lambda i: (i.T, i.m, i.n),
          "gamma": lambda i: (i.T, i.m), "x": lambda i: (i.T + 1, i.n), "u": lambda i: (i.T, i.m),
          "lam": lambda i: (i.T + 1, i.n)}


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


def solve(lq, insts, fused=True, **plan_kw):
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], **plan_kw)
    out = lq.solve(plan, prob, fused=fused)
    torch.cuda.synchronize()
    res = {k: out[k].cpu().numpy() for k in KEYS}
    per = [dict() for _ in insts]
    for k in KEYS:
        for j, a in enumerate(split(res[k], [SHAPES[k](i) for i in insts])):
            per[j][k] = a
    return per, out["status"].cpu().numpy()


def check(per, insts, tol=TOL):
    worst = 0.0
    for got, inst in zip(per, insts):
        ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0,
                              M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
        for k in KEYS:
            e = rel(got[k], ref[k])
            worst = max(worst, e)
            assert e <= tol, f"{k}: {e:.3e} (n={inst.n}, m={inst.m}, T={inst.T})"
    return worst


@pytest.mark.parametrize("n", [1, 2, 3, 4])
@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_every_small_size(lq, n, m):
    """Each compiled (n, m) at T = 1, 2 and 37 stages (odd segment counts and a
    ragged last segment at L = 3), plain and with every cross term."""
    rng = np.random.default_rng(100 * n + m)
    insts = [W.lq_instance(rng, n, m, T) for T in (1, 2, 37)]
    insts += [W.lq_instance_general(rng, n, m, T) for T in (1, 2, 37)]
    print(f"small path n={n} m={m}", flush=True)
    for L in (0, 1, 3):
        per, st = solve(lq, insts, seg_len=L)
        assert not st.any()
        check(per, insts)


@pytest.mark.parametrize("T,L", [(64, 4), (1000, 16), (4096, 16), (2048, 64), (777, 7)])
def test_small_long_horizons(lq, T, L):
    """Segment counts from 16 to 257 (value-scan levels up to 8), n = 2 and 4."""
    rng = np.random.default_rng(T + L)
    insts = [W.lq_instance(rng, 2, 1, T), W.lq_instance(rng, 4, 1, T), W.lq_instance_general(rng, 3, 2, T)]
    per, st = solve(lq, insts, seg_len=L)
    assert not st.any()
    check(per, insts)


@pytest.mark.parametrize("fused", [True, False])
def test_mixed_class_ragged_batch(lq, fused):
    """Size classes (1,1), (2,1), (4,1), (4,2), (3,3) and two tile-path sizes
    (5 and 12) interleaved in one batch: every instance against the oracle."""
    rng = np.random.default_rng(7)
    sizes = [(2, 1, 300), (12, 4, 129), (4, 1, 1), (1, 1, 50), (5, 2, 77), (4, 2, 513), (2, 1, 2), (3, 3, 91),
             (4, 1, 64), (12, 4, 1)]
    insts = [W.lq_instance(rng, n, m, T) if j % 2 else W.lq_instance_general(rng, n, m, T)
             for j, (n, m, T) in enumerate(sizes)]
    per, st = solve(lq, insts, fused=fused)
    assert not st.any()
    check(per, insts)


def test_small_path_matches_tile_path(lq, monkeypatch):
    """The per-lane kernels and the matrix-core tile kernels on the same ragged
    batch of small instances agree to 1e-12 (different association orders of
    the same arithmetic)."""
    rng = np.random.default_rng(8)
    insts = [W.lq_instance(rng, n, 1, T) for n, T in ((2, 700), (4, 1300), (3, 5))]
    insts.append(W.lq_instance_general(rng, 4, 3, 400))
    a, sa = solve(lq, insts)
    monkeypatch.setenv("LQSCAN_SMALL", "0")
    b, sb = solve(lq, insts)
    assert not sa.any() and not sb.any()
    for ga, gb in zip(a, b):
        for k in KEYS:
            assert rel(ga[k], gb[k]) < 1e-12, k


@pytest.mark.parametrize("n,m,Ts,L", [(2, 1, [1000], 4), (1, 1, [200, 37, 5], 3), (2, 2, [300, 64, 2, 129], 5),
                                      (2, 1, [1], 1), (4, 1, [1000], 4), (3, 2, [77, 5], 3), (4, 1, [796], 4),
                                      (3, 1, [1000, 47], 3), (4, 2, [9, 1, 40], 2), (1, 1, [2044], 4)])
def test_one_block_scans_equal_per_level(lq, monkeypatch, n, m, Ts, L):
    """Classes with at most 512 scan entries run every level of the rollout's
    affine scan in one workgroup, and so does the value scan up to its cap
    (512 entries at n <= 2, 352 at n = 3, 200 at n = 4): entries in LDS, a
    barrier between levels, the same arithmetic as the per-level launches
    (LQSCAN_SCAN1=0), so both agree to rounding and both match the oracle.
    Entry counts 251, 85, 104, 2, 251 (above the n = 4 cap: the affine scans
    only), 30, 200 (the n = 4 cap), 352 (the n = 3 cap), 29 and 512."""
    rng = np.random.default_rng(40 + n + len(Ts))
    insts = [W.lq_instance_general(rng, n, m, T) if j % 2 else W.lq_instance(rng, n, m, T) for j, T in enumerate(Ts)]
    a, sa = solve(lq, insts, seg_len=L)
    monkeypatch.setenv("LQSCAN_SCAN1", "0")
    b, sb = solve(lq, insts, seg_len=L)
    assert not sa.any() and not sb.any()
    check(a, insts)
    for ga, gb in zip(a, b):
        for k in KEYS:
            assert rel(ga[k], gb[k]) < 1e-14, k


def test_mixed_precision_plan_on_small_sizes(lq):
    """A mixed-precision plan of small instances (the per-lane path computes in
    FP64): within the mixed bound, in fact within the FP64 bound."""
    rng = np.random.default_rng(9)
    insts = [W.lq_instance(rng, 2, 1, 900), W.lq_instance(rng, 4, 1, 333)]
    per, st = solve(lq, insts, precision="mixed")
    assert not st.any()
    check(per, insts, tol=1e-10)


def test_adjoint_and_checkpoint_through_mixed_classes(lq):
    """lq_adjoint and the checkpointed adjoint (strides 1 and 3) on a batch
    that mixes per-lane and tile classes: gradients against the oracle."""
    rng = np.random.default_rng(10)
    insts = [W.lq_instance_general(rng, 2, 1, 61), W.lq_instance(rng, 12, 4, 90), W.lq_instance_general(rng, 4, 2, 33),
             W.lq_instance(rng, 1, 1, 7)]
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], seg_len=4)
    names = ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")
    refs = []
    for inst in insts:
        o = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, M=inst.M, q=inst.q, r=inst.r,
                            qT=inst.qT)
        refs.append(oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * o["x"],
                                      2 * o["u"], M=inst.M, q=inst.q, r=inst.r, qT=inst.qT))
    gshape = {"A": lambda i: (i.T, i.n, i.n), "B": lambda i: (i.T, i.n, i.m), "c": lambda i: (i.T, i.n),
              "Q": lambda i: (i.T, i.n, i.n), "R": lambda i: (i.T, i.m, i.m), "M": lambda i: (i.T, i.n, i.m),
              "q": lambda i: (i.T, i.n), "r": lambda i: (i.T, i.m), "QT": lambda i: (i.n, i.n),
              "qT": lambda i: (i.n,), "x0": lambda i: (i.n,)}
    for mode in ("stored", 1, 3):
        status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
        val, st = lq.value_buffers(plan), lq.state_buffers(plan)
        g = lq.grad_buffers(plan, names)
        if mode == "stored":
            ws = plan.new_workspace()
            lq.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
            lq.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], 2 * st["x"], 2 * st["u"], g, ws, status)
        else:
            ck = plan.new_checkpoint(mode)
            lq.lq_solve_ckpt(plan, prob, None, val, st["x"], st["u"], st["lam"], ck, mode, plan.new_workspace(),
                             status)
            aws = plan.new_adjoint_ckpt_workspace()
            aws.fill_(255)
            lq.lq_adjoint_ckpt(plan, prob, ck, mode, st["x"], st["u"], st["lam"], 2 * st["x"], 2 * st["u"], g, aws,
                               status)
        torch.cuda.synchronize()
        assert not status.cpu().numpy().any(), mode
        for f in names:
            for j, a in enumerate(split(g[f].cpu().numpy(), [gshape[f](i) for i in insts])):
                assert rel(a, refs[j][f]) < 1e-10, (mode, f, j)


@pytest.mark.parametrize("k", [0, 3, 4, 29, 39])
def test_small_path_nonfinite_stage(lq, k):
    """A NaN in A_k of a small instance inside a mixed batch: LQ_ERR_NONFINITE
    at stage k for it, the other instances unchanged and clean."""
    rng = np.random.default_rng(11)
    insts = [W.lq_instance(rng, 2, 1, 40), W.lq_instance(rng, 12, 4, 40), W.lq_instance(rng, 3, 1, 40)]
    clean, st0 = solve(lq, insts, seg_len=4)
    insts[0].A = insts[0].A.copy()
    insts[0].A[k, 1, 0] = np.nan
    bad, st = solve(lq, insts, seg_len=4)
    assert (int(st[0]) & 0xFF, int(st[0]) >> 8) == (4, k)
    assert st[1] == 0 and st[2] == 0 and not st0.any()
    for j in (1, 2):
        for key in KEYS:
            assert np.array_equal(bad[j][key], clean[j][key])


def test_small_path_not_pd_stage(lq):
    """R_k + B'S_{k+1}B indefinite at one stage of a small instance:
    LQ_ERR_NOT_PD at that stage."""
    inst = W.lq_instance(np.random.default_rng(12), 2, 1, 30)
    inst.R = inst.R.copy()
    inst.R[17] = -50.0
    _, st = solve(lq, [inst], seg_len=4)
    assert (int(st[0]) & 0xFF, int(st[0]) >> 8) == (2, 17)
