"""Ragged batch at full size: 4096 instances, T ~ U{32..2048}, n in {2, 4, 12},
m = max(1, n//3), solved together (one launch per phase for the whole batch),
every instance compared with the FP64 oracle; HIP-graph capture and replay;
autotuned per-class segment lengths."""
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


@pytest.fixture(scope="module")
def batch(lq):
    insts = W.cfg3_ragged()
    prob = lq.to_device(W.pack(insts))
    return insts, prob


def rel(a, b):
    den = np.max(np.abs(b))
    return np.max(np.abs(a - b)) / (den if den > 0 else 1.0)


def per_instance(flat, insts, shape):
    out, o = [], 0
    for i in insts:
        shp = shape(i)
        k = int(np.prod(shp))
        out.append(flat[o:o + k].reshape(shp))
        o += k
    return out


def check_all(insts, out, sample=None, tol=TOL):
    xs = per_instance(out["x"].cpu().numpy(), insts, lambda i: (i.T + 1, i.n))
    us = per_instance(out["u"].cpu().numpy(), insts, lambda i: (i.T, i.m))
    Ss = per_instance(out["S"].cpu().numpy(), insts, lambda i: (i.T + 1, i.n, i.n))
    idx = range(len(insts)) if sample is None else sample
    worst = 0.0
    for j in idx:
        i = insts[j]
        ref = oracle.lq_solve(i.A, i.B, i.c, i.Q, i.R, i.QT, i.x0)
        e = max(rel(xs[j], ref["x"]), rel(us[j], ref["u"]), rel(Ss[j], ref["S"]))
        worst = max(worst, e)
        assert e <= tol, (j, i.n, i.T, e)
    return worst


def test_ragged_batch_every_instance(lq, batch):
    insts, prob = batch
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts])
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    worst = check_all(insts, out)
    print(f"ragged batch: {len(insts)} instances, {plan.total_stages()} stages, worst rel err {worst:.2e}")


def test_ragged_batch_mixed_every_instance(lq, batch):
    """The ragged batch at its stated precision (FP32 products, FP64 inverses,
    Cholesky factors and symmetrisation): every instance against the FP64
    oracle at the mixed bound x, u, S <= 1e-4 (normwise relative per instance)."""
    insts, prob = batch
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], precision="mixed")
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    worst = check_all(insts, out, tol=1e-4)
    print(f"ragged batch, mixed precision: worst rel err {worst:.2e}")


def test_ragged_batch_graph_replay(lq, batch):
    """The forward solve captured once in a HIP graph; every replay (with eager
    work between replays) reproduces the eager result bit for bit."""
    insts, prob = batch
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts])
    ws = plan.new_workspace()
    status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    val = lq.value_buffers(plan)
    st = lq.state_buffers(plan)

    def fwd():
        lq.lq_scan_solve(plan, prob, None, val, ws, status)
        lq.lq_rollout(plan, prob, val, st["x"], st["u"], st["lam"], ws, status)

    fwd()
    torch.cuda.synchronize()
    ref_x, ref_S = st["x"].clone(), val["S"].clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fwd()
    torch.cuda.synchronize()
    for r in range(3):
        st["x"].zero_()
        val["S"].fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(st["x"], ref_x), r
        assert torch.equal(val["S"], ref_S), r
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        del junk
    assert int(status.abs().sum()) == 0


def test_full_step_graph_replay(lq):
    """The whole benchmark step -- lq_solve, lq_adjoint -- and the
    conditional-value rollout captured once in a HIP graph; every replay (with
    eager work between replays) reproduces the eager results bit for bit."""
    inst = W.lq_instance_general(np.random.default_rng(77), 12, 4, 1500)
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([12], [4], [1500], seg_len=16)
    ws, ws2 = plan.new_workspace(), plan.new_workspace()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    val = lq.value_buffers(plan)
    st = lq.state_buffers(plan)
    cv = lq.state_buffers(plan)
    names = ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")
    grads = lq.grad_buffers(plan, names)
    gx = torch.randn_like(st["x"])
    gu = torch.randn_like(st["u"])

    def step():
        lq.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
        lq.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, grads, ws, status)
        lq.lq_rollout_cv(plan, prob, val, cv["x"], cv["u"], cv["lam"], ws2, status)

    step()
    torch.cuda.synchronize()
    outs = {"x": st["x"], "S": val["S"], "cv_x": cv["x"], **{"g" + k: v for k, v in grads.items()}}
    ref = {k: v.clone() for k, v in outs.items()}
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            step()
    torch.cuda.synchronize()
    for r in range(3):
        for v in outs.values():
            v.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert torch.equal(v, ref[k]), (r, k)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        del junk
    assert int(status.abs().sum()) == 0


def test_ragged_batch_autotuned(lq, batch, tmp_path):
    from paper_2409_20027_amd import autotune
    insts, prob = batch
    cache = str(tmp_path / "tune.json")
    seg, report = autotune.tune(insts, cache_path=cache, sample_per_class=48, reps=2)
    print("autotuned:", autotune.seg_lens_summary(insts, seg))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], seg_lens=seg)
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    rng = np.random.default_rng(0)
    check_all(insts, out, sample=sorted(rng.choice(len(insts), 256, replace=False)))
    # a second call hits the cache and returns the same choice
    seg2, report2 = autotune.tune(insts, cache_path=cache, sample_per_class=48, reps=2)
    assert seg2 == seg and report2 == {}
    # the library reads the same cache (lq_plan_create_tuned): the same segments, so the same bits
    plan_c = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], autotune_cache=cache)
    assert plan_c.seg_len() == plan.seg_len()
    out_c = lq.solve(plan_c, prob)
    torch.cuda.synchronize()
    for k in ("x", "u", "S", "Gamma"):
        assert torch.equal(out_c[k], out[k]), k
