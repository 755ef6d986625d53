"""GPU parity of the adjoint (lq_adjoint and the autograd wrapper) against the
oracle's KKT adjoint and against central finite differences.

Loss: L = sum_k ||x_k||^2 + sum_k ||u_k||^2 (gx = 2x, gu = 2u).
Tolerance: 1e-10 normwise relative per gradient array (FP64).
"""
import numpy as np
import pytest

import oracle
from paper_2409_20027_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")
SHAPES = {"A": lambda i: (i.T, i.n, i.n), "B": lambda i: (i.T, i.n, i.m), "c": lambda i: (i.T, i.n),
          "Q": lambda i: (i.T, i.n, i.n), "R": lambda i: (i.T, i.m, i.m), "M": lambda i: (i.T, i.n, i.m),
          "q": lambda i: (i.T, i.n), "r": lambda i: (i.T, i.m), "QT": lambda i: (i.n, i.n),
          "qT": lambda i: (i.n,), "x0": lambda i: (i.n,)}


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


def gpu_grads(lq, insts, **plan_kw):
    packed = W.pack(insts)
    prob = lq.to_device(packed)
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], **plan_kw)
    out = lq.solve(plan, prob)
    gx, gu = 2 * out["x"], 2 * out["u"]
    want = [f for f in FIELDS if prob.get(f) is not None or f in ("M", "q", "r", "qT", "c")]
    g = lq.grad_buffers(plan, want)
    ws = plan.new_workspace()
    lq.lq_adjoint(plan, prob, {k: out[k] for k in ("S", "s", "Gamma", "gamma")}, out["x"], out["u"], out["lam"],
                  gx, gu, g, ws, out["status"])
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    per = [dict() for _ in insts]
    for f, t in g.items():
        for j, a in enumerate(split(t.cpu().numpy(), [SHAPES[f](i) for i in insts])):
            per[j][f] = a
    return per


def oracle_grads(inst):
    o = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0,
                        M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
    return oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * o["x"], 2 * o["u"],
                             M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)


def check(per, insts, tol=1e-10):
    worst = 0.0
    for got, inst in zip(per, insts):
        ref = oracle_grads(inst)
        for f, a in got.items():
            e = rel(a, ref[f])
            worst = max(worst, e)
            assert e <= tol, f"grad {f}: rel err {e:.3e} (n={inst.n}, m={inst.m}, T={inst.T})"
    return worst


@pytest.mark.parametrize("seg_len", [0, 1, 4, 7])
def test_adjoint_general_lq(lq, seg_len):
    inst = W.lq_instance_general(np.random.default_rng(31), 3, 2, 29)
    check(gpu_grads(lq, [inst], seg_len=seg_len), [inst])


def test_adjoint_sequential_mode(lq):
    inst = W.lq_instance_general(np.random.default_rng(32), 4, 1, 40)
    check(gpu_grads(lq, [inst], mode="sequential"), [inst])


def test_adjoint_ragged_batch(lq):
    rng = np.random.default_rng(33)
    insts = [W.lq_instance(rng, n, m, T) for n, m, T in [(2, 1, 5), (12, 4, 70), (4, 1, 1), (7, 3, 33)]]
    insts.append(W.lq_instance_general(rng, 5, 2, 21))
    check(gpu_grads(lq, insts), insts)


def test_adjoint_long_horizon_batch_sample(lq):
    """Sample of the differentiated-solve workload: n=12, m=4, T=4096, a few instances."""
    insts = W.cfg4_batch(batch=3, T=4096)
    check(gpu_grads(lq, insts), insts)


@pytest.mark.parametrize("radix", [2, 4, 8, 16, 32])
def test_adjoint_affine_scan_radix(lq, radix, monkeypatch):
    """Both reversed affine scans through every radix (one stage per segment, up to 301 entries)."""
    monkeypatch.setenv("LQSCAN_AFFINE_RADIX", str(radix))
    rng = np.random.default_rng(50 + radix)
    insts = [W.lq_instance_general(rng, 3, 2, 300), W.lq_instance(rng, 5, 2, 45), W.lq_instance(rng, 2, 1, 1)]
    check(gpu_grads(lq, insts, seg_len=1), insts)


def test_autograd_function_matches_oracle_and_fd(lq):
    inst = W.lq_instance_general(np.random.default_rng(34), 3, 2, 17)
    packed = W.pack([inst])
    prob = lq.to_device(packed)
    plan = lq.Plan([inst.n], [inst.m], [inst.T], seg_len=4)
    names = ("A", "B", "c", "Q", "R", "QT", "x0", "M", "q", "r", "qT")
    leaves = {f: prob[f].clone().requires_grad_(True) for f in names}

    def loss_of(t):
        x, u, _ = lq.solve_diff(plan, *[t[f] for f in names])
        return (x * x).sum() + (u * u).sum()

    L = loss_of(leaves)
    grads = torch.autograd.grad(L, [leaves[f] for f in names])
    ref = oracle_grads(inst)
    for f, g in zip(names, grads):
        assert rel(g.detach().cpu().numpy().reshape(ref[f].shape), ref[f]) < 1e-10, f
    # central finite differences of the GPU forward along random directions
    rng = np.random.default_rng(35)
    with torch.no_grad():
        for _ in range(16):
            d = {f: torch.tensor(rng.standard_normal(prob[f].shape), dtype=torch.float64, device="cuda")
                 for f in names}
            for f in ("Q", "R", "QT"):   # symmetric perturbations of symmetric inputs
                shp = SHAPES[f](inst)
                v = d[f].reshape(shp)
                d[f] = (0.5 * (v + v.transpose(-1, -2))).reshape(-1).contiguous()
            nrm = torch.sqrt(sum((v * v).sum() for v in d.values()))
            h = 1e-6
            plus = loss_of({f: prob[f] + h * d[f] / nrm for f in names})
            minus = loss_of({f: prob[f] - h * d[f] / nrm for f in names})
            fd = float((plus - minus) / (2 * h))
            an = float(sum((g * d[f] / nrm).sum() for f, g in zip(names, grads)))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


@pytest.mark.parametrize("seed", range(8))
def test_random_adjoint_configurations(lq, seed):
    """Seeded random sizes (n to 15, m to 4), horizons, segment lengths,
    dynamics between mildly and clearly unstable, optional terms present or
    absent and random loss gradients: every gradient against the oracle to
    1e-12 (a sweep of 80 such configurations peaks at 1e-14)."""
    names = ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")
    rng = np.random.default_rng(80000 + seed)
    n, m = int(rng.integers(1, 16)), int(rng.integers(1, 5))
    T = int(rng.choice([1, 2, int(rng.integers(3, 60)), int(rng.integers(60, 1200))]))
    inst = W.lq_instance_general(rng, n, m, T, a_scale=float(rng.uniform(0.05, 0.25)))
    for f in ("c", "M", "q", "r", "qT"):
        if rng.random() < 0.4:
            setattr(inst, f, None)
    L = int(rng.choice([0, 1, int(rng.integers(1, T + 3))]))
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([n], [m], [T], seg_lens=[L])
    out = lq.solve(plan, prob)
    gx = torch.tensor(rng.standard_normal((T + 1) * n), device="cuda")
    gu = torch.tensor(rng.standard_normal(T * m), device="cuda")
    have = [k for k in names if k in ("A", "B", "Q", "R", "QT", "x0") or getattr(inst, k) is not None]
    grads = lq.grad_buffers(plan, have)
    val = {k: out[k] for k in ("S", "s", "Gamma", "gamma")}
    lq.lq_adjoint(plan, prob, val, out["x"], out["u"], out["lam"], gx, gu, grads, plan.new_workspace(), out["status"])
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    g = oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0,
                          gx.cpu().numpy().reshape(T + 1, n), gu.cpu().numpy().reshape(T, m),
                          M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
    for k in have:
        a = grads[k].cpu().numpy().reshape(g[k].shape)
        assert rel(a, g[k]) < 1e-12, (k, n, m, T, L)


def test_maximum_sizes_full_horizon(lq):
    """The largest supported sizes (n = 15, m = 4) with every LQ term at
    T = 16384 and the default segment length: solution and gradients against
    the oracle at every stage, to 1e-10."""
    inst = W.lq_instance_general(np.random.default_rng(15004), 15, 4, 16384)
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([15], [4], [16384])
    out = lq.solve(plan, prob)
    torch.cuda.synchronize()
    assert int(out["status"].abs().sum()) == 0
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0,
                          M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
    T, n, m = 16384, 15, 4
    assert rel(out["x"].cpu().numpy().reshape(T + 1, n), ref["x"]) < 1e-10
    assert rel(out["u"].cpu().numpy().reshape(T, m), ref["u"]) < 1e-10
    assert rel(out["S"].cpu().numpy().reshape(T + 1, n, n), ref["S"]) < 1e-10
    check(gpu_grads(lq, [inst]), [inst])


def test_adjoint_mixed_batch_sample(lq):
    """Sample of the differentiated-solve workload in mixed precision (FP32
    products; FP64 inverses, Cholesky factors and symmetrisation): 3 instances
    of n=12, m=4, T=4096, every gradient against the FP64 oracle at the mixed
    bound 1e-3 (normwise relative)."""
    insts = W.cfg4_batch(batch=3, T=4096)
    worst = check(gpu_grads(lq, insts, precision="mixed"), insts, tol=1e-3)
    print(f"mixed adjoint, 3 x T=4096: worst rel err {worst:.2e}")


def test_finite_differences_long_horizon(lq):
    """Central finite differences (h = 1e-6) of L = sum ||x||^2 + ||u||^2 along
    16 random unit directions over (A, B, c, Q, R, Q_T, x0) -- N(0,1) entries,
    symmetrised for Q, R, Q_T, normalised to unit norm -- on one instance of
    the differentiated workload (n=12, m=4, T=4096, FP64): the GPU forward's
    difference quotient against the GPU adjoint's directional derivative, to
    1e-6 relative (the oracle's own quotient at this size is within 3e-8)."""
    inst = W.cfg4_batch(batch=1, T=4096)[0]
    names = ("A", "B", "c", "Q", "R", "QT", "x0")
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([12], [4], [4096])
    ws = plan.new_workspace()

    def loss(p):
        out = lq.solve(plan, p, workspace=ws)
        torch.cuda.synchronize()
        assert int(out["status"].abs().sum()) == 0
        return float((out["x"] * out["x"]).sum() + (out["u"] * out["u"]).sum()), out

    _, out = loss(prob)
    g = lq.grad_buffers(plan, names)
    lq.lq_adjoint(plan, prob, {k: out[k] for k in ("S", "s", "Gamma", "gamma")}, out["x"], out["u"], out["lam"],
                  2 * out["x"], 2 * out["u"], g, ws, out["status"])
    torch.cuda.synchronize()
    check([{f: g[f].cpu().numpy().reshape(SHAPES[f](inst)) for f in names}], [inst])   # oracle, 1e-10
    rng = np.random.default_rng(36)
    h = 1e-6
    worst = 0.0
    for _ in range(16):
        d = {f: rng.standard_normal(SHAPES[f](inst)) for f in names}
        for f in ("Q", "R", "QT"):
            d[f] = 0.5 * (d[f] + np.swapaxes(d[f], -1, -2))
        nrm = np.sqrt(sum(float((v * v).sum()) for v in d.values()))
        dd = {f: torch.tensor((v / nrm).reshape(-1), device="cuda") for f, v in d.items()}
        plus, _ = loss({**prob, **{f: prob[f] + h * dd[f] for f in names}})
        minus, _ = loss({**prob, **{f: prob[f] - h * dd[f] for f in names}})
        fd = (plus - minus) / (2 * h)
        an = float(sum((g[f] * dd[f]).sum() for f in names))
        e = abs(fd - an) / max(1.0, abs(an))
        worst = max(worst, e)
        assert e <= 1e-6, (fd, an)
    print(f"finite differences, n=12 T=4096: worst rel err {worst:.2e}")


def test_autograd_saved_tensors(lq):
    """The wrapper saves its inputs and outputs with save_for_backward: an
    in-place change of an input between forward and backward is refused, and
    with the cyclic garbage collector off, device memory returns to its level
    before the solve once the outputs are dropped (no output is held by its
    own grad_fn)."""
    import gc
    inst = W.lq_instance_general(np.random.default_rng(37), 4, 2, 200)
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([4], [2], [200], seg_len=8)
    names = lq.LQSolveFunction.NAMES
    leaves = {f: prob[f].clone().requires_grad_(True) for f in names}
    A = leaves["A"] * 1.0
    x, u, _ = lq.solve_diff(plan, A, *[leaves[f] for f in names[1:]])
    L = (x * x).sum() + (u * u).sum()
    with torch.no_grad():
        A.add_(1e-3)
    with pytest.raises(RuntimeError, match="modified by an inplace operation"):
        L.backward()
    del x, u, L, A
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        base = torch.cuda.memory_allocated()
        for _ in range(3):
            x, u, _ = lq.solve_diff(plan, *[leaves[f] for f in names])
            L = (x * x).sum() + (u * u).sum()
            grads = torch.autograd.grad(L, [leaves[f] for f in names])
            del x, u, L, grads
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
    finally:
        gc.enable()


# ---------------------------------------------------------------------------
# Level checkpointing: lq_solve_ckpt keeps one value-function carry per
# `stride` segments, lq_adjoint_ckpt recomputes S, s, Gamma, gamma from it
# (or, with no checkpoint, reruns the whole value pass).
# ---------------------------------------------------------------------------

def gpu_grads_ckpt(lq, insts, stride, **plan_kw):
    """Gradients through lq_solve_ckpt + lq_adjoint_ckpt (stride "recompute":
    lq_solve, then lq_adjoint_ckpt without a checkpoint).  The backward
    workspace is filled with NaN bytes first, so a value array the recompute
    failed to write shows in the gradients."""
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], **plan_kw)
    status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    val = lq.value_buffers(plan)
    st = lq.state_buffers(plan)
    ws = plan.new_workspace()
    if stride == "recompute":
        ckpt, s = None, 1
        lq.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
    else:
        ckpt, s = plan.new_checkpoint(stride), stride
        lq.lq_solve_ckpt(plan, prob, None, val, st["x"], st["u"], st["lam"], ckpt, s, ws, status)
    torch.cuda.synchronize()
    del val
    want = [f for f in FIELDS if prob.get(f) is not None or f in ("M", "q", "r", "qT", "c")]
    g = lq.grad_buffers(plan, want)
    aws = plan.new_adjoint_ckpt_workspace()
    aws.fill_(255)
    lq.lq_adjoint_ckpt(plan, prob, ckpt, s, st["x"], st["u"], st["lam"], 2 * st["x"], 2 * st["u"], g, aws, status)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    per = [dict() for _ in insts]
    for f, t in g.items():
        for j, a in enumerate(split(t.cpu().numpy(), [SHAPES[f](i) for i in insts])):
            per[j][f] = a
    return per


@pytest.mark.parametrize("stride", [1, 2, 3, 16, "recompute"])
def test_checkpointed_adjoint_ragged_batch(lq, stride):
    """Ragged batch with every optional term in some instances, segment
    lengths that leave ragged last segments and groups, T = 1 and a single
    segment: every gradient against the oracle to 1e-10."""
    rng = np.random.default_rng(90)
    insts = [W.lq_instance(rng, n, m, T) for n, m, T in [(2, 1, 5), (12, 4, 70), (4, 1, 1), (7, 3, 33)]]
    insts += [W.lq_instance_general(rng, 5, 2, 21), W.lq_instance_general(rng, 15, 4, 131)]
    print(f"checkpoint stride {stride}", flush=True)
    check(gpu_grads_ckpt(lq, insts, stride, seg_len=4), insts)


@pytest.mark.parametrize("stride", [1, 4, "recompute"])
def test_checkpointed_adjoint_long_horizon_sample(lq, stride):
    """Sample of the differentiated-solve workload (3 x n=12, m=4, T=4096,
    default segments) through the checkpointed adjoint: 1e-10 to the oracle."""
    insts = W.cfg4_batch(batch=3, T=4096)
    print(f"checkpoint stride {stride}, 3 x T=4096", flush=True)
    check(gpu_grads_ckpt(lq, insts, stride), insts)


def test_checkpoint_stride_one_equals_stored_path(lq):
    """With stride 1 the recompute reruns the forward's own Bellman sweeps from
    the same carries, so the gradients equal the stored-value path bit for
    bit."""
    rng = np.random.default_rng(91)
    insts = [W.lq_instance_general(rng, 6, 2, 300), W.lq_instance(rng, 12, 4, 1000)]
    a = gpu_grads(lq, insts)
    b = gpu_grads_ckpt(lq, insts, 1)
    for ga, gb in zip(a, b):
        for f in ga:
            assert np.array_equal(ga[f], gb[f]), f


def test_adjoint_without_value_functions(lq):
    """lq_adjoint with val = NULL reruns the value pass from the problem data
    (the recompute of lq_adjoint_ckpt without a checkpoint): on a batch mixing
    per-lane and tile classes the gradients equal those of the stored-value
    path bit for bit, since the rerun repeats the forward's own arithmetic."""
    rng = np.random.default_rng(93)
    insts = [W.lq_instance_general(rng, 3, 1, 77), W.lq_instance(rng, 12, 4, 500), W.lq_instance_general(rng, 6, 2, 41)]
    prob = lq.to_device(W.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], seg_len=8)
    status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    val, st = lq.value_buffers(plan), lq.state_buffers(plan)
    ws = plan.new_workspace()
    lq.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
    gx, gu = 2 * st["x"], 2 * st["u"]
    g_stored = lq.grad_buffers(plan, FIELDS)
    lq.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, g_stored, ws, status)
    g_none = lq.grad_buffers(plan, FIELDS)
    aws = plan.new_adjoint_ckpt_workspace()
    aws.fill_(255)
    lq.lq_adjoint(plan, prob, None, st["x"], st["u"], st["lam"], gx, gu, g_none, aws, status)
    torch.cuda.synchronize()
    assert int(status.abs().sum()) == 0
    for f in FIELDS:
        assert torch.equal(g_stored[f], g_none[f]), f


@pytest.mark.parametrize("checkpoint", [0, 1, 5, "recompute"])
def test_autograd_checkpoint_modes(lq, checkpoint):
    """The autograd wrapper in each mode (0: keep S and Gamma; k: stride-k
    checkpoint; "recompute": keep nothing) gives the oracle's gradients, and
    what it keeps between forward and backward shrinks accordingly."""
    inst = W.lq_instance_general(np.random.default_rng(92), 12, 4, 2000)
    prob = lq.to_device(W.pack([inst]))
    plan = lq.Plan([12], [4], [2000], seg_len=8)
    names = lq.LQSolveFunction.NAMES
    leaves = {f: prob[f].clone().requires_grad_(True) for f in names}
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    x, u, _ = lq.solve_diff(plan, *[leaves[f] for f in names], checkpoint=checkpoint)
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - base
    L = (x * x).sum() + (u * u).sum()
    grads = torch.autograd.grad(L, [leaves[f] for f in names])
    ref = oracle_grads(inst)
    for f, g in zip(names, grads):
        assert rel(g.detach().cpu().numpy().reshape(ref[f].shape), ref[f]) < 1e-10, f
    T, n, m = 2000, 12, 4
    value_bytes = 8 * ((T + 1) * n * n + (T + 1) * n + T * m * n + T * m)
    if checkpoint == 0:
        assert held >= value_bytes
    else:
        assert held < value_bytes / 2, (held, value_bytes)
    print(f"checkpoint={checkpoint}: {held / 2**20:.2f} MiB held after forward "
          f"(value arrays {value_bytes / 2**20:.2f} MiB)")


def test_tensor_form_solve_and_batch(lq):
    """lqscan.solve on stage-major tensors and lqscan.solve_batch on a list of
    problems of different sizes: x, u against the oracle (1e-10), gradients
    through autograd against the oracle's adjoint (1e-9), and a numerical
    failure raised as LQError with its stage."""
    rng = np.random.default_rng(94)
    insts = [W.lq_instance_general(rng, 5, 2, 40), W.lq_instance(rng, 2, 1, 17), W.lq_instance(rng, 12, 4, 64)]

    def tensors(inst, grad=False):
        d = {}
        for f, shp in (("A", (inst.T, inst.n, inst.n)), ("B", (inst.T, inst.n, inst.m)), ("c", (inst.T, inst.n)),
                       ("Q", (inst.T, inst.n, inst.n)), ("R", (inst.T, inst.m, inst.m)), ("QT", (inst.n, inst.n)),
                       ("x0", (inst.n,)), ("M", (inst.T, inst.n, inst.m)), ("q", (inst.T, inst.n)),
                       ("r", (inst.T, inst.m)), ("qT", (inst.n,))):
            v = getattr(inst, f)
            if v is None:
                continue
            d[f] = torch.tensor(np.asarray(v).reshape(shp), dtype=torch.float64, device="cuda", requires_grad=grad)
        return d

    def ref(inst):
        o = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, M=inst.M, q=inst.q, r=inst.r,
                            qT=inst.qT)
        g = oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * o["x"], 2 * o["u"],
                              M=inst.M, q=inst.q, r=inst.r, qT=inst.qT)
        return o, g

    # one problem, tensor form
    inst = insts[0]
    d = tensors(inst, grad=True)
    x, u = lq.solve(d["A"], d["B"], d.get("c"), d["Q"], d["R"], d["QT"], d["x0"], M=d.get("M"), q=d.get("q"),
                    r=d.get("r"), qT=d.get("qT"))
    o, g = ref(inst)
    assert rel(x.detach().cpu().numpy(), o["x"]) < 1e-10 and rel(u.detach().cpu().numpy(), o["u"]) < 1e-10
    ((x * x).sum() + (u * u).sum()).backward()
    for f, t in d.items():
        assert rel(t.grad.cpu().numpy().reshape(np.shape(g[f])), g[f]) < 1e-9, f
    # the batch
    ds = [tensors(i, grad=True) for i in insts]
    outs = lq.solve_batch(ds)
    loss = sum((x * x).sum() + (u * u).sum() for x, u in outs)
    loss.backward()
    for inst, dd, (x, u) in zip(insts, ds, outs):
        o, g = ref(inst)
        assert rel(x.detach().cpu().numpy(), o["x"]) < 1e-10 and rel(u.detach().cpu().numpy(), o["u"]) < 1e-10
        for f, t in dd.items():
            assert rel(t.grad.cpu().numpy().reshape(np.shape(g[f])), g[f]) < 1e-9, (inst.n, f)
    # R indefinite at stage 9: LQError naming the stage
    bad = tensors(insts[1])
    bad["R"][9] = -50.0
    with pytest.raises(lq.LQError, match="stage 9"):
        lq.solve(bad["A"], bad["B"], bad.get("c"), bad["Q"], bad["R"], bad["QT"], bad["x0"])


@pytest.mark.parametrize("seg_len", [1, 2, 3, 4, 5])
def test_tile_sweeps_short_and_odd_segments(lq, seg_len):
    """The tile-path sweeps stage their data two stages ahead in an unrolled
    pair of stages with an odd last stage after the loop: segments of one to
    five stages (T = 23, so the last segment is shorter except at L = 1) through
    the value pass, the rollout and both adjoint sweeps, against the oracle."""
    inst = W.lq_instance_general(np.random.default_rng(900 + seg_len), 6, 2, 23)
    check(gpu_grads(lq, [inst], seg_len=seg_len), [inst])
