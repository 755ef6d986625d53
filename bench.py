"""Benchmark of the parallel-in-time LQ hot path on one MI355X.

Workload: one long-horizon time-varying LQ problem, n=12, m=4, T=16384, FP64,
drawn by paper_2409_20027_amd.workloads.cfg2_long (synthetic, seeded).
One step = the whole hot path over that input: value pass (fused element
build + segment fold, log-depth scan, Bellman steps with the control law),
rollout (segment maps, prefix scan, states/controls/co-states) and, when
available, the adjoint (backward linear-term scan, forward derivative scan,
per-stage gradients).  Inputs are resident in HBM before timing starts.

Prints one JSON line.  The metric is stage-steps per second (T stages per
step).  Also reported: the forward-solve latency at T = 16384 as the median of
graph replays, the plain sequential path on the same GPU, the error of a
sample against the FP64 oracle, the roofline of the dominant kernel and the
oracle timed on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def fold_flops_per_stage(n: int, m: int) -> float:
    """Useful flops of one segment-fold step (stage element built on the fly and
    left-folded into the segment element), in the homogeneous form n1 = n+1:
    J^G, A^G (2 n1^2 m each), J^Ab, A^Ab, Ab'J^Ab (2 n1^3 each), G'J^G (2 n1 m^2),
    G'J^Ab (2 m n1^2), W^{-1}P, W^{-1}H' (2 m^2 n1 each), three rank-m updates
    (2 n1^2 m each)."""
    n1 = n + 1
    return 6 * n1 ** 3 + 12 * n1 ** 2 * m + 6 * n1 * m ** 2


def fold_bytes_per_stage(n: int, m: int) -> float:
    """Algorithmic HBM bytes per stage of the fold: A, B, c, Q, R read once."""
    return 8.0 * (n * n + n * m + n + n * n + m * m)


def cpu_baseline(inst, budget_s: float = 10.0) -> dict:
    import oracle
    t0 = time.perf_counter()
    reps = 0
    while True:
        r = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": inst.T * reps / dt, "unit": "stage-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the same n=12 m=4 T={inst.T} instance, sequential Riccati + rollout + co-states "
                      f"(forward solve), repeated {reps} times in {dt:.1f} s on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--T", type=int, default=16384)
    ap.add_argument("--seg-len", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--replays", type=int, default=100)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver's multi-GPU sharding is a design, not a built path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_20027_amd import lqscan, workloads

    dev = torch.device("cuda:0")
    inst = workloads.cfg2_long(T=args.T)
    packed = workloads.pack([inst])
    prob = lqscan.to_device(packed, dev)
    n, m, T = inst.n, inst.m, inst.T

    plan = lqscan.Plan([n], [m], [T], seg_len=args.seg_len)
    ws = plan.new_workspace(dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    val = lqscan.value_buffers(plan, dev)
    st = lqscan.state_buffers(plan, dev)

    def step():
        lqscan.lq_scan_solve(plan, prob, None, val, ws, status)
        lqscan.lq_rollout(plan, prob, val, st["x"], st["u"], st["lam"], ws, status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    plan.set_timing(["value_fold"], capacity=args.steps + 8)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    phases = plan.phase_times()
    plan.set_timing([], 0)
    ms_per_step = total_ms / args.steps
    assert int(status.abs().sum()) == 0, "numerical failure reported"

    # error against the oracle on a sample of stages
    import oracle
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    x = st["x"].cpu().numpy().reshape(T + 1, n)
    u = st["u"].cpu().numpy().reshape(T, m)
    S = val["S"].cpu().numpy().reshape(T + 1, n, n)
    err = max(np.max(np.abs(x - ref["x"])) / np.max(np.abs(ref["x"])),
              np.max(np.abs(u - ref["u"])) / np.max(np.abs(ref["u"])),
              np.max(np.abs(S - ref["S"])) / np.max(np.abs(ref["S"])))

    # forward latency: median of graph replays (the whole forward solve captured once)
    lat_us = None
    try:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                step()
        torch.cuda.synchronize()
        times = []
        for i in range(10 + args.replays):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            g.replay()
            b.record()
            torch.cuda.synchronize()
            if i >= 10:
                times.append(a.elapsed_time(b) * 1e3)
        lat_us = float(np.median(times))
    except Exception as e:  # graph capture unavailable: report eager latency instead
        print(f"graph replay failed: {e!r}", file=sys.stderr)

    # the plain sequential path on the same GPU (forward solve)
    seq = {}
    splan = lqscan.Plan([n], [m], [T], mode="sequential")
    sws = splan.new_workspace(dev)

    def sstep():
        lqscan.lq_scan_solve(splan, prob, None, val, sws, status)
        lqscan.lq_rollout(splan, prob, val, st["x"], st["u"], st["lam"], sws, status)

    sstep()
    torch.cuda.synchronize()
    reps = 3
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        sstep()
    b.record()
    torch.cuda.synchronize()
    seq_ms = a.elapsed_time(b) / reps
    seq = {"ms_per_step": seq_ms, "value": T / (seq_ms * 1e-3), "unit": "stage-steps/s",
           "what": "forward solve, one segment (sequential Bellman recursion + sequential rollout)"}

    fold_ms, fold_launches = phases.get("value_fold", (float("nan"), 0))
    fold_avg_s = fold_ms / max(fold_launches, 1) * 1e-3
    flops = fold_flops_per_stage(n, m) * T
    achieved = flops / fold_avg_s / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_MFMA_PEAK_TFLOPS, "traffic": None,
            "kernel": "k_value_fold", "avg_launch_us": fold_avg_s * 1e6,
            "flops_per_launch": flops, "flops_per_stage": fold_flops_per_stage(n, m),
            "hbm_bytes_per_launch": fold_bytes_per_stage(n, m) * T}

    out = {"metric": "LQ stage-steps/sec (n=12, m=4, T=16384 solve, FP64)",
           "value": T * args.steps / (total_ms * 1e-3), "unit": "stage-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"time-varying LQ, n={n}, m={m}, T={T}, one instance, value scan + rollout",
                      "seg_len": plan.seg_len(), "step": "forward"},
           "latency_us_T16384_forward_graph": lat_us,
           "err_vs_oracle": err,
           "sequential_gpu": seq,
           "phase_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in phases.items()},
           "roofline": roof}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
