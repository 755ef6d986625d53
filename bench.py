"""Benchmark of the parallel-in-time LQ hot path on one MI355X.

Workload: one long-horizon time-varying LQ problem, n=12, m=4, T=16384, FP64,
drawn by paper_2409_20027_amd.workloads.cfg2_long (synthetic, seeded).
One step = the whole hot path over that input, forward and adjoint:
  value pass   (fused element build + segment fold, log-depth scan of the
                segment elements, Bellman steps with the control law and the
                rollout's segment maps),
  rollout      (prefix scan of the segment maps, states / controls / co-states),
  adjoint      (backward linear-term scan, forward derivative scan, per-stage
                gradients of L = sum ||x||^2 + ||u||^2 w.r.t. A, B, c, Q, R,
                Q_T, x0).
Inputs (and the loss gradients 2x, 2u) are resident in HBM before timing.

Prints one JSON line.  The metric is stage-steps per second (T stages per
step).  Also reported: the forward-solve latency at T = 16384 (median of graph
replays), the plain sequential path on the same GPU, the error of the result
against the FP64 oracle, a per-kernel breakdown, the roofline of the dominant
kernel and the oracle timed on the host.
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
FP64_PEAK_TFLOPS = 78.6   # FP64 matrix cores (dense) = FP64 vector
CSRC = os.path.join(ROOT, "paper_2409_20027_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
CALIB_BYTES = 256 << 20   # the plain copy launched by --calib (read and written once)


PHASE_SOURCE = {"value": "lq_value.hip", "roll": "lq_rollout.hip", "adj": "lq_adjoint.hip"}


def source_hash(phase: str | None = None) -> str:
    """SHA-256 over the HIP sources a phase's kernel is built from (its .hip
    file and the tile and descriptor headers; all sources when phase is None),
    so that a stored counter reading is only used while that kernel's code is
    unchanged."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    if phase is not None:
        src = PHASE_SOURCE[phase.split("_")[0]]
        files = [f for f in files if f in (src, "lq_tile.hpp", "lq_desc.hpp")]
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from profiles/traffic_<kernel>.md (two
    rocprofv3 --pmc passes, FETCH_SIZE and WRITE_SIZE, scaled by the readings of
    a plain copy of known size), or None if absent or taken from other sources."""
    path = os.path.join(PROFILES, f"traffic_{kernel}.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith(("|", "#")):
                k, v = line.split(":", 1)
                rec[k.strip().strip("`*")] = v.strip().strip("`")
    if rec.get("source_sha256") != source_hash(kernel):
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None

# ---------------------------------------------------------------------------
# Per-stage algorithmic cost models of the kernels (n1 = n + 1, homogeneous
# form).  Flops count only the products the method needs (no tile padding);
# bytes count the HBM traffic a perfect kernel would do (read each input once,
# write each output once).
# ---------------------------------------------------------------------------


def kernel_models(n, m, T=16384, L=16):
    """Per-step algorithmic cost of each timed phase: flops, bytes and the
    number of kernel launches it takes (scans: one launch per level)."""
    n1 = n + 1
    d = 8.0
    per_stage = {
        # element build + rank-m left fold: J^B, J^A, B'J^B, B'J^A, A'J^A, B'A^', A'A^', the m x m
        # inverse and four rank-m products
        "value_fold": {"flops": 6 * n1 ** 3 + 12 * n1 ** 2 * m + 6 * n1 * m ** 2,
                       "bytes": d * (2 * n * n + n * m + n + m * m)},
        # Bellman step: S'B, S'A, B'S'B, B'S'A, A'S'A, Q_uu^{-1} Q_ux, Q_ux' Gamma, plus the
        # rollout's segment map (F = A + B Gamma, Phi F)
        "value_bellman": {"flops": 4 * n1 ** 3 + 6 * n1 ** 2 * m + 4 * n1 * m ** 2 + 2 * n1 ** 3 + 2 * n1 ** 2 * m,
                          "bytes": d * (2 * n * n + n * m + n + m * m + n * n + n + m * n + m)},
        "roll_apply": {"flops": 4 * n1 ** 2 + 4 * m * n1,
                       "bytes": d * (2 * n * n + 2 * m * n + 4 * n + 2 * m)},
        "adj_back_fold": {"flops": 2 * n1 ** 3 + 2 * n1 ** 2 * m + 2 * n1 * m,
                          "bytes": d * (n * n + 2 * n * m + 2 * m + n)},
        "adj_back_apply": {"flops": 4 * n1 ** 3 + 8 * n1 ** 2 * m + 4 * n1 * m ** 2 + 2 * n1 ** 2,
                           "bytes": d * (2 * n * n + 2 * n * m + m * m + 3 * n + 3 * m)},
        "adj_fwd_apply": {"flops": 6 * n1 ** 2 + 4 * m * n1 + 8 * n * n + 8 * n * m + 2 * m * m,
                          "bytes": d * (3 * n * n + 2 * n * m + 4 * n + 2 * m
                                        + 2 * n * n + 2 * n * m + 2 * n + m * m + m)},
    }
    out = {k: {"flops": v["flops"] * T, "bytes": v["bytes"] * T, "launches": 1, "units": T,
               "unit_name": "stages"} for k, v in per_stage.items()}
    # value scan: radix-2 Kogge-Stone over the segment elements 1 .. nseg-1
    # (the last one folded onto the terminal element); per level each entry
    # either combines with s + dd (a full combine, or a J-only one when the
    # right operand already covers the terminal) or carries its J over.  A combine reads 6 (n1 x n1) matrices
    # and writes 3; its flops: X' (2 n1^2 n), the n x n Gauss-Jordan inverse
    # (2 n^3), Z, J2 A1, the J rule (3 x 2 n1^3), A2 Z, X^{-1} C1, two C
    # products (2 n1^3 + 2 n1^2 n + 2 x 2 n1^3).
    nseg = -(-T // L)
    full_f = 2 * n1 * n1 * n + 2 * n ** 3 + 6 * n1 ** 3 + 2 * n1 ** 3 + 2 * n1 * n1 * n + 4 * n1 ** 3
    jonly_f = 2 * n1 * n1 * n + 2 * n ** 3 + 6 * n1 ** 3
    mat = d * n1 * n1
    fl = by = 0.0
    lev = combines = 0
    dd = 1
    last = nseg - 1
    while dd < last:
        lev += 1
        for s_ in range(1, last + 1):
            if s_ + dd > last:
                by += 2 * mat
            elif s_ + 2 * dd - 1 >= last:
                fl += jonly_f
                by += 5 * mat
                combines += 1
            else:
                fl += full_f
                by += 9 * mat
                combines += 1
        dd *= 2
    out["value_scan"] = {"flops": fl, "bytes": by, "launches": max(lev, 1), "units": combines,
                         "unit_name": "element combines"}
    return out


def cpu_baseline(inst, budget_s: float = 10.0) -> dict:
    import oracle
    o = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    gx, gu = 2 * o["x"], 2 * o["u"]
    t0 = time.perf_counter()
    reps = 0
    while True:
        r = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
        oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, gx, gu)
        reps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": inst.T * reps / dt, "unit": "stage-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the same n=12 m=4 T={inst.T} instance: sequential Riccati + rollout + co-states, "
                      f"then the KKT adjoint (forward + adjoint, as one GPU step), repeated {reps} times "
                      f"in {dt:.1f} s on one host core"}


# ---------------------------------------------------------------------------
# Whole-solve cost per stage (the scan method's product count of section 8(d)
# of the design and the bytes a perfect kernel would move), for the batched
# and small-case lines.  Forward: read A, B, c, Q, R, write x, u.  Forward +
# adjoint adds re-reading A, B, Q, R, x, u and the loss gradients, and writing
# the gradients of A, B, c, Q, R.
# ---------------------------------------------------------------------------


def stage_model(n: int, m: int, adjoint: bool = False) -> dict:
    words = 2 * n * n + n * m + 2 * n + m * m + m
    flops = 24.7 * n ** 3 + 8 * n * n * m
    if adjoint:
        words += 4 * n * n + 2 * n * m + 2 * m * m + 3 * n + 2 * m
        flops += 4 * n ** 3 + 8 * n * n * m
    return {"bytes": 8.0 * words, "flops": flops}


def fractions(sizes, ms: float, adjoint: bool = False) -> dict:
    """Achieved HBM and FP64 rates of a batch of (n, m, T) solved in ms, and
    their fractions of the MI355X peaks."""
    by = sum(T * stage_model(n, m, adjoint)["bytes"] for n, m, T in sizes)
    fl = sum(T * stage_model(n, m, adjoint)["flops"] for n, m, T in sizes)
    s = ms * 1e-3
    return {"GB/s": by / s / 1e9, "hbm_frac": by / s / 1e9 / HBM_PEAK_GBS, "TFLOP/s": fl / s / 1e12,
            "fp64_frac": fl / s / 1e12 / FP64_PEAK_TFLOPS}


def time_graph(fn, reps: int, warm: int = 3) -> float:
    """ms per call of fn captured once in a HIP graph: the median over `reps`
    replays, each bracketed by its own events (one eager call first)."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for _ in range(warm):
        g.replay()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def time_eager(fn, reps: int, warm: int = 1) -> float:
    """ms per call of fn launched eagerly (events around `reps` calls)."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def host_info() -> dict:
    threads = min(16, len(os.sched_getaffinity(0)))
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"threads": threads, "nproc": os.cpu_count(), "cpu_model": model}


def oracle_batch(insts, adjoint: bool) -> dict:
    """The oracle over a sample of a batch on the host cores: a thread pool
    (the oracle's C calls release the interpreter lock) over the instances,
    largest T n^3 first so that the pool balances; stage-steps per second."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    info = host_info()

    def one(i):
        o = oracle.lq_solve(i.A, i.B, i.c, i.Q, i.R, i.QT, i.x0)
        if adjoint:
            oracle.lq_adjoint(i.A, i.B, i.c, i.Q, i.R, i.QT, i.x0, 2 * o["x"], 2 * o["u"])
        return i.T

    order = sorted(insts, key=lambda i: -i.T * i.n ** 3)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(info["threads"]) as ex:
        stages = sum(ex.map(one, order))
    dt = time.perf_counter() - t0
    return {"value": stages / dt, "unit": "stage-steps/s", "cores": info["threads"], "kind": "oracle",
            "seconds": dt, "stages": stages, "nproc": info["nproc"], "cpu_model": info["cpu_model"]}


def solve_buffers(lqscan, plan, dev, grads=False):
    import torch
    b = {"ws": plan.new_workspace(dev), "status": torch.zeros(plan.batch, dtype=torch.int32, device=dev),
         "val": lqscan.value_buffers(plan, dev), "st": lqscan.state_buffers(plan, dev)}
    if grads:
        b["grads"] = lqscan.grad_buffers(plan, ("A", "B", "c", "Q", "R", "QT", "x0"), dev)
    return b


def batched(lqscan, workloads, dev, reps: int, with_cpu: bool) -> dict:
    """Throughput of the batched workloads (inputs generated on the device),
    each timed as graph replays of the captured solve (eager launches beside
    it), in FP64 and mixed precision, with the plain sequential path (one
    segment per instance) beside the scan, and HBM / FP64 fractions from the
    per-stage model of stage_model:
      differentiated batch  256 instances, n=12, m=4, T=4096, forward + adjoint;
      ragged batch          4096 instances, T ~ U{32..2048}, n in {2, 4, 12},
                            m = max(1, n/3), forward; also per size class and
                            with per-class segment lengths from the autotuner
                            (tuned twice to show the choice is stable)."""
    import torch

    from paper_2409_20027_amd import autotune

    res = {"timing": "ms_per_step: median of graph replays; eager_ms: eager launches"}

    def line(sizes, ms, eager, adjoint, **extra):
        stages = sum(t for _, _, t in sizes)
        d = {"ms_per_step": ms, "value": stages / (ms * 1e-3), "unit": "stage-steps/s", "eager_ms": eager,
             **fractions(sizes, ms, adjoint)}
        d.update(extra)
        return d

    # differentiated batch
    sizes = [(12, 4, 4096)] * 256
    prob = workloads.device_batch(sizes, seed=4, a_scale=0.02, r_fixed=0.1, device=dev)
    for prec in ("fp64", "mixed"):
        for mode in ("scan", "sequential"):
            plan = lqscan.Plan([12] * 256, [4] * 256, [4096] * 256, mode=mode, precision=prec)
            b = solve_buffers(lqscan, plan, dev, grads=True)
            st, val = b["st"], b["val"]
            lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])
            gx, gu = 2 * st["x"], 2 * st["u"]

            def step():
                lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])
                lqscan.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, b["grads"], b["ws"],
                                  b["status"])

            r = reps if mode == "scan" else 2
            ms = time_graph(step, r, warm=1)
            eager = time_eager(step, r)
            assert int(b["status"].abs().sum()) == 0
            res[f"batch256_T4096_fwd_adj_{prec}_{mode}"] = line(sizes, ms, eager, True, seg_len=plan.seg_len())
            del b, gx, gu, plan
    # level checkpointing: the forward keeps one carry per `stride` segments
    # (or nothing: "recompute"), the adjoint recomputes S, Gamma from it; the
    # bytes kept between forward and backward against the stored value arrays
    plan = lqscan.Plan([12] * 256, [4] * 256, [4096] * 256)
    b = solve_buffers(lqscan, plan, dev, grads=True)
    st, val = b["st"], b["val"]
    gx, gu = 2 * st["x"], 2 * st["u"]
    aws = plan.new_adjoint_ckpt_workspace(dev)
    value_bytes = sum(int(t.numel()) * 8 for t in val.values())
    stored_ms = res["batch256_T4096_fwd_adj_fp64_scan"]["ms_per_step"]
    ck = {"stored_value_bytes": value_bytes, "stored_ms_per_step": stored_ms}
    for stride in (1, 4, 16, "recompute"):
        ckpt = None if stride == "recompute" else plan.new_checkpoint(stride, dev)
        s_ = 1 if ckpt is None else stride

        def step():
            if ckpt is None:
                lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])
            else:
                lqscan.lq_solve_ckpt(plan, prob, None, val, st["x"], st["u"], st["lam"], ckpt, s_, b["ws"],
                                     b["status"])
            lqscan.lq_adjoint_ckpt(plan, prob, ckpt, s_, st["x"], st["u"], st["lam"], gx, gu, b["grads"], aws,
                                   b["status"])

        ms = time_graph(step, reps, warm=1)
        assert int(b["status"].abs().sum()) == 0
        kept = 0 if ckpt is None else plan.checkpoint_bytes(stride)
        ck[f"stride_{stride}"] = dict(line(sizes, ms, None, True), checkpoint_bytes=kept,
                                      bytes_saved=value_bytes - kept, time_added_ms=ms - stored_ms)
        del ckpt
    res["batch256_T4096_fwd_adj_fp64_checkpointed"] = ck
    del b, gx, gu, aws, plan, val, st
    del prob
    torch.cuda.empty_cache()
    if with_cpu:
        insts = workloads.cfg4_batch(batch=48, T=4096)
        res["batch256_T4096_fwd_adj_oracle"] = dict(oracle_batch(insts, True),
                                                    sample="48 of the 256 instances (seed 4), forward + adjoint")
        del insts

    # ragged batch, ordered by size class
    _, ns, ms_, Ts = workloads.cfg3_ragged_sizes()
    order = np.lexsort((Ts, ns))
    sizes = [(int(ns[i]), int(ms_[i]), int(Ts[i])) for i in order]
    prob = workloads.device_batch(sizes, seed=3, a_scale=0.05, device=dev)

    def make_prob(sel):
        return workloads.device_batch([sizes[j] for j in sel], seed=5, a_scale=0.05, device=dev)

    tuned = {}
    t0 = time.perf_counter()
    tuned["fp64"], _ = autotune.tune_sizes(sizes, make_prob, precision="fp64")
    tune_s = time.perf_counter() - t0
    again, _ = autotune.tune_sizes(sizes, make_prob, precision="fp64")
    tuned["mixed"], _ = autotune.tune_sizes(sizes, make_prob, precision="mixed")
    res["ragged4096_autotune"] = {"seconds": tune_s, "choice_fp64": autotune.seg_lens_summary(sizes, tuned["fp64"]),
                                  "choice_mixed": autotune.seg_lens_summary(sizes, tuned["mixed"]),
                                  "fp64_second_tune_same_choice": again == tuned["fp64"],
                                  "fp64_second_tune_differs_for": sum(a != b for a, b in zip(again, tuned["fp64"])),
                                  "reps": autotune.DEFAULT_REPS, "margin": autotune.MARGIN}
    for prec in ("fp64", "mixed"):
        for mode in ("scan", "sequential", "autotuned"):
            kw = {"seg_lens": tuned[prec]} if mode == "autotuned" else {"mode": mode}
            plan = lqscan.Plan([z[0] for z in sizes], [z[1] for z in sizes], [z[2] for z in sizes], precision=prec,
                               **kw)
            b = solve_buffers(lqscan, plan, dev)

            def fwd():
                lqscan.lq_solve(plan, prob, None, b["val"], b["st"]["x"], b["st"]["u"], b["st"]["lam"], b["ws"],
                                b["status"])

            r = reps if mode != "sequential" else 3
            ms = time_graph(fwd, r, warm=1)
            eager = time_eager(fwd, r)
            assert int(b["status"].abs().sum()) == 0
            res[f"ragged4096_fwd_{prec}_{mode}"] = line(sizes, ms, eager, False)
            del b, plan
    # the second tuning's choice on the same batch: what a flip costs
    plan = lqscan.Plan([z[0] for z in sizes], [z[1] for z in sizes], [z[2] for z in sizes], seg_lens=again)
    b = solve_buffers(lqscan, plan, dev)

    def fwd2():
        lqscan.lq_solve(plan, prob, None, b["val"], b["st"]["x"], b["st"]["u"], b["st"]["lam"], b["ws"], b["status"])

    res["ragged4096_autotune"]["fp64_second_tune_ms_per_step"] = time_graph(fwd2, reps, warm=1)
    res["ragged4096_autotune"]["fp64_first_tune_ms_per_step"] = res["ragged4096_fwd_fp64_autotuned"]["ms_per_step"]
    del b, plan
    del prob
    torch.cuda.empty_cache()
    # per size class (autotuned FP64 segment lengths): stage-steps/s and the
    # fraction of the class's own HBM ceiling
    for n in (2, 4, 12):
        sel = [j for j, z in enumerate(sizes) if z[0] == n]
        sub = [sizes[j] for j in sel]
        cprob = workloads.device_batch(sub, seed=6, a_scale=0.05, device=dev)
        for mode, kw in (("autotuned", {"seg_lens": [tuned["fp64"][j] for j in sel]}), ("sequential", {"mode": "sequential"})):
            plan = lqscan.Plan([z[0] for z in sub], [z[1] for z in sub], [z[2] for z in sub], **kw)
            b = solve_buffers(lqscan, plan, dev)

            def fwd():
                lqscan.lq_solve(plan, cprob, None, b["val"], b["st"]["x"], b["st"]["u"], b["st"]["lam"], b["ws"],
                                b["status"])

            ms = time_graph(fwd, reps, warm=1)
            assert int(b["status"].abs().sum()) == 0
            m_ = max(1, n // 3)
            ceil = HBM_PEAK_GBS * 1e9 / stage_model(n, m_)["bytes"]
            d = line(sub, ms, None, False, instances=len(sub), hbm_ceiling_stage_per_s=ceil)
            d["frac_of_hbm_ceiling"] = d["value"] / ceil
            res[f"ragged4096_class_n{n}_{mode}"] = d
            del b, plan
        del cprob
        torch.cuda.empty_cache()
    if with_cpu:
        rng, ns_, ms2, Ts_ = workloads.cfg3_ragged_sizes()
        pick = np.arange(0, len(Ts_), 8)
        insts = [workloads.lq_instance(np.random.default_rng(1000 + int(j)), int(ns_[j]), int(ms2[j]), int(Ts_[j]))
                 for j in pick]
        res["ragged4096_fwd_oracle"] = dict(oracle_batch(insts, False),
                                            sample=f"every 8th instance of the ragged batch ({len(insts)} "
                                                   f"instances), forward")
        del insts
    return res


def ragged_replay(lqscan, workloads, dev, replays: int) -> dict:
    """Graph replays of the captured ragged-batch forward solve (4096
    instances, default segments, FP64), for a kernel trace: under
    rocprofv3 --kernel-trace the dispatches of each replay show whether the
    gaps between the per-phase and per-level launches matter against the
    batch solve (--gap-summary reads that trace)."""
    import torch

    _, ns, ms_, Ts = workloads.cfg3_ragged_sizes()
    order = np.lexsort((Ts, ns))
    sizes = [(int(ns[i]), int(ms_[i]), int(Ts[i])) for i in order]
    prob = workloads.device_batch(sizes, seed=3, a_scale=0.05, device=dev)
    res = {}
    for mode in ("scan", "sequential"):
        plan = lqscan.Plan([z[0] for z in sizes], [z[1] for z in sizes], [z[2] for z in sizes], mode=mode)
        b = solve_buffers(lqscan, plan, dev)

        def fwd():
            lqscan.lq_solve(plan, prob, None, b["val"], b["st"]["x"], b["st"]["u"], b["st"]["lam"], b["ws"],
                            b["status"])

        res[mode] = {"ms_per_replay": time_graph(fwd, replays, warm=1), "replays": replays}
        assert int(b["status"].abs().sum()) == 0
        del b, plan
    return res


def batch_profile(lqscan, workloads, dev, reps: int) -> dict:
    """The batched workloads' kernels for counter passes: `reps` eager steps of
    the differentiated batch (256 x n=12, m=4, T=4096, forward + adjoint) and
    of the ragged batch's forward solve (4096 instances, default segments),
    with no tuning or graph capture around them."""
    import torch

    out = {}
    sizes = [(12, 4, 4096)] * 256
    prob = workloads.device_batch(sizes, seed=4, a_scale=0.02, r_fixed=0.1, device=dev)
    plan = lqscan.Plan([12] * 256, [4] * 256, [4096] * 256)
    b = solve_buffers(lqscan, plan, dev, grads=True)
    st, val = b["st"], b["val"]
    lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])
    gx, gu = 2 * st["x"], 2 * st["u"]

    def step():
        lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])
        lqscan.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, b["grads"], b["ws"], b["status"])

    out["batch256_T4096_fwd_adj_ms"] = time_eager(step, reps)
    del b, gx, gu, plan, prob, st, val
    torch.cuda.empty_cache()
    _, ns, ms_, Ts = workloads.cfg3_ragged_sizes()
    order = np.lexsort((Ts, ns))
    rs = [(int(ns[i]), int(ms_[i]), int(Ts[i])) for i in order]
    prob = workloads.device_batch(rs, seed=3, a_scale=0.05, device=dev)
    plan = lqscan.Plan([z[0] for z in rs], [z[1] for z in rs], [z[2] for z in rs])
    b = solve_buffers(lqscan, plan, dev)

    def fwd():
        lqscan.lq_solve(plan, prob, None, b["val"], b["st"]["x"], b["st"]["u"], b["st"]["lam"], b["ws"], b["status"])

    out["ragged4096_fwd_ms"] = time_eager(fwd, reps)
    return out


def gap_summary(path: str, split_us: float = 5.0) -> dict:
    """Launch gaps inside graph replays, from a rocprofv3 kernel trace (CSV
    with Kernel_Name, Start_Timestamp, End_Timestamp): the library's
    dispatches (kernel names in namespace lqk) ordered by start; a replay is a
    run of them whose start-to-previous-end gaps stay below split_us
    (consecutive replays are separated by event records and a host wait).  Per
    replay: dispatches, span, busy time (union of kernel intervals), idle time
    between kernels and its share of the span."""
    import csv

    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    groups, cur = [], []
    for a, b, k in rows:
        ours = "lqk::" in k
        if cur and (not ours or a - cur[-1][1] > split_us * 1e3):
            groups.append(cur)
            cur = []
        if ours:
            cur.append((a, b, k))
    if cur:
        groups.append(cur)
    out = []
    for g in groups:
        if len(g) < 3:
            continue
        span = g[-1][1] - g[0][0]
        busy, end = 0, g[0][0]
        for a, b, _ in g:
            busy += max(0, b - max(a, end))
            end = max(end, b)
        out.append({"dispatches": len(g), "span_us": span / 1e3, "busy_us": busy / 1e3,
                    "idle_us": (span - busy) / 1e3, "idle_frac": (span - busy) / span if span else 0.0})
    return {"replays": out, "max_idle_frac": max((o["idle_frac"] for o in out), default=None)}


def paper_ip_solves(lqscan, workloads, reps: int, with_cpu: bool) -> dict:
    """The paper's own experiments (Sec. V): interior-point solves of the
    torque-limited pendulum and force-limited cart-pole swing-ups at horizons
    N = 20 .. 1000, wall time of the whole solve (host loop over Newton steps
    with one gradient-norm readback per step), parallel-in-time path against
    the sequential-in-time path on the same GPU (one segment per solve), and
    the FP64 oracle on one host core.  Costs and time spans are proposed (the
    paper does not print them)."""
    import torch
    args = dict(mu0=workloads.IP_MU0, zeta=workloads.IP_ZETA, mu_min=workloads.IP_MU_MIN, tol=workloads.IP_TOL,
                max_iter=workloads.IP_MAX_ITER, alpha0=workloads.NMPC_ALPHA0, nu0=workloads.NMPC_NU0)
    out = {"unit": "ms per interior-point solve", "seg_len_parallel": workloads.IP_SEG_LEN}
    if with_cpu:
        import oracle
    for name, mk in (("pendulum", workloads.pendulum_problem), ("cartpole", workloads.cartpole_problem)):
        rows = {}
        for N in workloads.PAPER_HORIZONS:
            p = mk(N)
            row = {}
            for label, kw, r in (("parallel_ms", dict(seg_len=workloads.IP_SEG_LEN), reps),
                                 ("sequential_ms", dict(mode="sequential"), 1)):
                s = lqscan.NewtonMPC(p, **kw)
                o = s.ip_solve(**args, trace=False)   # warm-up (first launches, allocations)
                torch.cuda.synchronize()
                ts = []
                for _ in range(r):
                    t0 = time.perf_counter()
                    o = s.ip_solve(**args, trace=False)
                    torch.cuda.synchronize()
                    ts.append((time.perf_counter() - t0) * 1e3)
                row[label] = min(ts)
                row["newton_iters" if label == "parallel_ms" else "newton_iters_sequential"] = o["iters"]
            if with_cpu:
                t0 = time.perf_counter()
                ro = oracle.nmpc_ip_solve(p, **args)
                row["oracle_ms"] = (time.perf_counter() - t0) * 1e3
                row["oracle_newton_iters"] = ro["iters"]
            rows[str(N)] = row
        out[name] = rows
    return out


def paper_admm_solves(lqscan, workloads, with_cpu: bool, seq_max_n: int = 200) -> dict:
    """ADMM solves of the same swing-ups (Sec. II-C, Sec. V: rho = 1 pendulum,
    0.5 cart-pole, per unit time; stop at |r_p|, |r_d| <= 1e-2): wall time of
    the whole solve, parallel path (segments of 4) for every N, the sequential
    path up to seq_max_n (it grows linearly and the cart-pole needs thousands
    of Newton iterations), and the oracle on one host core."""
    import torch
    out = {"unit": "ms per ADMM solve", "seg_len_parallel": workloads.IP_SEG_LEN}
    if with_cpu:
        import oracle
    for name, mk in (("pendulum", workloads.pendulum_problem), ("cartpole", workloads.cartpole_problem)):
        rows = {}
        for N in workloads.PAPER_HORIZONS:
            p = mk(N)
            args = dict(rho=workloads.ADMM_RHO[name] * p.h, eps=workloads.ADMM_EPS, tol=workloads.IP_TOL,
                        max_iter=workloads.IP_MAX_ITER, max_admm=workloads.ADMM_MAX_ITER,
                        alpha0=workloads.NMPC_ALPHA0, nu0=workloads.NMPC_NU0)
            row = {}
            for label, kw in (("parallel_ms", dict(seg_len=workloads.IP_SEG_LEN)), ("sequential_ms", dict(mode="sequential"))):
                if label == "sequential_ms" and N > seq_max_n:
                    continue
                s = lqscan.NewtonMPC(p, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                o = s.admm_solve(**args)
                torch.cuda.synchronize()
                row[label] = (time.perf_counter() - t0) * 1e3
                if label == "parallel_ms":
                    row["admm_iters"], row["newton_iters"] = o["admm_iters"], o["newton_iters"]
            if with_cpu:
                t0 = time.perf_counter()
                ro = oracle.nmpc_admm_solve(p, **args)
                row["oracle_ms"] = (time.perf_counter() - t0) * 1e3
                row["oracle_admm_iters"] = ro["admm_iters"]
            rows[str(N)] = row
        out[name] = rows
    return out


def paper_mpc(lqscan, workloads, with_cpu: bool, batches=(1, 64, 1024, 4096)) -> dict:
    """Receding-horizon MPC of Sec. V (N = 60 at 100 Hz, 4 s = 400 plant steps,
    fixed IP budget per step, warm start): wall time of whole closed-loop
    simulations, a batch of simulations from different initial states in one
    launch sequence, against the oracle's sequential simulation on one host
    core."""
    import torch
    kw = dict(mu_levels=workloads.MPC_MU_LEVELS, iters=workloads.MPC_ITERS, alpha0=workloads.NMPC_ALPHA0,
              nu0=workloads.NMPC_NU0)
    out = {"unit": "closed-loop simulations per second", "plant_steps": workloads.MPC_STEPS,
           "horizon": workloads.MPC_N}
    if with_cpu:
        import oracle
    for name in ("pendulum", "cartpole"):
        rows = {}
        for B in batches:
            xs = workloads.mpc_initial_states(name, B, seed=5)
            p = workloads.mpc_problem(name, xs if B > 1 else xs[0])
            s = lqscan.NewtonMPC(p)
            s.mpc_simulate(2, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            o = s.mpc_simulate(workloads.MPC_STEPS, **kw)
            dt = time.perf_counter() - t0
            x = o["x"] if B > 1 else o["x"][None]
            settled = float(np.mean(np.max(np.abs(x[:, -1] - p.xref[0]), axis=1) < 0.05))
            rows[str(B)] = {"s": dt, "sims_per_s": B / dt, "seg_len": s.plan.seg_len(), "settled_fraction": settled}
        if with_cpu:
            xs = workloads.mpc_initial_states(name, 1, seed=5)
            t0 = time.perf_counter()
            oracle.nmpc_mpc_simulate(workloads.mpc_problem(name, xs[0]), xs[0], steps=workloads.MPC_STEPS, **kw)
            rows["oracle_one_core"] = {"s": time.perf_counter() - t0}
            rows["oracle_one_core"]["sims_per_s"] = 1.0 / rows["oracle_one_core"]["s"]
        out[name] = rows
    return out


def cv_rollout(lqscan, plan, prob, val, ws, status, inst, with_cpu: bool, reps: int = 20) -> dict:
    """lq_rollout (closed-loop maps) and lq_rollout_cv (conditional value
    functions, eq:value-fun-prefix-sum) from the same value pass: time per
    call, the CV phases, and the CV states' error against the oracle's."""
    import oracle
    import torch
    dev = prob["A"].device
    out = {}
    for name, fn in (("affine", lqscan.lq_rollout), ("cv", lqscan.lq_rollout_cv)):
        st = lqscan.state_buffers(plan, dev)
        fn(plan, prob, val, st["x"], st["u"], st["lam"], ws, status)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn(plan, prob, val, st["x"], st["u"], st["lam"], ws, status)
        b.record()
        torch.cuda.synchronize()
        out[f"{name}_us"] = a.elapsed_time(b) / reps * 1e3
        if name == "cv":
            plan.set_timing(["cv_fold", "cv_scan", "cv_start", "roll_apply"], capacity=4 * reps + 8)
            for _ in range(reps):
                fn(plan, prob, val, st["x"], st["u"], st["lam"], ws, status)
            out["cv_phase_us"] = {k: v[0] / reps * 1e3 for k, v in plan.phase_times().items()}
            plan.set_timing([], 0)
            t0 = time.perf_counter()
            xc = oracle.lq_states_cv(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
            cpu_s = time.perf_counter() - t0
            x = st["x"].cpu().numpy().reshape(inst.T + 1, inst.n)
            out["err_x_vs_oracle_cv"] = float(np.max(np.abs(x - xc)) / np.max(np.abs(xc)))
            if with_cpu:
                out["oracle_cv_states_s"] = cpu_s
    assert int(status.abs().sum()) == 0, "numerical failure reported"
    out["what"] = ("rollout of the value pass's result at n=12, m=4, T=16384: closed-loop affine scan vs "
                   "prefix conditional value functions (fold + prefix scan + segment-start solve + sweep)")
    return out


def cfg0_small(lqscan, workloads, dev, replays: int, with_cpu: bool) -> dict:
    """The small case (n=2, m=1, T=64, FP64): latency of the forward solve and
    of forward + adjoint as graph replays, scan and sequential, the error
    against the oracle, and the oracle's time per solve on one host core."""
    import oracle
    inst = workloads.cfg0_small()
    prob = lqscan.to_device(workloads.pack([inst]), dev)
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    gref = oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * ref["x"], 2 * ref["u"])
    out = {"workload": "time-varying LQ, n=2, m=1, T=64, one instance, FP64"}
    for mode in ("scan", "sequential"):
        plan = lqscan.Plan([2], [1], [64], mode=mode)
        b = solve_buffers(lqscan, plan, dev, grads=True)
        st, val = b["st"], b["val"]

        def fwd():
            lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])

        fwd()
        gx, gu = 2 * st["x"], 2 * st["u"]

        def step():
            fwd()
            lqscan.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, b["grads"], b["ws"], b["status"])

        lat_f = time_graph(fwd, replays) * 1e3
        lat_s = time_graph(step, replays) * 1e3
        assert int(b["status"].abs().sum()) == 0
        err = max(float(np.max(np.abs(st["x"].cpu().numpy().reshape(65, 2) - ref["x"])) / np.max(np.abs(ref["x"]))),
                  max(float(np.max(np.abs(b["grads"][k].cpu().numpy().reshape(gref[k].shape) - gref[k]))
                            / np.max(np.abs(gref[k]))) for k in ("A", "Q", "x0")))
        out[mode] = {"forward_latency_us": lat_f, "forward_adjoint_latency_us": lat_s,
                     "stage_steps_per_s_fwd_adj": 64 / (lat_s * 1e-6), "seg_len": plan.seg_len(),
                     "err_vs_oracle": err}
    if with_cpu:
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 1.0:
            r = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
            oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * r["x"], 2 * r["u"])
            reps += 1
        us = (time.perf_counter() - t0) / reps * 1e6
        out["oracle_one_core"] = {"forward_adjoint_us": us, "stage_steps_per_s_fwd_adj": 64 / (us * 1e-6)}
    return out


def cfg1_newton(lqscan, workloads, reps: int, with_cpu: bool) -> dict:
    """The interior-point Newton loop on the tanh model (n=4, m=1, T=1024, six
    barrier levels of ten Newton steps), FP64 and mixed: wall time of the
    60-step solve with every step replayed from one captured HIP graph (no
    host synchronisation inside), ms per Newton step and stage-steps/s
    (T stages per Newton step); final cost against the FP64 oracle's and the
    number of decisions that differ; the oracle's loop on one host core."""
    import torch

    import oracle
    p = workloads.nmpc_problem(seed=1, T=1024)
    levels, iters = workloads.NMPC_MU_LEVELS, workloads.NMPC_ITERS_PER_LEVEL
    a0, nu0 = workloads.NMPC_ALPHA0, workloads.NMPC_NU0
    steps = len(levels) * iters
    t0 = time.perf_counter()
    ref = oracle.nmpc_solve(p, levels, iters, a0, nu0)
    cpu_s = time.perf_counter() - t0
    out = {"workload": "tanh-network dynamics, n=4, m=1, T=1024, 6 barrier levels x 10 Newton steps",
           "newton_steps": steps}
    for prec in ("fp64", "mixed"):
        s = lqscan.NewtonMPC(p, precision=prec)
        trace = s.run(levels, iters, a0, nu0)
        g = s._capture_step()

        def solve():
            s.init(a0, nu0)
            for mu in levels:
                s._sc[:, lqscan.NMPC_MU] = mu
                for _ in range(iters):
                    g.replay()

        solve()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            solve()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ms = float(np.median(ts)) * 1e3
        out[prec] = {"ms_per_solve": ms, "ms_per_newton_step": ms / steps,
                     "stage_steps_per_s": p.T * steps / (ms * 1e-3),
                     "final_cost_rel_err": abs(trace["cost"][-1] - ref["cost"][-1]) / abs(ref["cost"][-1]),
                     "decision_mismatches": int(np.sum(trace["accept"] != ref["accept"]))}
    if with_cpu:
        out["oracle_one_core"] = {"ms_per_solve": cpu_s * 1e3, "ms_per_newton_step": cpu_s * 1e3 / steps,
                                  "stage_steps_per_s": p.T * steps / cpu_s}
    return out


def cfg2_mixed(lqscan, dev, prob, inst, ref, gref, steps: int, replays: int) -> dict:
    """The headline workload (n=12, m=4, T=16384, forward + adjoint) in mixed
    precision: FP32 products, FP64 inverses, Cholesky factors and
    symmetrisation; errors against the FP64 oracle."""
    n, m, T = inst.n, inst.m, inst.T
    plan = lqscan.Plan([n], [m], [T], precision="mixed")
    b = solve_buffers(lqscan, plan, dev, grads=True)
    st, val = b["st"], b["val"]

    def fwd():
        lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], b["ws"], b["status"])

    fwd()
    gx, gu = 2 * st["x"], 2 * st["u"]

    def step():
        fwd()
        lqscan.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, b["grads"], b["ws"], b["status"])

    ms = time_eager(step, steps, warm=3)
    lat = time_graph(fwd, replays) * 1e3
    assert int(b["status"].abs().sum()) == 0

    def rel(a, r):
        return float(np.max(np.abs(a - r)) / np.max(np.abs(r)))

    err = {"x": rel(st["x"].cpu().numpy().reshape(T + 1, n), ref["x"]),
           "u": rel(st["u"].cpu().numpy().reshape(T, m), ref["u"]),
           "S": rel(val["S"].cpu().numpy().reshape(T + 1, n, n), ref["S"]),
           **{f"grad_{k}": rel(b["grads"][k].cpu().numpy().reshape(gref[k].shape), gref[k]) for k in ("A", "Q", "x0")}}
    return {"ms_per_step": ms, "value": T / (ms * 1e-3), "unit": "stage-steps/s", "dtype": "f32 products, f64 inverses",
            "latency_us_T16384_forward": lat, "err_vs_oracle": err, **fractions([(n, m, T)], ms, True)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--T", type=int, default=16384)
    ap.add_argument("--seg-len", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-seq", action="store_true")
    ap.add_argument("--replays", type=int, default=100)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workloads")
    ap.add_argument("--no-paper", action="store_true", help="skip the pendulum / cart-pole interior-point solves")
    ap.add_argument("--no-cv", action="store_true", help="skip the conditional-value rollout comparison")
    ap.add_argument("--calib", action="store_true",
                    help="also launch one plain copy of 256 MiB (scale reference for HBM counters)")
    ap.add_argument("--section", choices=("paper_ip", "paper_admm", "paper_mpc", "batched", "cfg0", "cfg1",
                                          "ragged_replay", "batch_profile"),
                    default=None, help="run only this section (GPU paths only) and print its JSON")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline workload only (no mixed-precision, small-case or Newton sections)")
    ap.add_argument("--gap-summary", metavar="KERNEL_TRACE_CSV", default=None,
                    help="summarise launch gaps inside graph replays from a rocprofv3 kernel trace (no GPU)")
    args = ap.parse_args()
    if args.gap_summary:
        print(json.dumps(gap_summary(args.gap_summary)))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: sharding the horizon or the batch over several GPUs is a "
              "design in this repository, not a built path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2409_20027_amd import lqscan, workloads

    dev = torch.device("cuda:0")
    if args.section:
        fn = {"paper_ip": lambda: paper_ip_solves(lqscan, workloads, 3, False),
              "paper_admm": lambda: paper_admm_solves(lqscan, workloads, False),
              "paper_mpc": lambda: paper_mpc(lqscan, workloads, False),
              "batched": lambda: batched(lqscan, workloads, dev, max(3, min(args.steps, 10)), False),
              "cfg0": lambda: cfg0_small(lqscan, workloads, dev, args.replays, False),
              "cfg1": lambda: cfg1_newton(lqscan, workloads, 3, False),
              "ragged_replay": lambda: ragged_replay(lqscan, workloads, dev, max(3, min(args.steps, 10))),
              "batch_profile": lambda: batch_profile(lqscan, workloads, dev, max(1, min(args.steps, 10)))}[args.section]
        print(json.dumps({args.section: fn()}))
        return

    inst = workloads.cfg2_long(T=args.T)
    packed = workloads.pack([inst])
    prob = lqscan.to_device(packed, dev)
    n, m, T = inst.n, inst.m, inst.T

    plan = lqscan.Plan([n], [m], [T], seg_len=args.seg_len)
    ws = plan.new_workspace(dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    val = lqscan.value_buffers(plan, dev)
    st = lqscan.state_buffers(plan, dev)
    gnames = ("A", "B", "c", "Q", "R", "QT", "x0")
    grads = lqscan.grad_buffers(plan, gnames, dev)

    def forward():
        lqscan.lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)

    forward()
    torch.cuda.synchronize()
    gx, gu = 2 * st["x"], 2 * st["u"]   # loss gradients, fixed inputs of the adjoint

    def step():
        forward()
        lqscan.lq_adjoint(plan, prob, val, st["x"], st["u"], st["lam"], gx, gu, grads, ws, status)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.calib:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)   # one elementwise kernel: reads and writes 256 MiB once
        torch.cuda.synchronize()
        del src, dst

    # profiling pass: every phase timed with events (not the headline number)
    prof_steps = min(args.steps, 10)
    plan.set_timing(list(lqscan.PHASES), capacity=prof_steps * len(lqscan.PHASES) + 8)
    for _ in range(prof_steps):
        step()
    phases = plan.phase_times()
    plan.set_timing([], 0)
    breakdown = {k: v[0] / prof_steps for k, v in phases.items()}
    models = kernel_models(n, m, T, plan.seg_len())
    # every modelled phase against both peaks: algorithmic bytes and flops per
    # step over the phase's time per step
    phase_roofline = {}
    for ph, mdl_ in models.items():
        if ph not in breakdown or breakdown[ph] <= 0:
            continue
        sec = breakdown[ph] * 1e-3
        gbs_, tf_ = mdl_["bytes"] / sec / 1e9, mdl_["flops"] / sec / 1e12
        phase_roofline[ph] = {"us_per_step": breakdown[ph] * 1e3, "GB/s": gbs_, "hbm_frac": gbs_ / HBM_PEAK_GBS,
                              "TFLOP/s": tf_, "fp64_frac": tf_ / FP64_PEAK_TFLOPS}
    dominant = max((k for k in breakdown if k in models), key=lambda k: breakdown[k])

    # timed pass: events only around the dominant kernel
    plan.set_timing([dominant], capacity=args.steps + 8)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    dom_ms, dom_launches = plan.phase_times()[dominant]
    plan.set_timing([], 0)
    ms_per_step = total_ms / args.steps
    assert int(status.abs().sum()) == 0, "numerical failure reported"

    # error of this run's result against the FP64 oracle (every stage)
    import oracle
    ref = oracle.lq_solve(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0)
    gref = oracle.lq_adjoint(inst.A, inst.B, inst.c, inst.Q, inst.R, inst.QT, inst.x0, 2 * ref["x"], 2 * ref["u"])

    def rel(a, b):
        return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))

    err = {"x": rel(st["x"].cpu().numpy().reshape(T + 1, n), ref["x"]),
           "u": rel(st["u"].cpu().numpy().reshape(T, m), ref["u"]),
           "S": rel(val["S"].cpu().numpy().reshape(T + 1, n, n), ref["S"]),
           "grad_A": rel(grads["A"].cpu().numpy().reshape(T, n, n), gref["A"]),
           "grad_Q": rel(grads["Q"].cpu().numpy().reshape(T, n, n), gref["Q"]),
           "grad_x0": rel(grads["x0"].cpu().numpy(), gref["x0"])}

    # forward latency at T: median of graph replays of the captured forward solve
    lat_us = None
    try:
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            forward()
            torch.cuda.synchronize()
            with torch.cuda.graph(g, stream=s):
                forward()
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
    except Exception as e:
        print(f"graph replay failed: {e!r}", file=sys.stderr)

    # the plain sequential path on the same GPU (one segment per instance)
    seq = None
    if not args.no_seq:
        splan = lqscan.Plan([n], [m], [T], mode="sequential")
        sws = splan.new_workspace(dev)

        def sstep():
            lqscan.lq_solve(splan, prob, None, val, st["x"], st["u"], st["lam"], sws, status)
            lqscan.lq_adjoint(splan, prob, val, st["x"], st["u"], st["lam"], gx, gu, grads, sws, status)

        sstep()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 2
        a.record()
        for _ in range(reps):
            sstep()
        b.record()
        torch.cuda.synchronize()
        seq_ms = a.elapsed_time(b) / reps
        seq = {"ms_per_step": seq_ms, "value": T / (seq_ms * 1e-3), "unit": "stage-steps/s",
               "what": "same step (forward + adjoint) with one segment: sequential recursions on the GPU"}

    # the two rollouts of the same value pass: closed-loop maps (lq_rollout)
    # and conditional value functions (lq_rollout_cv)
    cv = None
    if not args.no_cv:
        cv = cv_rollout(lqscan, plan, prob, val, ws, status, inst, not args.no_cpu)

    mdl = models[dominant]
    # average duration of one kernel launch of the dominant phase (a scan phase
    # is timed as a whole: its time divided by its number of levels)
    avg_s = dom_ms / max(dom_launches, 1) / mdl["launches"] * 1e-3
    flops = mdl["flops"] / mdl["launches"]
    nbytes = mdl["bytes"] / mdl["launches"]
    tf = flops / avg_s / 1e12
    gbs = nbytes / avg_s / 1e9
    if tf / FP64_PEAK_TFLOPS >= gbs / HBM_PEAK_GBS:
        roof = {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP64_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS}
    roof.update({"traffic": stored_traffic(dominant), "kernel": dominant, "avg_launch_us": avg_s * 1e6,
                 "launches_per_step": mdl["launches"], "flops_per_launch": flops,
                 "algorithmic_bytes_per_launch": nbytes,
                 "units_per_step": mdl["units"], "unit": roof["unit"], "unit_of_work": mdl["unit_name"],
                 "other_bound": ({"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
                                 if roof["bound"] == "mfma" else
                                 {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / FP64_PEAK_TFLOPS})})

    out = {"metric": "LQ stage-steps/sec (forward + adjoint, n=12, m=4, T=16384, FP64)",
           "value": T * args.steps / (total_ms * 1e-3), "unit": "stage-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"time-varying LQ, n={n}, m={m}, T={T}, one instance; value scan + rollout "
                                  f"+ adjoint per step", "seg_len": plan.seg_len()},
           "latency_us_T16384_forward": lat_us,
           "err_vs_oracle": err,
           "sequential_gpu": seq,
           "kernel_ms_per_step": breakdown,
           "phase_roofline": phase_roofline,
           "cv_rollout": cv,
           "roofline": roof}
    if not args.only_headline:
        out["mixed_precision"] = cfg2_mixed(lqscan, dev, prob, inst, ref, gref, args.steps, args.replays)
        out["small_case"] = cfg0_small(lqscan, workloads, dev, args.replays, not args.no_cpu)
        out["newton_ip"] = cfg1_newton(lqscan, workloads, 3, not args.no_cpu)
    if not args.no_batch:
        out["batched"] = batched(lqscan, workloads, dev, max(3, min(args.steps, 10)), not args.no_cpu)
    if not args.no_paper:
        out["paper_ip_solves"] = paper_ip_solves(lqscan, workloads, 3, not args.no_cpu)
        out["paper_admm_solves"] = paper_admm_solves(lqscan, workloads, not args.no_cpu)
        out["paper_mpc"] = paper_mpc(lqscan, workloads, not args.no_cpu)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
