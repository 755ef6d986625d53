"""Segment-length autotuner for ragged batches.

The scan trades work for depth.  Folding L stages per segment and scanning the
T/L segment elements does about twice the sequential work with depth
O(L + log(T/L)), while L = T is the plain sequential recursion (least work,
depth T).  The best L depends on the state size, the horizon and on how many
instances share the GPU, so it is measured instead of assumed.

Instances are grouped into classes (n, m, T bucket).  For each class the tuner
times the forward solve (lq_solve) of the class's instances
for every candidate L with HIP events and keeps the fastest.  Results are cached
in a JSON file keyed by class, batch-size bucket and precision, and returned as
one segment length per instance for lq_plan_create_seg.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

DEFAULT_CANDIDATES = (0, 4, 8, 16, 32, 64, -1)   # 0 = library default, -1 = sequential (L = T)


def _bucket(v: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, v)))))


def class_key(n, m, T, count, precision):
    return f"n{n}_m{m}_T{_bucket(T)}_B{_bucket(count)}_{precision}"


def _time_forward(lq, insts, seg, precision, reps, torch):
    from . import workloads
    prob = lq.to_device(workloads.pack(insts))
    plan = lq.Plan([i.n for i in insts], [i.m for i in insts], [i.T for i in insts], precision=precision,
                   seg_lens=[i.T if seg < 0 else seg for i in insts])
    ws = plan.new_workspace()
    status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
    val = lq.value_buffers(plan)
    st = lq.state_buffers(plan)

    def fwd():
        lq.lq_solve(plan, prob, None, val, st["x"], st["u"], None, ws, status)

    fwd()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fwd()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(insts, *, precision="fp64", candidates=DEFAULT_CANDIDATES, reps=3, cache_path=None,
         sample_per_class=None):
    """Per-instance segment lengths for a ragged batch (list of LQInstance).

    Classes already in the cache are not re-timed.  `sample_per_class` limits
    the number of instances of a class that are timed (the whole class when
    None).  Returns (seg_lens, report) where report maps class -> {L: ms}.
    """
    import torch

    from . import lqscan as lq

    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    classes = {}
    for idx, i in enumerate(insts):
        classes.setdefault((i.n, i.m, _bucket(i.T)), []).append(idx)
    report, choice = {}, {}
    for (n, m, tb), members in classes.items():
        key = class_key(n, m, tb, len(members), precision)
        if key in cache:
            choice[(n, m, tb)] = cache[key]["L"]
            continue
        sel = members if sample_per_class is None else members[:sample_per_class]
        group = [insts[j] for j in sel]
        times = {}
        for L in candidates:
            times[L] = _time_forward(lq, group, L, precision, reps, torch)
        best = min(times, key=times.get)
        choice[(n, m, tb)] = best
        report[key] = {str(k): v for k, v in times.items()}
        cache[key] = {"L": best, "ms": report[key]}
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    seg_lens = []
    for i in insts:
        L = choice[(i.n, i.m, _bucket(i.T))]
        seg_lens.append(i.T if L < 0 else L)
    return seg_lens, report


def seg_lens_summary(insts, seg_lens):
    """Text summary: chosen L per (n, T-bucket)."""
    rows = {}
    for i, L in zip(insts, seg_lens):
        rows.setdefault((i.n, _bucket(i.T)), set()).add("seq" if L >= i.T else L)
    return {f"n={n},T<={tb}": sorted(map(str, v)) for (n, tb), v in sorted(rows.items())}


__all__ = ["tune", "class_key", "seg_lens_summary", "DEFAULT_CANDIDATES", "np"]
