"""Segment-length autotuner for ragged batches.

The scan trades work for depth.  Folding L stages per segment and scanning the
T/L segment elements does about twice the sequential work with depth
O(L + log(T/L)), while L = T is the plain sequential recursion (least work,
depth T).  The best L depends on the state size, the horizon and on how many
instances share the GPU, so it is measured instead of assumed.

Instances are grouped into classes (n, m, T bucket).  For each class the tuner
times the forward solve (lq_solve) of the class's instances for every
candidate L with HIP events (the median of `reps` timed samples, each
bracketed by its own events and repeating the solve until it lasts at least
MIN_SAMPLE_MS).  Of the candidates within MARGIN of the fastest it takes the
first in the candidate order (the library default L = 0 first), and keeps it
only if it beats the default by more than MARGIN on the medians and then wins
CONFIRM_WINS of CONFIRM_PAIRS interleaved head-to-head samples against it;
otherwise the default stays.  Candidates that time within noise of each other
therefore do not flip the choice from one tuning to the next.  A class timed
alone can prefer the scan where, inside the whole batch, the GPU is already
full and the sequential recursion (least work) is faster; so the per-class
choice is then refined on the whole batch, switching classes to L = T while
that makes the batch faster by more than MARGIN (with the same confirmation).  Results are cached in a JSON file keyed by
class, batch-size bucket and precision, and returned as one segment length per
instance for lq_plan_create_seg.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

DEFAULT_CANDIDATES = (0, 4, 8, 16, 32, 64, -1)   # 0 = library default, -1 = sequential (L = T)
DEFAULT_REPS = 5
# A candidate replaces the current choice only if it is faster by more than
# this fraction (repeated timings of one configuration vary by a few percent).
MARGIN = 0.05


def _bucket(v: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, v)))))


def class_key(n, m, T, count, precision):
    return f"n{n}_m{m}_T{_bucket(T)}_B{_bucket(count)}_{precision}"


# A timed sample repeats the solve until it lasts at least this long, so that
# classes whose solve takes a few microseconds are not timed at the
# resolution of a single launch.
MIN_SAMPLE_MS = 0.5
# A candidate that beats the default on the medians must also win this many
# of CONFIRM_PAIRS interleaved head-to-head samples against it.
CONFIRM_PAIRS = 8
CONFIRM_WINS = 6


class _Timer:
    """Forward solves (lq_solve) of one plan, timed in samples of `k` calls
    bracketed by HIP events; ms per call."""

    def __init__(self, lq, prob, sizes, seg_lens, precision, torch):
        self.torch = torch
        plan = lq.Plan([z[0] for z in sizes], [z[1] for z in sizes], [z[2] for z in sizes], precision=precision,
                       seg_lens=seg_lens)
        ws = plan.new_workspace()
        status = torch.zeros(plan.batch, dtype=torch.int32, device="cuda")
        val = lq.value_buffers(plan)
        st = lq.state_buffers(plan)
        self._keep = (plan, ws, status, val, st)

        def fwd():
            lq.lq_solve(plan, prob, None, val, st["x"], st["u"], None, ws, status)

        self.fwd = fwd
        fwd()
        torch.cuda.synchronize()
        one = self.sample(1)
        self.k = max(1, int(np.ceil(MIN_SAMPLE_MS / max(one, 1e-3))))

    def sample(self, k=None):
        k = self.k if k is None else k
        a, b = self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(k):
            self.fwd()
        b.record()
        self.torch.cuda.synchronize()
        return a.elapsed_time(b) / k

    def median(self, reps):
        return float(np.median([self.sample() for _ in range(reps)]))


def _time_forward_lens(lq, prob, sizes, seg_lens, precision, reps, torch):
    return _Timer(lq, prob, sizes, seg_lens, precision, torch).median(reps)


def _pick(times: dict, default, order):
    """Among the candidates within MARGIN of the fastest, the first in `order`
    (so that candidates timing within noise of each other do not flip the
    choice from one tuning to the next); it replaces `default` only if it beats
    it by more than MARGIN."""
    fastest = min(times.values())
    near = [L for L in order if times[L] <= (1.0 + MARGIN) * fastest]
    pick = default if default in near else near[0]
    return pick if times[pick] < (1.0 - MARGIN) * times[default] else default


def _confirmed(ta: "_Timer", tb: "_Timer") -> bool:
    """True if b is faster than a in at least CONFIRM_WINS of CONFIRM_PAIRS
    interleaved samples and by more than MARGIN on their medians."""
    pa, pb = [], []
    for _ in range(CONFIRM_PAIRS):
        pa.append(ta.sample())
        pb.append(tb.sample())
    wins = sum(b < a for a, b in zip(pa, pb))
    return wins >= CONFIRM_WINS and float(np.median(pb)) < (1.0 - MARGIN) * float(np.median(pa))


def tune_sizes(sizes, make_prob, *, precision="fp64", candidates=DEFAULT_CANDIDATES, reps=DEFAULT_REPS, cache_path=None,
               sample_per_class=None, refine=True):
    """Per-instance segment lengths for a batch given as (n, m, T) sizes.

    make_prob(list of indices) returns the packed device problem of those
    instances (in that order).  Classes already in the cache are not
    re-timed; `sample_per_class` limits the number of instances of a class
    that are timed (the whole class when None).  Returns (seg_lens, report)
    where report maps class -> {L: ms}.  With refine, classes are then
    switched to the sequential recursion where that makes the whole batch
    faster (timed on the whole batch).
    """
    import torch

    from . import lqscan as lq

    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    classes = {}
    for idx, (n, m, T) in enumerate(sizes):
        classes.setdefault((n, m, _bucket(T)), []).append(idx)
    report, choice = {}, {}
    for (n, m, tb), members in classes.items():
        key = class_key(n, m, tb, len(members), precision)
        if key in cache:
            choice[(n, m, tb)] = cache[key]["L"]
            continue
        sel = members if sample_per_class is None else members[:sample_per_class]
        prob = make_prob(sel)
        sub = [sizes[j] for j in sel]
        timers = {L: _Timer(lq, prob, sub, [z[2] if L < 0 else L for z in sub], precision, torch)
                  for L in candidates}
        times = {L: t.median(reps) for L, t in timers.items()}
        best = _pick(times, candidates[0], candidates)
        if best != candidates[0] and not _confirmed(timers[candidates[0]], timers[best]):
            best = candidates[0]
        del prob, timers
        choice[(n, m, tb)] = best
        report[key] = {str(k): v for k, v in times.items()}
        cache[key] = {"L": best, "ms": report[key]}
    if refine and report and len(classes) > 1:   # (a batch answered from the cache is final)
        # A class timed alone may prefer the scan where, inside the whole batch
        # (enough instances to fill the GPU), the sequential recursion is
        # faster: try switching each class (largest first) to L = T on the
        # whole batch and keep a switch if the batch gets faster.
        prob = make_prob(list(range(len(sizes))))

        def seglens(ch):
            return [T if ch[(n, m, _bucket(T))] < 0 else ch[(n, m, _bucket(T))] for n, m, T in sizes]

        def timer(ch):
            return _Timer(lq, prob, sizes, seglens(ch), precision, torch)

        cur = timer(choice)
        best_t = cur.median(reps)
        order = sorted(classes, key=lambda k: -sum(sizes[j][2] for j in classes[k]))
        for key3 in order:
            if choice[key3] < 0:
                continue
            trial = dict(choice)
            trial[key3] = -1
            tt = timer(trial)
            t = tt.median(reps)
            if t < (1.0 - MARGIN) * best_t and _confirmed(cur, tt):
                best_t, choice, cur = t, trial, tt
                ck = class_key(key3[0], key3[1], key3[2], len(classes[key3]), precision)
                cache[ck] = {"L": -1, "ms": cache.get(ck, {}).get("ms", {}), "refined_on_batch": True}
        # and the plain sequential recursion for every class
        allseq = {k: -1 for k in choice}
        ta = timer(allseq)
        t = ta.median(reps)
        if t < (1.0 - MARGIN) * best_t and _confirmed(cur, ta):
            best_t, choice = t, allseq
            for key3 in classes:
                ck = class_key(key3[0], key3[1], key3[2], len(classes[key3]), precision)
                cache[ck] = {"L": -1, "ms": cache.get(ck, {}).get("ms", {}), "refined_on_batch": True}
        report["batch_ms"] = best_t
        del prob
    if cache_path:
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    seg_lens = []
    for n, m, T in sizes:
        L = choice[(n, m, _bucket(T))]
        seg_lens.append(T if L < 0 else L)
    return seg_lens, report


def tune(insts, *, precision="fp64", candidates=DEFAULT_CANDIDATES, reps=DEFAULT_REPS, cache_path=None,
         sample_per_class=None, refine=True):
    """tune_sizes for a list of LQInstance (host arrays, packed and uploaded per class)."""
    from . import lqscan as lq
    from . import workloads

    sizes = [(i.n, i.m, i.T) for i in insts]

    def make_prob(sel):
        return lq.to_device(workloads.pack([insts[j] for j in sel]))

    return tune_sizes(sizes, make_prob, precision=precision, candidates=candidates, reps=reps,
                      cache_path=cache_path, sample_per_class=sample_per_class, refine=refine)


def seg_lens_summary(insts, seg_lens):
    """Text summary: chosen L per (n, T-bucket); insts are LQInstance or (n, m, T)."""
    rows = {}
    for i, L in zip(insts, seg_lens):
        n, T = (i[0], i[2]) if isinstance(i, tuple) else (i.n, i.T)
        rows.setdefault((n, _bucket(T)), set()).add("seq" if L >= T else L)
    return {f"n={n},T<={tb}": sorted(map(str, v)) for (n, tb), v in sorted(rows.items())}


__all__ = ["tune", "tune_sizes", "class_key", "seg_lens_summary", "DEFAULT_CANDIDATES", "DEFAULT_REPS", "MARGIN"]
