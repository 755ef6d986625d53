"""Thin Python binding of the C ABI in include/lqscan.h.

Every function named ``lq_*`` here marshals its arguments and calls the C
entry point of the same name; all arithmetic happens in the HIP library.
PyTorch only provides device memory (tensors) and the stream.  There is no
CPU fallback: importing this module fails if liblqscan.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblqscan.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(hipcc for gfx950) first -- there is no fallback path")

_lib = ctypes.CDLL(LIB_PATH)

LQ_OK, LQ_ERR_ARG, LQ_ERR_NOT_PD, LQ_ERR_SINGULAR = 0, -1, -2, -3
LQ_ERR_NONFINITE, LQ_ERR_HIP, LQ_ERR_WORKSPACE, LQ_ERR_UNSUPPORTED = -4, -5, -6, -7
LQ_FP64, LQ_MIXED = 0, 1
LQ_SCAN, LQ_SEQUENTIAL = 0, 1

_P = ctypes.c_void_p
_PROBLEM_FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")


class LQProblemC(ctypes.Structure):
    _fields_ = [(f, _P) for f in _PROBLEM_FIELDS]


class LQValueC(ctypes.Structure):
    _fields_ = [(f, _P) for f in ("S", "s", "Gamma", "gamma")]


class LQGradsC(ctypes.Structure):
    _fields_ = [(f, _P) for f in _PROBLEM_FIELDS]


_i32p = ctypes.POINTER(ctypes.c_int32)
_plan_p = ctypes.c_void_p

_lib.lq_version.restype = ctypes.c_char_p
_lib.lq_plan_create.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.POINTER(_plan_p)]
_lib.lq_plan_create.restype = ctypes.c_int
_lib.lq_plan_create_seg.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int32, _i32p,
                                    ctypes.POINTER(_plan_p)]
_lib.lq_plan_create_seg.restype = ctypes.c_int
_lib.lq_plan_create_tuned.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int32, ctypes.c_char_p,
                                      ctypes.POINTER(_plan_p)]
_lib.lq_plan_create_tuned.restype = ctypes.c_int
_lib.lq_plan_destroy.argtypes = [_plan_p]
_lib.lq_plan_destroy.restype = None
for _f, _rt in (("lq_plan_workspace_bytes", ctypes.c_size_t), ("lq_plan_elements_bytes", ctypes.c_size_t),
                ("lq_plan_seg_len", ctypes.c_int32), ("lq_plan_total_stages", ctypes.c_int64)):
    getattr(_lib, _f).argtypes = [_plan_p]
    getattr(_lib, _f).restype = _rt
_lib.lq_build_elements.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, _P, _P]
_lib.lq_build_elements.restype = ctypes.c_int
_lib.lq_scan_solve.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, ctypes.POINTER(LQValueC), _P, _P, _P]
_lib.lq_scan_solve.restype = ctypes.c_int
_lib.lq_rollout.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), ctypes.POINTER(LQValueC), _P, _P, _P, _P, _P, _P]
_lib.lq_rollout.restype = ctypes.c_int
_lib.lq_rollout_cv.argtypes = _lib.lq_rollout.argtypes
_lib.lq_rollout_cv.restype = ctypes.c_int
_lib.lq_solve.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, ctypes.POINTER(LQValueC), _P, _P, _P, _P, _P, _P]
_lib.lq_solve.restype = ctypes.c_int
_lib.lq_solve_static.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, ctypes.POINTER(LQValueC), _P, _P, _P, _P,
                                 _P]
_lib.lq_solve_static.restype = ctypes.c_int
_lib.lq_plan_static_bytes.argtypes = [_plan_p]
_lib.lq_plan_static_bytes.restype = ctypes.c_size_t
_lib.lq_adjoint.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), ctypes.POINTER(LQValueC), _P, _P, _P, _P, _P,
                            ctypes.POINTER(LQGradsC), _P, _P, _P]
_lib.lq_adjoint.restype = ctypes.c_int
_lib.lq_plan_checkpoint_bytes.argtypes = [_plan_p, ctypes.c_int32]
_lib.lq_plan_checkpoint_bytes.restype = ctypes.c_size_t
_lib.lq_plan_adjoint_ckpt_workspace_bytes.argtypes = [_plan_p]
_lib.lq_plan_adjoint_ckpt_workspace_bytes.restype = ctypes.c_size_t
_lib.lq_solve_ckpt.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, ctypes.POINTER(LQValueC), _P, _P, _P, _P,
                               ctypes.c_int32, _P, _P, _P]
_lib.lq_solve_ckpt.restype = ctypes.c_int
_lib.lq_adjoint_ckpt.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), _P, ctypes.c_int32, _P, _P, _P, _P, _P,
                                 ctypes.POINTER(LQGradsC), _P, _P, _P]
_lib.lq_adjoint_ckpt.restype = ctypes.c_int
_lib.lq_plan_set_timing.argtypes = [_plan_p, ctypes.c_uint32, ctypes.c_int32]
_lib.lq_plan_set_timing.restype = ctypes.c_int
_lib.lq_plan_phase_times.argtypes = [_plan_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.lq_plan_phase_times.restype = ctypes.c_int
_lib.lq_selftest_tile_mm.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P]
_lib.lq_selftest_tile_mm.restype = ctypes.c_int
_lib.lq_selftest_tile_inverse.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P]
_lib.lq_selftest_tile_inverse.restype = ctypes.c_int

EXPORTED = ("lq_plan_create", "lq_plan_create_seg", "lq_plan_create_tuned", "lq_plan_destroy", "lq_plan_workspace_bytes", "lq_plan_elements_bytes",
            "lq_plan_seg_len", "lq_plan_total_stages", "lq_build_elements", "lq_scan_solve", "lq_rollout", "lq_rollout_cv",
            "lq_solve", "lq_solve_static", "lq_plan_static_bytes", "lq_adjoint",
            "lq_plan_checkpoint_bytes", "lq_plan_adjoint_ckpt_workspace_bytes", "lq_solve_ckpt", "lq_adjoint_ckpt", "lq_selftest_tile_mm", "lq_selftest_tile_inverse", "lq_version", "lq_plan_set_timing", "lq_plan_phase_times")

PHASES = ("build", "value_fold", "value_scan", "value_bellman", "roll_fold", "roll_scan", "roll_apply",
          "adj_back_fold", "adj_back_scan", "adj_back_apply", "adj_fwd_fold", "adj_fwd_scan", "adj_fwd_apply",
          "cv_fold", "cv_scan", "cv_start", "adj_recompute")


class LQError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} returned {code}")
        self.code = code


def _check(fn, code):
    if code != LQ_OK:
        raise LQError(fn, code)


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _f64(t):
    if t is not None and t.dtype != torch.float64:
        raise ValueError("problem and output arrays are float64")
    return _ptr(t)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def lq_version() -> str:
    return _lib.lq_version().decode()


# ---------------------------------------------------------------------------
# Plan
# ---------------------------------------------------------------------------

class Plan:
    """Owns an lq_plan* (sizes, segment decomposition, device descriptor tables)."""

    def __init__(self, nx, nu, T, *, precision: str = "fp64", mode: str = "scan", seg_len: int = 0,
                 seg_lens=None, autotune_cache: str | None = None):
        """seg_lens: one segment length per instance; autotune_cache: the
        autotuner's JSON cache, read by the library (lq_plan_create_tuned)."""
        nx, nu, T = (list(map(int, v)) if hasattr(v, "__len__") else [int(v)] for v in (nx, nu, T))
        self.batch = len(T)
        self.nx, self.nu, self.T = nx, nu, T
        self.precision, self.mode = precision, mode
        arr = ctypes.c_int32 * self.batch
        prec = {"fp64": LQ_FP64, "mixed": LQ_MIXED}[precision]
        h = _plan_p()
        if autotune_cache is not None:
            code = _lib.lq_plan_create_tuned(self.batch, arr(*nx), arr(*nu), arr(*T), prec,
                                             os.fsencode(autotune_cache), ctypes.byref(h))
            _check("lq_plan_create_tuned", code)
        elif seg_lens is not None:
            code = _lib.lq_plan_create_seg(self.batch, arr(*nx), arr(*nu), arr(*T), prec,
                                           arr(*[int(v) for v in seg_lens]), ctypes.byref(h))
            _check("lq_plan_create_seg", code)
        else:
            code = _lib.lq_plan_create(self.batch, arr(*nx), arr(*nu), arr(*T), prec,
                                       {"scan": LQ_SCAN, "sequential": LQ_SEQUENTIAL}[mode], int(seg_len),
                                       ctypes.byref(h))
            _check("lq_plan_create", code)
        self._h = h

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self) -> int:
        return int(_lib.lq_plan_workspace_bytes(self._h))

    def elements_bytes(self) -> int:
        return int(_lib.lq_plan_elements_bytes(self._h))

    def seg_len(self) -> int:
        return int(_lib.lq_plan_seg_len(self._h))

    def total_stages(self) -> int:
        return int(_lib.lq_plan_total_stages(self._h))

    def new_workspace(self, device="cuda"):
        return torch.empty(max(self.workspace_bytes(), 256), dtype=torch.uint8, device=device)

    def checkpoint_bytes(self, stride: int) -> int:
        return int(_lib.lq_plan_checkpoint_bytes(self._h, int(stride)))

    def adjoint_ckpt_workspace_bytes(self) -> int:
        return int(_lib.lq_plan_adjoint_ckpt_workspace_bytes(self._h))

    def new_checkpoint(self, stride: int, device="cuda"):
        return torch.empty(max(self.checkpoint_bytes(stride) // 8, 32), dtype=torch.float64, device=device)

    def new_adjoint_ckpt_workspace(self, device="cuda"):
        return torch.empty(max(self.adjoint_ckpt_workspace_bytes(), 256), dtype=torch.uint8, device=device)

    def new_elements(self, device="cuda"):
        return torch.empty(max(self.elements_bytes() // 8, 32), dtype=torch.float64, device=device)

    def set_timing(self, phases, capacity=4096):
        """Enable event timing around the named phases (see PHASES)."""
        mask = 0
        for ph in phases:
            mask |= 1 << PHASES.index(ph)
        _check("lq_plan_set_timing", _lib.lq_plan_set_timing(self._h, mask, int(capacity)))

    def phase_times(self) -> dict:
        """{phase: (total_ms, launches)} since the last call; waits for the events."""
        ms = (ctypes.c_double * len(PHASES))()
        cnt = (ctypes.c_int64 * len(PHASES))()
        _check("lq_plan_phase_times", _lib.lq_plan_phase_times(self._h, ms, cnt))
        return {ph: (ms[i], cnt[i]) for i, ph in enumerate(PHASES) if cnt[i] > 0}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lq_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_struct(prob: dict) -> LQProblemC:
    return LQProblemC(*[_f64(prob.get(f)) for f in _PROBLEM_FIELDS])


def _value_struct(val: dict) -> LQValueC:
    return LQValueC(*[_f64(val.get(f)) for f in ("S", "s", "Gamma", "gamma")])


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def lq_build_elements(plan: Plan, prob: dict, elements, status=None, stream=None):
    _check("lq_build_elements", _lib.lq_build_elements(plan.handle, ctypes.byref(_problem_struct(prob)),
                                                       _f64(elements), _ptr(status), _stream(stream)))


def lq_scan_solve(plan: Plan, prob: dict, elements, value: dict, workspace, status=None, stream=None):
    _check("lq_scan_solve", _lib.lq_scan_solve(plan.handle, ctypes.byref(_problem_struct(prob)), _f64(elements),
                                               ctypes.byref(_value_struct(value)), _ptr(workspace), _ptr(status),
                                               _stream(stream)))


def lq_rollout(plan: Plan, prob: dict, value: dict, x, u, lam, workspace, status=None, stream=None):
    _check("lq_rollout", _lib.lq_rollout(plan.handle, ctypes.byref(_problem_struct(prob)),
                                         ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                         _ptr(workspace), _ptr(status), _stream(stream)))


def lq_rollout_cv(plan: Plan, prob: dict, value: dict, x, u, lam, workspace, status=None, stream=None):
    _check("lq_rollout_cv", _lib.lq_rollout_cv(plan.handle, ctypes.byref(_problem_struct(prob)),
                                               ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                               _ptr(workspace), _ptr(status), _stream(stream)))


def lq_solve(plan: Plan, prob: dict, elements, value: dict, x, u, lam, workspace, status=None, stream=None):
    _check("lq_solve", _lib.lq_solve(plan.handle, ctypes.byref(_problem_struct(prob)), _f64(elements),
                                     ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                     _ptr(workspace), _ptr(status), _stream(stream)))


def lq_solve_static(plan: Plan, prob: dict, elements, value: dict, x, u, lam, status=None, stream=None):
    _check("lq_solve_static", _lib.lq_solve_static(plan.handle, ctypes.byref(_problem_struct(prob)), _f64(elements),
                                                   ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                                   _ptr(status), _stream(stream)))


def lq_plan_static_bytes(plan: Plan) -> int:
    return int(_lib.lq_plan_static_bytes(plan.handle))


LQ_STATIC_SCRATCH_BYTES = 32 << 20


def lq_adjoint(plan: Plan, prob: dict, value: dict | None, x, u, lam, gx, gu, grads: dict, workspace, status=None,
               stream=None):
    """value None: the value functions are recomputed (the workspace must be
    plan.new_adjoint_ckpt_workspace())."""
    g = LQGradsC(*[_f64(grads.get(f)) for f in _PROBLEM_FIELDS])
    vs = None if value is None else ctypes.byref(_value_struct(value))
    _check("lq_adjoint", _lib.lq_adjoint(plan.handle, ctypes.byref(_problem_struct(prob)), vs, _f64(x), _f64(u),
                                         _f64(lam), _f64(gx), _f64(gu), ctypes.byref(g), _ptr(workspace),
                                         _ptr(status), _stream(stream)))


def lq_solve_ckpt(plan: Plan, prob: dict, elements, value: dict, x, u, lam, ckpt, stride: int, workspace,
                  status=None, stream=None):
    _check("lq_solve_ckpt", _lib.lq_solve_ckpt(plan.handle, ctypes.byref(_problem_struct(prob)), _f64(elements),
                                               ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                               _f64(ckpt), int(stride), _ptr(workspace), _ptr(status),
                                               _stream(stream)))


def lq_adjoint_ckpt(plan: Plan, prob: dict, ckpt, stride: int, x, u, lam, gx, gu, grads: dict, workspace,
                    status=None, stream=None):
    g = LQGradsC(*[_f64(grads.get(f)) for f in _PROBLEM_FIELDS])
    _check("lq_adjoint_ckpt", _lib.lq_adjoint_ckpt(plan.handle, ctypes.byref(_problem_struct(prob)), _f64(ckpt),
                                                   int(stride), _f64(x), _f64(u), _f64(lam), _f64(gx), _f64(gu),
                                                   ctypes.byref(g), _ptr(workspace), _ptr(status),
                                                   _stream(stream)))


def lq_selftest_tile_inverse(X, Xinv, n1, homog, ok, stream=None):
    _check("lq_selftest_tile_inverse", _lib.lq_selftest_tile_inverse(_f64(X), _f64(Xinv), int(n1), int(homog),
                                                                     _ptr(ok), _stream(stream)))


def lq_selftest_tile_mm(X, Y, Z, D, tx=False, ty=False, precision="fp64", stream=None):
    _check("lq_selftest_tile_mm", _lib.lq_selftest_tile_mm(_f64(X), _f64(Y), _f64(Z), _f64(D), int(tx), int(ty),
                                                           {"fp64": LQ_FP64, "mixed": LQ_MIXED}[precision],
                                                           _stream(stream)))


# ---------------------------------------------------------------------------
# Convenience: packed tensors and a whole solve
# ---------------------------------------------------------------------------

def to_device(packed: dict, device="cuda") -> dict:
    """numpy packed arrays (workloads.pack) -> float64 device tensors."""
    out = {}
    for f in _PROBLEM_FIELDS:
        v = packed.get(f)
        out[f] = None if v is None else torch.as_tensor(v, dtype=torch.float64).to(device).contiguous()
    return out


def value_buffers(plan: Plan, device="cuda") -> dict:
    n = torch.tensor(plan.nx, dtype=torch.int64)
    m = torch.tensor(plan.nu, dtype=torch.int64)
    T = torch.tensor(plan.T, dtype=torch.int64)
    z = lambda k: torch.empty(int(k), dtype=torch.float64, device=device)
    return {"S": z(((T + 1) * n * n).sum()), "s": z(((T + 1) * n).sum()),
            "Gamma": z((T * m * n).sum()), "gamma": z((T * m).sum())}


def state_buffers(plan: Plan, device="cuda") -> dict:
    n = torch.tensor(plan.nx, dtype=torch.int64)
    m = torch.tensor(plan.nu, dtype=torch.int64)
    T = torch.tensor(plan.T, dtype=torch.int64)
    z = lambda k: torch.empty(int(k), dtype=torch.float64, device=device)
    return {"x": z(((T + 1) * n).sum()), "u": z((T * m).sum()), "lam": z(((T + 1) * n).sum())}


def solve(plan_or_A, *args, **kw):
    """Two forms.

    solve(plan, prob, ...): the packed batch on a plan (see _solve_plan),
    returns the flat packed outputs and the status array.

    solve(A, B, c, Q, R, QT, x0, *, M=None, q=None, r=None, qT=None,
    precision="fp64", seg_len=0, checkpoint=1): one problem given as
    stage-major float64 device tensors (A [T, n, n], B [T, n, m], c [T, n],
    Q [T, n, n], R [T, m, m], QT [n, n], x0 [n], M [T, n, m], q [T, n],
    r [T, m], qT [n]; c may be None); returns (x [T + 1, n], u [T, m]),
    differentiable with respect to every tensor argument (the adjoint, with
    the level checkpoint of `checkpoint`).  It waits for the solve to check
    the status and raises LQError on a numerical failure."""
    if isinstance(plan_or_A, Plan):
        return _solve_plan(plan_or_A, *args, **kw)
    return _solve_tensors(plan_or_A, *args, **kw)


_PLAN_CACHE: dict = {}


def _cached_plan(sizes, precision: str, seg_len: int) -> Plan:
    """Plans of the tensor-form solves, kept for the last 32 size lists."""
    key = (tuple(sizes), precision, int(seg_len))
    p = _PLAN_CACHE.get(key)
    if p is None:
        if len(_PLAN_CACHE) >= 32:
            _PLAN_CACHE.pop(next(iter(_PLAN_CACHE)))
        p = Plan([z[0] for z in sizes], [z[1] for z in sizes], [z[2] for z in sizes], precision=precision,
                 seg_len=seg_len)
        _PLAN_CACHE[key] = p
    return p


_OPTIONAL = ("c", "M", "q", "r", "qT")


def _sizes_of(A, B):
    if A.dim() != 3 or B.dim() != 3 or A.shape[1] != A.shape[2] or B.shape[:2] != A.shape[:2]:
        raise ValueError("A must be [T, n, n] and B [T, n, m]")
    return int(A.shape[1]), int(B.shape[2]), int(A.shape[0])


def _stage_shapes(n, m, T):
    return {"A": (T, n, n), "B": (T, n, m), "c": (T, n), "Q": (T, n, n), "R": (T, m, m), "QT": (n, n), "x0": (n,),
            "M": (T, n, m), "q": (T, n), "r": (T, m), "qT": (n,)}


def _packed(problems, sizes):
    """Flat packed fields of a list of problem dicts (autograd-preserving); an
    optional field absent from every problem stays None, absent from some is
    zero there."""
    out = {}
    for f in LQSolveFunction.NAMES:
        have = [p.get(f) is not None for p in problems]
        if f in _OPTIONAL and not any(have):
            out[f] = None
            continue
        parts = []
        for p, (n, m, T) in zip(problems, sizes):
            shp = _stage_shapes(n, m, T)[f]
            t = p.get(f)
            if t is None:
                if f not in _OPTIONAL:
                    raise ValueError(f"missing {f}")
                t = torch.zeros(shp, dtype=torch.float64, device=problems[0]["A"].device)
            if tuple(t.shape) != shp:
                raise ValueError(f"{f} has shape {tuple(t.shape)}, expected {shp}")
            parts.append(t.to(torch.float64).contiguous().reshape(-1))
        out[f] = torch.cat(parts) if len(parts) > 1 else parts[0]
    return out


def _check_status(status):
    bad = torch.nonzero(status).flatten().tolist()
    if bad:
        w = int(status[bad[0]])
        raise LQError(f"lq_solve (instance {bad[0]}, stage {w >> 8})", -(w & 0xFF))


def _solve_tensors(A, B, c, Q, R, QT, x0, *, M=None, q=None, r=None, qT=None, precision="fp64", seg_len=0,
                   checkpoint=1):
    n, m, T = _sizes_of(A, B)
    prob = {"A": A, "B": B, "c": c, "Q": Q, "R": R, "QT": QT, "x0": x0, "M": M, "q": q, "r": r, "qT": qT}
    pk = _packed([prob], [(n, m, T)])
    plan = _cached_plan([(n, m, T)], precision, seg_len)
    x, u, status = solve_diff(plan, *[pk[f] for f in LQSolveFunction.NAMES], checkpoint=checkpoint)
    _check_status(status)
    return x.view(T + 1, n), u.view(T, m)


def solve_batch(problems, *, precision="fp64", seg_len=0, checkpoint=1):
    """A ragged batch given as a list of problem dicts (the tensors of the
    tensor form of solve; sizes may differ, optional fields may be absent):
    one batched, differentiable solve; returns a list of (x [T+1, n],
    u [T, m]).  Waits to check the status, as solve does."""
    sizes = [_sizes_of(p["A"], p["B"]) for p in problems]
    pk = _packed(problems, sizes)
    plan = _cached_plan(sizes, precision, seg_len)
    x, u, status = solve_diff(plan, *[pk[f] for f in LQSolveFunction.NAMES], checkpoint=checkpoint)
    _check_status(status)
    out, ox, ou = [], 0, 0
    for n, m, T in sizes:
        out.append((x[ox:ox + (T + 1) * n].view(T + 1, n), u[ou:ou + T * m].view(T, m)))
        ox += (T + 1) * n
        ou += T * m
    return out


def _solve_plan(plan: Plan, prob: dict, *, materialise_elements: bool = False, fused: bool = True, workspace=None,
                stream=None, rollout: str = "affine") -> dict:
    """lq_solve (fused = False: lq_scan_solve then lq_rollout; rollout = "cv":
    lq_scan_solve then lq_rollout_cv); returns flat packed device tensors and
    the status array."""
    if rollout not in ("affine", "cv"):
        raise ValueError(f"rollout must be 'affine' or 'cv', not {rollout!r}")
    dev = prob["A"].device
    ws = workspace if workspace is not None else plan.new_workspace(dev)
    status = torch.zeros(plan.batch, dtype=torch.int32, device=dev)
    val = value_buffers(plan, dev)
    st = state_buffers(plan, dev)
    el = None
    if materialise_elements:
        el = plan.new_elements(dev)
        lq_build_elements(plan, prob, el, status, stream)
    if rollout == "cv":
        lq_scan_solve(plan, prob, el, val, ws, status, stream)
        lq_rollout_cv(plan, prob, val, st["x"], st["u"], st["lam"], ws, status, stream)
    elif fused:
        lq_solve(plan, prob, el, val, st["x"], st["u"], st["lam"], ws, status, stream)
    else:
        lq_scan_solve(plan, prob, el, val, ws, status, stream)
        lq_rollout(plan, prob, val, st["x"], st["u"], st["lam"], ws, status, stream)
    out = dict(val)
    out.update(st)
    out["status"] = status
    out["elements"] = el
    return out


def grad_buffers(plan: Plan, which, device="cuda") -> dict:
    """Gradient output buffers (same packing as the problem) for the named fields."""
    n = torch.tensor(plan.nx, dtype=torch.int64)
    m = torch.tensor(plan.nu, dtype=torch.int64)
    T = torch.tensor(plan.T, dtype=torch.int64)
    size = {"A": (T * n * n).sum(), "B": (T * n * m).sum(), "c": (T * n).sum(), "Q": (T * n * n).sum(),
            "R": (T * m * m).sum(), "M": (T * n * m).sum(), "q": (T * n).sum(), "r": (T * m).sum(),
            "QT": (n * n).sum(), "qT": n.sum(), "x0": n.sum()}
    return {f: torch.empty(int(size[f]), dtype=torch.float64, device=device) for f in which}


class LQSolveFunction(torch.autograd.Function):
    """(x, u) = LQ solution of the packed problem; gradients by the adjoint.

    Inputs are flat packed float64 device tensors (lq_problem layout); c, M, q,
    r, qT may be None.  `checkpoint` picks what the forward keeps for the
    backward pass:
      k >= 1       level checkpointing: lq_solve_ckpt keeps one value-function
                   carry per k segments (lq_plan_checkpoint_bytes) and the
                   backward's lq_adjoint_ckpt recomputes S, Gamma from it;
      "recompute"  nothing but x, u and the co-states: lq_adjoint_ckpt reruns
                   the whole value pass;
      0            S, s, Gamma, gamma themselves (lq_solve, then lq_adjoint).
    The problem tensors and the outputs x, u are saved with save_for_backward
    (so an in-place change of an input between forward and backward is
    detected and no output is referenced from its own grad_fn); the co-states,
    checkpoint or value arrays are intermediates kept on ctx.
    """

    NAMES = ("A", "B", "c", "Q", "R", "QT", "x0", "M", "q", "r", "qT")

    @staticmethod
    def forward(ctx, plan, checkpoint, A, B, c, Q, R, QT, x0, M, q, r, qT):
        prob = {"A": A, "B": B, "c": c, "Q": Q, "R": R, "QT": QT, "x0": x0, "M": M, "q": q, "r": r, "qT": qT}
        dev = A.device
        ws = plan.new_workspace(dev)
        status = torch.zeros(plan.batch, dtype=torch.int32, device=dev)
        val = value_buffers(plan, dev)
        st = state_buffers(plan, dev)
        ctx.plan, ctx.lam, ctx.checkpoint = plan, st["lam"], checkpoint
        ctx.val = ctx.ckpt = None
        if checkpoint == 0:
            lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
            ctx.val = val
        elif checkpoint == "recompute":
            lq_solve(plan, prob, None, val, st["x"], st["u"], st["lam"], ws, status)
        else:
            if not (isinstance(checkpoint, int) and checkpoint >= 1):
                raise ValueError(f"checkpoint must be 0, a stride >= 1 or 'recompute', not {checkpoint!r}")
            ctx.ckpt = plan.new_checkpoint(checkpoint, dev)
            lq_solve_ckpt(plan, prob, None, val, st["x"], st["u"], st["lam"], ctx.ckpt, checkpoint, ws, status)
        ctx.save_for_backward(A, B, c, Q, R, QT, x0, M, q, r, qT, st["x"], st["u"])
        ctx.mark_non_differentiable(status)
        return st["x"], st["u"], status

    @staticmethod
    def backward(ctx, gx, gu, _gstatus):
        saved = ctx.saved_tensors
        names = LQSolveFunction.NAMES
        prob = dict(zip(names, saved[:len(names)]))
        x, u = saved[len(names):]
        plan = ctx.plan
        want = [f for i, f in enumerate(names) if ctx.needs_input_grad[i + 2]]
        dev = x.device
        gx = torch.zeros_like(x) if gx is None else gx.contiguous()
        gu = torch.zeros_like(u) if gu is None else gu.contiguous()
        g = grad_buffers(plan, want, dev)
        status = torch.zeros(plan.batch, dtype=torch.int32, device=dev)
        if ctx.val is not None:
            lq_adjoint(plan, prob, ctx.val, x, u, ctx.lam, gx, gu, g, plan.new_workspace(dev), status)
        else:
            stride = 1 if ctx.ckpt is None else ctx.checkpoint
            lq_adjoint_ckpt(plan, prob, ctx.ckpt, stride, x, u, ctx.lam, gx, gu, g,
                            plan.new_adjoint_ckpt_workspace(dev), status)
        return (None, None) + tuple(g.get(f) for f in names)


def solve_diff(plan: Plan, A, B, c, Q, R, QT, x0, M=None, q=None, r=None, qT=None, *, checkpoint=1):
    """Differentiable LQ solve on packed device tensors; returns (x, u, status).

    checkpoint: stride of the level checkpoint kept for the backward pass
    (default 1: one carry per segment), "recompute" (keep nothing), or 0 (keep
    the value functions and gains)."""
    return LQSolveFunction.apply(plan, checkpoint, A, B, c, Q, R, QT, x0, M, q, r, qT)


# ---------------------------------------------------------------------------
# Newton / interior point (newton_step)
# ---------------------------------------------------------------------------

(NMPC_MU, NMPC_ALPHA, NMPC_NU, NMPC_COST, NMPC_PRED, NMPC_RHO, NMPC_ACCEPTED, NMPC_COST_NEW, NMPC_GRAD,
 NMPC_RP, NMPC_RD, NMPC_LEVEL_TOL, NMPC_LEVEL_MAX, NMPC_LEVEL_ITERS, NMPC_LEVEL_DONE, NMPC_NSCAL) = range(16)
NMPC_TANH, NMPC_PENDULUM, NMPC_CARTPOLE = 0, 1, 2


class NMPCProblemC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nu", ctypes.c_int32), ("T", ctypes.c_int32), ("h", ctypes.c_double),
                ("W", _P), ("Bm", _P), ("Q", _P), ("R", _P), ("QT", _P), ("xref", _P), ("x0", _P),
                ("umin", ctypes.c_double), ("umax", ctypes.c_double), ("model", ctypes.c_int32),
                ("param", ctypes.c_double * 4), ("admm_rho", ctypes.c_double), ("admm_z", _P), ("admm_v", _P)]


class NMPCStateC(ctypes.Structure):
    _fields_ = [("x", _P), ("u", _P), ("scal", _P)]


_lib.nmpc_workspace_bytes.argtypes = [_plan_p]
_lib.nmpc_workspace_bytes.restype = ctypes.c_size_t
_lib.nmpc_init.argtypes = [_plan_p, ctypes.POINTER(NMPCProblemC), ctypes.POINTER(NMPCStateC), _P, _P]
_lib.nmpc_init.restype = ctypes.c_int
_lib.newton_step.argtypes = [_plan_p, ctypes.POINTER(NMPCProblemC), ctypes.POINTER(NMPCStateC), _P, _P, _P]
_lib.newton_step.restype = ctypes.c_int
_lib.nmpc_admm_update.argtypes = [_plan_p, ctypes.POINTER(NMPCProblemC), ctypes.POINTER(NMPCStateC), ctypes.c_int32,
                                  _P]
_lib.nmpc_admm_update.restype = ctypes.c_int
_lib.nmpc_shift.argtypes = [_plan_p, ctypes.POINTER(NMPCProblemC), ctypes.POINTER(NMPCStateC), _P, _P, _P]
_lib.nmpc_shift.restype = ctypes.c_int
EXPORTED = EXPORTED + ("nmpc_workspace_bytes", "nmpc_init", "newton_step", "nmpc_admm_update", "nmpc_shift")


def nmpc_workspace_bytes(plan: Plan) -> int:
    return int(_lib.nmpc_workspace_bytes(plan.handle))


def nmpc_init(plan, prob_c, state_c, workspace, stream=None):
    _check("nmpc_init", _lib.nmpc_init(plan.handle, ctypes.byref(prob_c), ctypes.byref(state_c), _ptr(workspace),
                                       _stream(stream)))


def newton_step(plan, prob_c, state_c, workspace, status=None, stream=None):
    _check("newton_step", _lib.newton_step(plan.handle, ctypes.byref(prob_c), ctypes.byref(state_c),
                                           _ptr(workspace), _ptr(status), _stream(stream)))


def nmpc_shift(plan, prob_c, state_c, x0, u_applied, stream=None):
    _check("nmpc_shift", _lib.nmpc_shift(plan.handle, ctypes.byref(prob_c), ctypes.byref(state_c), _ptr(x0),
                                         _ptr(u_applied), _stream(stream)))


def nmpc_admm_update(plan, prob_c, state_c, init, stream=None):
    _check("nmpc_admm_update", _lib.nmpc_admm_update(plan.handle, ctypes.byref(prob_c), ctypes.byref(state_c),
                                                     int(init), _stream(stream)))


class NewtonMPC:
    """Interior-point / ADMM Newton solver for x' = x + h f(x, u) with |u| bounded.

    `p` has numpy fields nx, nu, T, h, W, Bm, Q, R, QT, xref, x0, u0, umin,
    umax and optionally model (NMPC_TANH, NMPC_PENDULUM, NMPC_CARTPOLE) and
    param (the model constants); W and Bm are read by the tanh model only.
    A batch of problems that differ only in x0 ([B, nx]) and u0 ([B, T, nu])
    is solved at once (every decision per instance).  All iterations run on
    the GPU through newton_step; the host sets the barrier weight.  In
    ip_solve / admm_solve a barrier level ends on the device (the NMPC_LEVEL_*
    scalars of newton_step): a captured graph of `level_chunk` steps is
    replayed and the scalars are read back once per replay (eager, graph=False:
    one step and one read-back per iteration, the level ended by the host).
    """

    def __init__(self, p, device="cuda", seg_len=0, precision="fp64", mode="scan", level_chunk=4):
        t = lambda a: torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        self.p = p
        model = int(getattr(p, "model", NMPC_TANH) or 0)
        self.B = 1 if np.ndim(p.x0) == 1 else int(np.shape(p.x0)[0])
        B = self.B
        if seg_len == 0 and mode == "scan" and B > 1:
            # a batch fills the GPU by itself.  Tile kernels (n > 4, one wave per
            # segment): about 1536 segments in all, so that large batches run the
            # plain recursion per instance (N = 60: B = 256 best at 6 segments,
            # B >= 1024 at one).  Per-lane kernels (n <= 4, one lane per segment):
            # about 16384 segments, at least 4 stages each (N = 60, receding-horizon
            # simulations: B = 64 and 1024 best at 4 stages per segment, 4096 at 15)
            if p.nx <= 4:
                nseg = max(1, min(-(-16384 // B), p.T // 4))
            else:
                nseg = max(1, -(-1536 // B))
            seg_len = max(1, -(-p.T // nseg))
        self.plan = Plan([p.nx] * B, [p.nu] * B, [p.T] * B, seg_len=seg_len, precision=precision, mode=mode)
        names = ("Q", "R", "QT", "xref") + (("W", "Bm") if model == NMPC_TANH else ())
        self.dev = {k: t(getattr(p, k)) for k in names}
        self.x0 = t(p.x0).reshape(-1).clone()
        self.dev["x0"] = self.x0
        self.x = torch.zeros(B * (p.T + 1) * p.nx, dtype=torch.float64, device=device)
        u0 = np.asarray(p.u0, np.float64)
        if B > 1 and u0.ndim == 2:
            u0 = np.broadcast_to(u0, (B,) + u0.shape)
        self.u0 = t(np.ascontiguousarray(u0)).reshape(-1).clone()
        self.u = self.u0.clone()
        self.scal = torch.zeros(B * NMPC_NSCAL, dtype=torch.float64, device=device)
        self._sc = self.scal.view(B, NMPC_NSCAL)
        self.level_chunk = max(1, int(level_chunk))
        # per-step copies of the scalars inside a replayed chunk, and their host mirror
        self._hist = torch.zeros(self.level_chunk, B * NMPC_NSCAL, dtype=torch.float64, device=device)
        self._hist_host = torch.empty(self.level_chunk, B * NMPC_NSCAL, dtype=torch.float64, pin_memory=True)
        self.ws = torch.empty(nmpc_workspace_bytes(self.plan), dtype=torch.uint8, device=device)
        d = self.dev
        prm = getattr(p, "param", None)
        prm = (ctypes.c_double * 4)(*([float(v) for v in prm] if prm is not None else [0.0] * 4))
        self.prob_c = NMPCProblemC(p.nx, p.nu, p.T, float(p.h), _f64(d.get("W")), _f64(d.get("Bm")), _f64(d["Q"]),
                                   _f64(d["R"]), _f64(d["QT"]), _f64(d["xref"]), _f64(self.x0),
                                   float(p.umin), float(p.umax), model, prm)
        self.state_c = NMPCStateC(_f64(self.x), _f64(self.u), _f64(self.scal))
        # ip_solve's chunk graph and the single-step graphs of admm_solve and
        # mpc_simulate, kept across calls while the problem struct (sizes, parameters,
        # pointers) is byte for byte the one they were captured with
        self._chunk_graph, self._chunk_key = None, None
        self._step_graphs = {}
        self._admm_zv = None

    def _shape(self, a, rows, cols):
        a = a.cpu().numpy()
        return a.reshape(rows, cols) if self.B == 1 else a.reshape(self.B, rows, cols)

    def init(self, alpha0, nu0, reset_u=True):
        """Nominal controls back to u0 (unless reset_u is False), x to their rollout,
        damping to (alpha0, nu0)."""
        if reset_u:
            self.u.copy_(self.u0)
        self.scal.zero_()
        self._sc[:, NMPC_ALPHA] = alpha0
        self._sc[:, NMPC_NU] = nu0
        nmpc_init(self.plan, self.prob_c, self.state_c, self.ws)

    def step(self, mu):
        self._sc[:, NMPC_MU] = mu
        newton_step(self.plan, self.prob_c, self.state_c, self.ws)

    def run(self, mu_levels, iters, alpha0, nu0):
        """Fixed iterations per barrier level; traces of instance 0."""
        self.init(alpha0, nu0)
        n_it = len(mu_levels) * iters
        before = torch.zeros(n_it, NMPC_NSCAL, dtype=torch.float64, device=self.x.device)
        after = torch.zeros_like(before)
        it = 0
        for mu in mu_levels:
            for _ in range(iters):
                self._sc[:, NMPC_MU] = mu
                before[it].copy_(self._sc[0])
                newton_step(self.plan, self.prob_c, self.state_c, self.ws)
                after[it].copy_(self._sc[0])
                it += 1
        torch.cuda.synchronize()
        a = after.cpu().numpy()
        return {"u": self._shape(self.u, self.p.T, self.p.nu), "x": self._shape(self.x, self.p.T + 1, self.p.nx),
                "cost": a[:, NMPC_COST], "accept": a[:, NMPC_ACCEPTED] > 0.5,
                "alpha": before.cpu().numpy()[:, NMPC_ALPHA], "pred": a[:, NMPC_PRED], "rho": a[:, NMPC_RHO]}

    def _capture_step(self):
        """newton_step captured once into a HIP graph (its kernel sequence, replayed per
        iteration; the barrier weight and every decision live in device memory).  One eager
        step first (the state is reset afterwards by init)."""
        newton_step(self.plan, self.prob_c, self.state_c, self.ws)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            newton_step(self.plan, self.prob_c, self.state_c, self.ws)
        torch.cuda.current_stream().wait_stream(side)
        return g

    def _kept_step_graph(self):
        """The captured single step for the current problem struct (captured on first
        use; a few structs kept)."""
        key = (bytes(self.prob_c), 1)
        g = self._step_graphs.get(key)
        if g is None:
            if len(self._step_graphs) >= 8:
                self._step_graphs.clear()
            g = self._step_graphs[key] = self._capture_step()
        return g

    def _kept_chunk_graph(self, k):
        """_capture_chunk(k) for the current problem struct, kept like _kept_step_graph."""
        key = (bytes(self.prob_c), int(k))
        g = self._step_graphs.get(key)
        if g is None:
            if len(self._step_graphs) >= 8:
                self._step_graphs.clear()
            g = self._step_graphs[key] = self._capture_chunk(k)
        return g

    def _capture_chunk(self, k):
        """k <= level_chunk newton_step calls captured into one HIP graph, each followed
        by a copy of the device scalars into its slot of self._hist; returns (graph, k).
        One eager step first (the state is reset afterwards by init)."""
        k = max(1, min(int(k), self.level_chunk))
        newton_step(self.plan, self.prob_c, self.state_c, self.ws)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(g, stream=side):
            for j in range(k):
                newton_step(self.plan, self.prob_c, self.state_c, self.ws)
                self._hist[j].copy_(self.scal)
        torch.cuda.current_stream().wait_stream(side)
        return g, k

    def _newton_level(self, mu, tol, max_iter, host, rows, graph=None):
        """Newton iterations until the one that starts from |dJ/du|_inf <= tol (or
        max_iter).  With a chunk graph (_capture_chunk) the level ends on the
        device and the host reads the scalars back once per replay of
        level_chunk steps; eagerly, once per step."""
        if isinstance(graph, tuple):
            return self._newton_level_device(mu, tol, max_iter, rows, graph)
        li = 0
        hv = host.view(self.B, NMPC_NSCAL)
        # the host ends this level: no level control left on the device from an
        # earlier level ended there (admm_solve mixes both)
        self._sc[:, [NMPC_LEVEL_TOL, NMPC_LEVEL_DONE]] = 0.0
        while li < max_iter:
            self._sc[:, NMPC_MU] = mu
            if graph is not None:
                graph.replay()
            else:
                newton_step(self.plan, self.prob_c, self.state_c, self.ws)
            host.copy_(self.scal, non_blocking=True)
            torch.cuda.current_stream().synchronize()
            li += 1
            if rows is not None:
                rows.append((mu, float(hv[0, NMPC_COST]), float(hv[0, NMPC_GRAD]), float(hv[0, NMPC_ACCEPTED]),
                             float(hv[0, NMPC_PRED])))
            if float(hv[:, NMPC_GRAD].max()) <= tol:
                break
        return li

    def _newton_level_device(self, mu, tol, max_iter, rows, graph):
        graph, k = graph
        cols = [NMPC_MU, NMPC_LEVEL_TOL, NMPC_LEVEL_MAX, NMPC_LEVEL_ITERS, NMPC_LEVEL_DONE]
        self._sc[:, cols] = torch.tensor([mu, tol, float(max_iter), 0.0, 0.0], dtype=torch.float64,
                                         device=self.scal.device)
        hist = self._hist_host[:k].view(k, self.B, NMPC_NSCAL)
        seen = 0
        while True:
            graph.replay()
            self._hist_host[:k].copy_(self._hist[:k], non_blocking=True)
            torch.cuda.current_stream().synchronize()
            for j in range(k):
                it = int(hist[j, 0, NMPC_LEVEL_ITERS])
                if it > seen:
                    seen = it
                    if rows is not None:
                        r = hist[j, 0]
                        rows.append((mu, float(r[NMPC_COST]), float(r[NMPC_GRAD]), float(r[NMPC_ACCEPTED]),
                                     float(r[NMPC_PRED])))
            if bool((hist[-1, :, NMPC_LEVEL_DONE] >= 0.5).all()):
                break
        return int(hist[-1, :, NMPC_LEVEL_ITERS].max())

    def admm_solve(self, *, rho, eps, tol, max_iter, max_admm, alpha0, nu0, graph=True, chunk="auto"):
        """ADMM of Sec. II-C for the control box with newton_step as the inner solver:
        z = min(0, h(u0)), v = 0; repeat Newton iterations on J_AD to |dJ_AD/du|_inf <= tol
        (or max_iter), then nmpc_admm_update, until |r_p|_inf, |r_d|_inf <= eps or max_admm.
        rho is the weight of each stage's augmentation term.  graph: replay newton_step from a
        captured HIP graph, kept for later solves of the same problem; chunk > 1 (at most
        level_chunk): graphs of that many steps with the inner levels ended on the device,
        as in ip_solve, instead of one step per read-back; "auto": chunks of three while
        the inner levels average at least five iterations, else one step per read-back
        (steps past a short level's end cost more than the read-backs they save).  The
        results do not depend on the chunk.  Returns dict(u, x, z, v, admm_iters,
        newton_iters, inner, rp, rd)."""
        dev = self.x.device
        if self._admm_zv is None:   # kept, so that the captured step's pointers stay valid
            self._admm_zv = torch.zeros(2, self.B * self.p.T * 2 * self.p.nu, dtype=torch.float64, device=dev)
        z, v = self._admm_zv[0], self._admm_zv[1]
        z.zero_()
        v.zero_()
        self.prob_c.admm_rho = float(rho)
        self.prob_c.admm_z = _f64(z)
        self.prob_c.admm_v = _f64(v)
        try:
            # chunk sizes in use (auto: 3 for long inner levels, 1 for short ones)
            sizes = (min(3, self.level_chunk), 1) if chunk == "auto" else (max(1, min(int(chunk), self.level_chunk)),)
            graphs = {}
            if graph:   # captured before init (a capture runs one eager step)
                for k in sizes:
                    graphs[k] = self._kept_step_graph() if k == 1 else self._kept_chunk_graph(k)
            self.init(alpha0, nu0)
            nmpc_admm_update(self.plan, self.prob_c, self.state_c, 1)
            host = torch.empty(self.B * NMPC_NSCAL, dtype=torch.float64, pin_memory=True)
            hv = host.view(self.B, NMPC_NSCAL)
            inner, rps, rds = [], [], []
            for _ in range(max_admm):
                k = sizes[0] if not inner or sum(inner) >= 5 * len(inner) else sizes[-1]
                inner.append(self._newton_level(0.0, tol, max_iter, host, None, graphs.get(k)))
                nmpc_admm_update(self.plan, self.prob_c, self.state_c, 0)
                host.copy_(self.scal, non_blocking=True)
                torch.cuda.current_stream().synchronize()
                rps.append(float(hv[:, NMPC_RP].max()))
                rds.append(float(hv[:, NMPC_RD].max()))
                if rps[-1] <= eps and rds[-1] <= eps:
                    break
        finally:
            self.prob_c.admm_rho = 0.0
            self.prob_c.admm_z = None
            self.prob_c.admm_v = None
        return {"u": self._shape(self.u, self.p.T, self.p.nu), "x": self._shape(self.x, self.p.T + 1, self.p.nx),
                "z": self._shape(z, self.p.T, 2 * self.p.nu), "v": self._shape(v, self.p.T, 2 * self.p.nu),
                "admm_iters": len(inner), "newton_iters": int(sum(inner)), "inner": np.array(inner),
                "rp": np.array(rps), "rd": np.array(rds)}

    def mpc_simulate(self, steps, *, mu_levels, iters, alpha0, nu0, graph=True):
        """Receding-horizon simulation of every instance (Sec. V): per plant step a
        fixed IP budget (iters Newton iterations at each barrier weight), warm start
        from the previous solution shifted by one stage (nmpc_shift), the first control
        applied to the plant (one Euler step).  No host synchronisation inside the
        simulation.  Returns dict(x [B, steps+1, nx], u [B, steps, nu]) (no batch axis
        for B = 1)."""
        B, n, m = self.B, self.p.nx, self.p.nu
        dev = self.x.device
        g = self._kept_step_graph() if graph else None
        x_init = self.x0.clone()
        x_cl = torch.empty(steps + 1, B * n, dtype=torch.float64, device=dev)
        u_cl = torch.empty(steps, B * m, dtype=torch.float64, device=dev)
        try:
            self.u.copy_(self.u0)
            x_cl[0].copy_(self.x0)
            for t in range(steps):
                self.init(alpha0, nu0, reset_u=False)
                for mu in mu_levels:
                    for _ in range(iters):
                        self._sc[:, NMPC_MU] = mu
                        if g is not None:
                            g.replay()
                        else:
                            newton_step(self.plan, self.prob_c, self.state_c, self.ws)
                nmpc_shift(self.plan, self.prob_c, self.state_c, self.x0, u_cl[t])
                x_cl[t + 1].copy_(self.x0)
            torch.cuda.synchronize()
        finally:
            self.x0.copy_(x_init)
        xs = x_cl.cpu().numpy().reshape(steps + 1, B, n).transpose(1, 0, 2)
        us = u_cl.cpu().numpy().reshape(steps, B, m).transpose(1, 0, 2)
        return {"x": xs[0] if B == 1 else xs, "u": us[0] if B == 1 else us}

    def ip_solve(self, *, mu0, zeta, mu_min, tol, max_iter, alpha0, nu0, trace=True, graph=True):
        """The interior-point method of Sec. II-B with converged inner Newton loops:
        mu = mu0, mu0 zeta, ... while mu > mu_min; a level ends after the iteration
        that starts from |dJ_mu/du|_inf <= tol, or after max_iter iterations.

        graph: the level ends on the device and a HIP graph of level_chunk steps,
        captured on the first solve (and again if prob_c has changed since), is
        replayed with one device-to-host copy of the scalars per replay (into pinned
        memory); eagerly (graph=False) the gradient norm is read back after every
        step.  Returns dict(u, x, iters, level_iters, and with trace the
        per-iteration mu, cost, grad, accept, pred).
        """
        g = None
        if graph:
            key = bytes(self.prob_c)
            if self._chunk_key != key:
                self._chunk_graph, self._chunk_key = self._capture_chunk(self.level_chunk), key
            g = self._chunk_graph
        self.init(alpha0, nu0)
        host = torch.empty(self.B * NMPC_NSCAL, dtype=torch.float64, pin_memory=True)
        rows, level_iters = ([] if trace else None), []
        mu = float(mu0)
        while mu > mu_min:
            level_iters.append(self._newton_level(mu, tol, max_iter, host, rows, g))
            mu *= zeta
        out = {"u": self._shape(self.u, self.p.T, self.p.nu), "x": self._shape(self.x, self.p.T + 1, self.p.nx),
               "iters": int(sum(level_iters)), "level_iters": np.array(level_iters)}
        if trace:
            r = np.array(rows).reshape(-1, 5)
            out.update(mu=r[:, 0], cost=r[:, 1], grad=r[:, 2], accept=r[:, 3] > 0.5, pred=r[:, 4])
        return out
