"""Thin Python binding of the C ABI in include/lqscan.h.

Every function named ``lq_*`` here marshals its arguments and calls the C
entry point of the same name; all arithmetic happens in the HIP library.
PyTorch only provides device memory (tensors) and the stream.  There is no
CPU fallback: importing this module fails if liblqscan.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

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
_lib.lq_adjoint.argtypes = [_plan_p, ctypes.POINTER(LQProblemC), ctypes.POINTER(LQValueC), _P, _P, _P, _P, _P,
                            ctypes.POINTER(LQGradsC), _P, _P, _P]
_lib.lq_adjoint.restype = ctypes.c_int
_lib.lq_plan_set_timing.argtypes = [_plan_p, ctypes.c_uint32, ctypes.c_int32]
_lib.lq_plan_set_timing.restype = ctypes.c_int
_lib.lq_plan_phase_times.argtypes = [_plan_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
_lib.lq_plan_phase_times.restype = ctypes.c_int
_lib.lq_selftest_tile_mm.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]
_lib.lq_selftest_tile_mm.restype = ctypes.c_int

EXPORTED = ("lq_plan_create", "lq_plan_destroy", "lq_plan_workspace_bytes", "lq_plan_elements_bytes",
            "lq_plan_seg_len", "lq_plan_total_stages", "lq_build_elements", "lq_scan_solve", "lq_rollout",
            "lq_adjoint", "lq_selftest_tile_mm", "lq_version", "lq_plan_set_timing", "lq_plan_phase_times")

PHASES = ("build", "value_fold", "value_scan", "value_bellman", "roll_fold", "roll_scan", "roll_apply",
          "adj_back", "adj_fwd")


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

    def __init__(self, nx, nu, T, *, precision: str = "fp64", mode: str = "scan", seg_len: int = 0):
        nx, nu, T = (list(map(int, v)) if hasattr(v, "__len__") else [int(v)] for v in (nx, nu, T))
        self.batch = len(T)
        self.nx, self.nu, self.T = nx, nu, T
        self.precision, self.mode = precision, mode
        arr = ctypes.c_int32 * self.batch
        h = _plan_p()
        code = _lib.lq_plan_create(self.batch, arr(*nx), arr(*nu), arr(*T),
                                   {"fp64": LQ_FP64, "mixed": LQ_MIXED}[precision],
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


def lq_adjoint(plan: Plan, prob: dict, value: dict, x, u, lam, gx, gu, grads: dict, workspace, status=None,
               stream=None):
    g = LQGradsC(*[_f64(grads.get(f)) for f in _PROBLEM_FIELDS])
    _check("lq_adjoint", _lib.lq_adjoint(plan.handle, ctypes.byref(_problem_struct(prob)),
                                         ctypes.byref(_value_struct(value)), _f64(x), _f64(u), _f64(lam),
                                         _f64(gx), _f64(gu), ctypes.byref(g), _ptr(workspace), _ptr(status),
                                         _stream(stream)))


def lq_selftest_tile_mm(X, Y, Z, D, tx=False, ty=False, stream=None):
    _check("lq_selftest_tile_mm", _lib.lq_selftest_tile_mm(_f64(X), _f64(Y), _f64(Z), _f64(D), int(tx), int(ty),
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


def solve(plan: Plan, prob: dict, *, materialise_elements: bool = False, workspace=None, stream=None) -> dict:
    """lq_scan_solve + lq_rollout; returns flat packed device tensors and the status array."""
    dev = prob["A"].device
    ws = workspace if workspace is not None else plan.new_workspace(dev)
    status = torch.zeros(plan.batch, dtype=torch.int32, device=dev)
    val = value_buffers(plan, dev)
    st = state_buffers(plan, dev)
    el = None
    if materialise_elements:
        el = plan.new_elements(dev)
        lq_build_elements(plan, prob, el, status, stream)
    lq_scan_solve(plan, prob, el, val, ws, status, stream)
    lq_rollout(plan, prob, val, st["x"], st["u"], st["lam"], ws, status, stream)
    out = dict(val)
    out.update(st)
    out["status"] = status
    out["elements"] = el
    return out
