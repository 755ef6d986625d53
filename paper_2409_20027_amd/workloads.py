"""Seeded synthetic workloads for the LQ subproblem and the Newton/IP problem.

This module only draws random numbers and packs arrays.  It holds none of the
solver's arithmetic, so both the CPU oracle's tests and the GPU path's tests and
benchmark can use it without sharing any method code.

Index convention: stages k = 0..T-1, terminal state x_T (the paper's t = 1..N
with terminal x_{N+1}; k = t - 1).  All arrays are float64, C-contiguous,
stage-major with row-major matrices:

    A [T, n, n]   B [T, n, m]   c [T, n]
    Q [T, n, n]   R [T, m, m]   M [T, n, m] (optional)
    q [T, n]      r [T, m]      (optional)
    QT [n, n]     qT [n] (optional)   x0 [n]

Recipe (one generator per instance, draws in this order):
    Z  = standard_normal((T, n*n + n*m + n))  -> A = I + a_scale*Z_A,
                                                 B = 0.1*Z_B, c = 0.01*Z_c
    U  = random((T, n [+ m]))                 -> Q = diag(0.5 + 1.5*U_Q),
                                                 R = diag(0.1 + 0.9*U_R)
                                                 (or R = r_fixed*I, no draw)
    x0 = standard_normal(n)
    QT = 10*I (no draw)
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LQ_FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r")


@dataclasses.dataclass
class LQInstance:
    n: int
    m: int
    T: int
    A: np.ndarray
    B: np.ndarray
    c: np.ndarray | None
    Q: np.ndarray
    R: np.ndarray
    QT: np.ndarray
    x0: np.ndarray
    M: np.ndarray | None = None
    q: np.ndarray | None = None
    r: np.ndarray | None = None
    qT: np.ndarray | None = None

    def arrays(self):
        return {k: getattr(self, k) for k in
                ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")}


def lq_instance(rng: np.random.Generator, n: int, m: int, T: int, *,
                a_scale: float = 0.05, r_fixed: float | None = None,
                qt_scale: float = 10.0) -> LQInstance:
    """One time-varying LQ instance drawn as described in the module docstring."""
    nn, nm = n * n, n * m
    Z = rng.standard_normal((T, nn + nm + n))
    U = rng.random((T, n + (0 if r_fixed is not None else m)))
    x0 = rng.standard_normal(n)
    eye = np.eye(n)
    A = eye[None] + a_scale * Z[:, :nn].reshape(T, n, n)
    B = 0.1 * Z[:, nn:nn + nm].reshape(T, n, m)
    c = 0.01 * Z[:, nn + nm:]
    Q = np.zeros((T, n, n))
    idx = np.arange(n)
    Q[:, idx, idx] = 0.5 + 1.5 * U[:, :n]
    R = np.zeros((T, m, m))
    jdx = np.arange(m)
    if r_fixed is not None:
        R[:, jdx, jdx] = r_fixed
    else:
        R[:, jdx, jdx] = 0.1 + 0.9 * U[:, n:]
    QT = qt_scale * np.eye(n)
    return LQInstance(n, m, T, np.ascontiguousarray(A), np.ascontiguousarray(B),
                      np.ascontiguousarray(c), Q, R, QT, np.ascontiguousarray(x0))


def lq_instance_general(rng: np.random.Generator, n: int, m: int, T: int, *,
                        a_scale: float = 0.1, cross: float = 0.2) -> LQInstance:
    """A dense LQ instance with every optional term present (M, q, r, qT, c).

    Q and R are drawn as random SPD matrices and the cross term M is scaled so
    that the joint stage Hessian [[Q, M], [M^T, R]] stays positive definite.
    """
    inst = lq_instance(rng, n, m, T, a_scale=a_scale)
    GQ = rng.standard_normal((T, n, n)) / math.sqrt(n)
    GR = rng.standard_normal((T, m, m)) / math.sqrt(m)
    Q = np.einsum("tij,tkj->tik", GQ, GQ) + np.eye(n)[None]
    R = np.einsum("tij,tkj->tik", GR, GR) + 0.5 * np.eye(m)[None]
    M = cross * rng.standard_normal((T, n, m)) / math.sqrt(n * m)
    inst.Q = np.ascontiguousarray(Q)
    inst.R = np.ascontiguousarray(R)
    inst.M = np.ascontiguousarray(M)
    inst.q = rng.standard_normal((T, n))
    inst.r = rng.standard_normal((T, m))
    GT = rng.standard_normal((n, n)) / math.sqrt(n)
    inst.QT = GT @ GT.T + np.eye(n)
    inst.qT = rng.standard_normal(n)
    return inst


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def cfg0_small(seed: int = 0) -> LQInstance:
    """n=2, m=1, T=64, A = I + 0.05 N(0,1)."""
    return lq_instance(np.random.default_rng(seed), 2, 1, 64, a_scale=0.05)


def cfg2_long(seed: int = 2, T: int = 16384) -> LQInstance:
    """Quadrotor-sized long horizon: n=12, m=4, A = I + 0.02 N(0,1), R = 0.1 I."""
    return lq_instance(np.random.default_rng(seed), 12, 4, T, a_scale=0.02, r_fixed=0.1)


def cfg4_batch(seed: int = 4, batch: int = 256, T: int = 4096):
    """Batch of identical-shape long-horizon instances (n=12, m=4)."""
    rng = np.random.default_rng(seed)
    return [lq_instance(rng, 12, 4, T, a_scale=0.02, r_fixed=0.1) for _ in range(batch)]


def cfg3_ragged_sizes(seed: int = 3, count: int = 4096, tmin: int = 32, tmax: int = 2048):
    """Sizes of the ragged batch: T ~ U{tmin..tmax}, n ~ U{2,4,12}, m = max(1, n//3)."""
    rng = np.random.default_rng(seed)
    Ts = rng.integers(tmin, tmax + 1, size=count)
    ns = rng.choice(np.array([2, 4, 12]), size=count)
    ms = np.maximum(1, ns // 3)
    return rng, ns.astype(np.int32), ms.astype(np.int32), Ts.astype(np.int32)


def cfg3_ragged(seed: int = 3, count: int = 4096, tmin: int = 32, tmax: int = 2048):
    """The ragged batch itself: sizes from cfg3_ragged_sizes, then one instance each."""
    rng, ns, ms, Ts = cfg3_ragged_sizes(seed, count, tmin, tmax)
    return [lq_instance(rng, int(n), int(m), int(T), a_scale=0.05)
            for n, m, T in zip(ns, ms, Ts)]


def device_batch(sizes, *, seed: int, a_scale: float = 0.05, r_fixed: float | None = None,
                 qt_scale: float = 10.0, device="cuda"):
    """A batch drawn like lq_instance, generated on the device and packed.

    sizes: list of (n, m, T) in packing order; consecutive instances of equal
    (n, m) are drawn as one block, so order a ragged batch by size class.
    The distributions are those of lq_instance (A = I + a N(0,1), B ~ 0.1 N,
    c ~ 0.01 N, Q = diag(U[0.5, 2]), R = diag(U[0.1, 1]) or r_fixed I,
    Q_T = qt_scale I, x0 ~ N(0, 1)); the numbers come from torch's generator,
    not from the numpy stream, so this serves throughput measurement, not
    parity.  Returns the packed dict of device tensors (lq_problem fields).
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = dict(dtype=torch.float64, device=device)
    parts = {k: [] for k in ("A", "B", "c", "Q", "R", "QT", "x0")}
    i = 0
    while i < len(sizes):
        n, m, _ = sizes[i]
        j = i
        while j < len(sizes) and sizes[j][0] == n and sizes[j][1] == m:
            j += 1
        Ts = sum(int(t) for _, _, t in sizes[i:j])
        cnt = j - i
        eye = torch.eye(n, **f64)
        parts["A"].append((eye + a_scale * torch.randn(Ts, n, n, generator=g, **f64)).reshape(-1))
        parts["B"].append((0.1 * torch.randn(Ts, n, m, generator=g, **f64)).reshape(-1))
        parts["c"].append((0.01 * torch.randn(Ts, n, generator=g, **f64)).reshape(-1))
        qd = 0.5 + 1.5 * torch.rand(Ts, n, generator=g, **f64)
        parts["Q"].append(torch.diag_embed(qd).reshape(-1))
        if r_fixed is not None:
            rd = torch.full((Ts, m), float(r_fixed), **f64)
        else:
            rd = 0.1 + 0.9 * torch.rand(Ts, m, generator=g, **f64)
        parts["R"].append(torch.diag_embed(rd).reshape(-1))
        parts["QT"].append((qt_scale * eye).repeat(cnt, 1, 1).reshape(-1))
        parts["x0"].append(torch.randn(cnt, n, generator=g, **f64).reshape(-1))
        i = j
    out = {k: torch.cat(v).contiguous() for k, v in parts.items()}
    out.update({"M": None, "q": None, "r": None, "qT": None})
    return out


# ---------------------------------------------------------------------------
# Packing of a (possibly ragged) batch into the flat stage-major layout
# ---------------------------------------------------------------------------

def pack(instances) -> dict:
    """Concatenate a list of LQInstance into the flat packed layout.

    An optional field (c, M, q, r, qT) is packed if any instance has it, with
    zeros for the instances that do not (None means zero); it is None only if
    no instance has it.
    """
    out = {"n": np.array([i.n for i in instances], np.int32),
           "m": np.array([i.m for i in instances], np.int32),
           "T": np.array([i.T for i in instances], np.int32)}
    shapes = {"A": lambda i: (i.T, i.n, i.n), "B": lambda i: (i.T, i.n, i.m), "c": lambda i: (i.T, i.n),
              "Q": lambda i: (i.T, i.n, i.n), "R": lambda i: (i.T, i.m, i.m), "M": lambda i: (i.T, i.n, i.m),
              "q": lambda i: (i.T, i.n), "r": lambda i: (i.T, i.m), "QT": lambda i: (i.n, i.n),
              "qT": lambda i: (i.n,), "x0": lambda i: (i.n,)}
    for f, shp in shapes.items():
        vals = [getattr(i, f) for i in instances]
        if all(v is None for v in vals):
            out[f] = None
            continue
        out[f] = np.ascontiguousarray(np.concatenate(
            [(np.zeros(shp(i)) if v is None else v).reshape(-1) for v, i in zip(vals, instances)]))
    return out


# ---------------------------------------------------------------------------
# Newton / interior-point workload: x' = x + h (tanh(W x) + B u), |u| <= 1
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class NMPCProblem:
    nx: int
    nu: int
    T: int
    h: float
    W: np.ndarray      # [nx, nx]
    Bm: np.ndarray     # [nx, nu]
    Q: np.ndarray      # [nx, nx]
    R: np.ndarray      # [nu, nu]
    QT: np.ndarray     # [nx, nx]
    xref: np.ndarray   # [T+1, nx]
    x0: np.ndarray     # [nx]
    u0: np.ndarray     # [T, nu] strictly feasible initial controls
    umin: float = -1.0
    umax: float = 1.0
    model: int = 0                  # NMPC_TANH, NMPC_PENDULUM or NMPC_CARTPOLE
    param: np.ndarray | None = None  # model constants (pendulum g, l, m, b; cart-pole g, l, m_c, m_p)


def nmpc_problem(seed: int = 1, nx: int = 4, nu: int = 1, T: int = 1024,
                 h: float = 0.02) -> NMPCProblem:
    """Synthetic tanh-network dynamics with a sinusoidal tracking reference.

    Draw order: W ~ N(0, 1/nx), B ~ N(0, 1), x0 ~ N(0, 0.5^2), u0 ~ N(0, 0.1^2)
    (clipped to |u| <= 0.9 so that the barrier starts strictly feasible).
    Q = I, R = 0.1 I, QT = 10 I, ref[k, i] = 0.5 sin(2 pi k / 256 + pi i / 4).
    """
    rng = np.random.default_rng(seed)
    W = rng.standard_normal((nx, nx)) / math.sqrt(nx)
    Bm = rng.standard_normal((nx, nu))
    x0 = 0.5 * rng.standard_normal(nx)
    u0 = np.clip(0.1 * rng.standard_normal((T, nu)), -0.9, 0.9)
    k = np.arange(T + 1)[:, None]
    i = np.arange(nx)[None, :]
    xref = 0.5 * np.sin(2 * math.pi * k / 256.0 + math.pi * i / 4.0)
    return NMPCProblem(nx, nu, T, h, W, Bm, np.eye(nx), 0.1 * np.eye(nu), 10.0 * np.eye(nx),
                       np.ascontiguousarray(xref), x0, np.ascontiguousarray(u0))


NMPC_TANH, NMPC_PENDULUM, NMPC_CARTPOLE = 0, 1, 2
PENDULUM_TF = 4.0   # seconds (the time spans are not printed)
CARTPOLE_TF = 3.0

# Sec. V: pendulum g = 9.81, l = 1, m = 1, b = 1e-3, |tau| < 5;
# cart-pole g = 9.81, l = 0.5, m_c = 10, m_p = 1, |F| < 60.
PENDULUM_PARAM = (9.81, 1.0, 1.0, 1e-3)
PENDULUM_UMAX = 5.0
CARTPOLE_PARAM = (9.81, 0.5, 10.0, 1.0)
CARTPOLE_UMAX = 60.0
# Interior-point schedule of Sec. V: mu from 0.1, times 0.2 while above 1e-4.
IP_MU0, IP_ZETA, IP_MU_MIN = 0.1, 0.2, 1e-4
# Inner Newton loop: converged after the iteration that starts from a nominal
# with |dJ_mu/du|_inf <= IP_TOL (the threshold itself is not printed), at
# most IP_MAX_ITER iterations per barrier level.
IP_TOL, IP_MAX_ITER = 1e-6, 100
# Segment length of the parallel path for these small systems (n <= 4):
# shorter segments than the default (fewer stages in the per-segment kernels,
# which dominate at n <= 4) measured fastest for N >= 100.
IP_SEG_LEN = 4
# ADMM of Sec. V: rho = 1 (pendulum), 0.5 (cart-pole) per unit time (each
# stage's augmentation term is weighted h rho, like the stage cost), stop at
# |r_p|_inf, |r_d|_inf <= 1e-2; the inner Newton loops share IP_TOL and
# IP_MAX_ITER; at most ADMM_MAX_ITER ADMM iterations.
ADMM_RHO = {"pendulum": 1.0, "cartpole": 0.5}
ADMM_EPS = 1e-2
ADMM_MAX_ITER = 5000
# Horizon lengths of the runtime figures of Sec. V.
PAPER_HORIZONS = (20, 40, 80, 100, 200, 400, 800, 1000)


def pendulum_problem(N: int, seed: int = 0, t_final: float = PENDULUM_TF) -> NMPCProblem:
    """Torque-limited pendulum swing-up over a fixed time t_final in N Euler steps.

    x = (theta, omega), theta = 0 hanging down; from rest at the bottom to the
    upright x_ref = (pi, 0) at the end: control effort h * 1.0 * tau^2 / 2 per
    step (a Riemann sum, so that the problem is the same for every N), no
    running state cost, Q_T = diag(100, 10), |tau| < 5.  Initial controls:
    u0 ~ N(0, 0.1^2) (strictly feasible).
    """
    rng = np.random.default_rng(seed)
    u0 = 0.1 * rng.standard_normal((N, 1))
    h = t_final / N
    xref = np.tile(np.array([math.pi, 0.0]), (N + 1, 1))
    return NMPCProblem(2, 1, N, h, None, None, np.zeros((2, 2)), np.array([[h * 1.0]]),
                       np.diag([100.0, 10.0]), xref, np.zeros(2), u0, -PENDULUM_UMAX, PENDULUM_UMAX,
                       NMPC_PENDULUM, np.array(PENDULUM_PARAM))


def cartpole_problem(N: int, seed: int = 0, t_final: float = CARTPOLE_TF) -> NMPCProblem:
    """Force-limited cart-pole swing-up over a fixed time t_final in N Euler steps.

    x = (p, theta, v, omega), theta = 0 hanging down; from rest to the upright
    x_ref = (0, pi, 0, 0) at the end: control effort h * 0.01 * F^2 / 2 per
    step, no running state cost, Q_T = diag(100, 100, 10, 10), |F| < 60.
    Initial controls: u0 ~ N(0, 1).
    """
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((N, 1))
    h = t_final / N
    xref = np.tile(np.array([0.0, math.pi, 0.0, 0.0]), (N + 1, 1))
    return NMPCProblem(4, 1, N, h, None, None, np.zeros((4, 4)), np.array([[h * 0.01]]),
                       np.diag([100.0, 100.0, 10.0, 10.0]), xref, np.zeros(4), u0, -CARTPOLE_UMAX, CARTPOLE_UMAX,
                       NMPC_CARTPOLE, np.array(CARTPOLE_PARAM))


# Receding-horizon MPC of Sec. V: N = 60 stages at 100 Hz, 4 s of plant time.
MPC_N, MPC_H, MPC_STEPS = 60, 0.01, 400
# Per MPC step (proposed; the paper gives no budget): the IP schedule's five
# barrier levels with MPC_ITERS Newton iterations each, warm start from the
# previous solution shifted by one stage, damping restarted.
MPC_ITERS = 2
MPC_MU_LEVELS = tuple(IP_MU0 * IP_ZETA ** k for k in range(5))


def mpc_problem(name: str, x_init: np.ndarray) -> NMPCProblem:
    """Stabilisation MPC (Sec. V): the pendulum upright, the cart-pole upright
    with the cart at 0, from the states x_init ([B, nx]); stage cost
    h (x - x_ref)'Q(x - x_ref)/2 + h R u^2/2 (pendulum Q = diag(100, 10),
    R = 0.1; cart-pole Q = diag(10, 50, 1, 1), R = 1e-3), Q_T = diag(100, 10)
    / diag(100, 100, 10, 10), bounds |tau| < 5, |F| < 60, zero initial
    controls.  Costs and initial states are proposed (not printed)."""
    N, h = MPC_N, MPC_H
    x_init = np.ascontiguousarray(np.asarray(x_init, np.float64))
    B = 1 if x_init.ndim == 1 else x_init.shape[0]
    if name == "pendulum":
        p = pendulum_problem(N, t_final=N * h)
        Qc, Rc, QT = np.diag([100.0, 10.0]), 0.1, np.diag([100.0, 10.0])
    else:
        p = cartpole_problem(N, t_final=N * h)
        Qc, Rc, QT = np.diag([10.0, 50.0, 1.0, 1.0]), 1e-3, np.diag([100.0, 100.0, 10.0, 10.0])
    u0 = np.zeros((N, 1)) if B == 1 else np.zeros((B, N, 1))
    return dataclasses.replace(p, Q=h * Qc, R=np.array([[h * Rc]]), QT=QT, x0=x_init, u0=u0)


def mpc_initial_states(name: str, count: int, seed: int = 7) -> np.ndarray:
    """Initial states around the upright equilibrium, inside the region this
    short-horizon, input-bounded controller recovers (the torque limit 5 is
    half of m g l): pendulum theta ~ pi + U(-0.3, 0.3), omega ~ U(-0.3, 0.3);
    cart-pole p ~ U(-0.3, 0.3), theta ~ pi + U(-0.4, 0.4), v, omega ~
    U(-0.3, 0.3)."""
    rng = np.random.default_rng(seed)
    if name == "pendulum":
        return np.stack([math.pi + rng.uniform(-0.3, 0.3, count), rng.uniform(-0.3, 0.3, count)], axis=1)
    return np.stack([rng.uniform(-0.3, 0.3, count), math.pi + rng.uniform(-0.4, 0.4, count),
                     rng.uniform(-0.3, 0.3, count), rng.uniform(-0.3, 0.3, count)], axis=1)


NMPC_MU_LEVELS = (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)
NMPC_ITERS_PER_LEVEL = 10
NMPC_ALPHA0 = 1e-3
NMPC_NU0 = 2.0
