"""Python access to the FP64 CPU oracle (oracle/lqoracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg use this module; the GPU library never does.
The shared object is compiled with gcc on first use (or by the build step).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqoracle.c")
_LIB = os.path.join(_HERE, "liblqoracle.so")
_lock = threading.Lock()
_lib = None

ERR_NOT_PD = -2
ERR_SINGULAR = -3
ERR_NONFINITE = -4


def build(force: bool = False) -> str:
    """Compile lqoracle.c into liblqoracle.so with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-fno-fast-math",
                        "-ffp-contract=off", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_P = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            i, d = ctypes.c_int, ctypes.c_double
            L.oracle_lq_solve.argtypes = [i, i, i] + [_P] * 11 + [_P] * 7 + [_I]
            L.oracle_lq_solve.restype = i
            L.oracle_value_element.argtypes = [i, i] + [_P] * 8 + [_P]
            L.oracle_value_element.restype = i
            L.oracle_value_terminal.argtypes = [i, _P, _P, _P]
            L.oracle_value_terminal.restype = None
            L.oracle_value_combine.argtypes = [i, _P, _P, _P]
            L.oracle_value_combine.restype = i
            L.oracle_costate_combine.argtypes = [i, _P, _P, _P]
            L.oracle_costate_combine.restype = None
            L.oracle_stateprop_combine.argtypes = [i, _P, _P, _P]
            L.oracle_stateprop_combine.restype = None
            L.oracle_lq_states_cv.argtypes = [i, i, i] + [_P] * 12 + [_I]
            L.oracle_lq_states_cv.restype = i
            L.oracle_lq_adjoint.argtypes = [i, i, i] + [_P] * 11 + [_P] * 2 + [_P] * 11 + [_I]
            L.oracle_lq_adjoint.restype = i
            L.oracle_nmpc_cost.argtypes = [i, i, i, d, i, _P] + [_P] * 7 + [d, d, d, _P, _P, d, _P]
            L.oracle_nmpc_cost.restype = d
            L.oracle_nmpc_rollout.argtypes = [i, i, i, d, i, _P, _P, _P, _P, _P, _P]
            L.oracle_nmpc_rollout.restype = i
            L.oracle_nmpc_f.argtypes = [i, _P, i, i, _P, _P, _P]
            L.oracle_nmpc_f.restype = i
            L.oracle_nmpc_expand.argtypes = [i, i, i, d, i, _P] + [_P] * 6 + [d, d, d, _P, _P, d, _P, _P] + [_P] * 7
            L.oracle_nmpc_expand.restype = None
            L.oracle_nmpc_newton_step.argtypes = ([i, i, i, d, i, _P] + [_P] * 7 + [d, d, d, _P, _P, d]
                                                  + [_P, _P, _P, _P, _P, _P, _P, _P])
            L.oracle_nmpc_newton_step.restype = i
            L.oracle_nmpc_solve.argtypes = ([i, i, i, d, i, _P] + [_P] * 7 + [d, d, _P, i, i, d, d]
                                            + [_P, _P, _P, _I, _P])
            L.oracle_nmpc_solve.restype = i
            L.oracle_nmpc_ip_solve.argtypes = ([i, i, i, d, i, _P] + [_P] * 7 + [d, d, d, d, d, d, i, d, d]
                                               + [_P, _P, i, _P, _P, _P, _P, _I, _I])
            L.oracle_nmpc_ip_solve.restype = i
            L.oracle_nmpc_admm_solve.argtypes = ([i, i, i, d, i, _P] + [_P] * 7 + [d, d, d, d, d, i, i, d, d]
                                                 + [_P, _P, _P, _P, i, _I, _P, _P, _I])
            L.oracle_nmpc_admm_solve.restype = i
            L.oracle_nmpc_admm_update.argtypes = [i, i, d, d, d, _P, _P, _P, i, _P, _P]
            L.oracle_nmpc_admm_update.restype = None
            L.oracle_nmpc_mpc_simulate.argtypes = ([i, i, i, d, i, _P] + [_P] * 8 + [d, d, _P, i, i, d, d, i]
                                                   + [_P, _P])
            L.oracle_nmpc_mpc_simulate.restype = i
            _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _f(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    def __init__(self, code, stage):
        super().__init__(f"oracle status {code} at stage {stage}")
        self.code, self.stage = code, stage


def lq_solve(A, B, c, Q, R, QT, x0, M=None, q=None, r=None, qT=None, *, check=True):
    """Sequential Riccati + rollout + co-states (FP64).

    Returns dict with S [T+1,n,n], s [T+1,n], Gamma [T,m,n], gamma [T,m],
    x [T+1,n], u [T,m], lam [T+1,n], status, fail_k.
    """
    A, B, c, Q, R, QT, x0, M, q, r, qT = map(_f, (A, B, c, Q, R, QT, x0, M, q, r, qT))
    T, n, m = A.shape[0], A.shape[1], B.shape[2]
    out = {"S": np.zeros((T + 1, n, n)), "s": np.zeros((T + 1, n)),
           "Gamma": np.zeros((T, m, n)), "gamma": np.zeros((T, m)),
           "x": np.zeros((T + 1, n)), "u": np.zeros((T, m)), "lam": np.zeros((T + 1, n))}
    fk = ctypes.c_int(-1)
    st = lib().oracle_lq_solve(n, m, T, _p(A), _p(B), _p(c), _p(Q), _p(R), _p(M), _p(q), _p(r),
                               _p(QT), _p(qT), _p(x0), _p(out["S"]), _p(out["s"]),
                               _p(out["Gamma"]), _p(out["gamma"]), _p(out["x"]), _p(out["u"]),
                               _p(out["lam"]), ctypes.byref(fk))
    out["status"], out["fail_k"] = st, fk.value
    if check and st != 0:
        raise OracleError(st, fk.value)
    return out


def lq_states_cv(A, B, c, Q, R, QT, x0, M=None, q=None, r=None, qT=None, *, check=True):
    """Optimal states from the prefix conditional value functions and the
    suffix value functions (eq:value-fun-prefix-sum); x [T+1, n]."""
    A, B, c, Q, R, QT, x0, M, q, r, qT = map(_f, (A, B, c, Q, R, QT, x0, M, q, r, qT))
    T, n, m = A.shape[0], A.shape[1], B.shape[2]
    x = np.zeros((T + 1, n))
    fk = ctypes.c_int(-1)
    st = lib().oracle_lq_states_cv(n, m, T, _p(A), _p(B), _p(c), _p(Q), _p(R), _p(M), _p(q), _p(r),
                                   _p(QT), _p(qT), _p(x0), _p(x), ctypes.byref(fk))
    if check and st != 0:
        raise OracleError(st, fk.value)
    return x


def elem_size(n):
    return 3 * n * n + 2 * n


def unpack_elem(e, n):
    nn = n * n
    return {"A": e[:nn].reshape(n, n), "b": e[nn:nn + n], "C": e[nn + n:2 * nn + n].reshape(n, n),
            "eta": e[2 * nn + n:2 * nn + 2 * n], "J": e[2 * nn + 2 * n:].reshape(n, n)}


def pack_elem(A, b, C, eta, J):
    return np.concatenate([np.ravel(A), np.ravel(b), np.ravel(C), np.ravel(eta), np.ravel(J)]).astype(np.float64)


def value_element(A, B, c, Q, R, M=None, q=None, r=None):
    """eq:value-fun-elem-init (P^{-1}-free form) for one stage."""
    A, B, c, Q, R, M, q, r = map(_f, (A, B, c, Q, R, M, q, r))
    n, m = B.shape
    e = np.zeros(elem_size(n))
    st = lib().oracle_value_element(n, m, _p(A), _p(B), _p(c), _p(Q), _p(R), _p(M), _p(q), _p(r), _p(e))
    if st != 0:
        raise OracleError(st, 0)
    return e


def value_terminal(QT, qT=None):
    QT, qT = _f(QT), _f(qT)
    n = QT.shape[0]
    e = np.zeros(elem_size(n))
    lib().oracle_value_terminal(n, _p(QT), _p(qT), _p(e))
    return e


def value_combine(e1, e2, n):
    """eq:value-fun-param: e1 (earlier) (x) e2 (later)."""
    e1, e2 = _f(e1), _f(e2)
    out = np.zeros(elem_size(n))
    st = lib().oracle_value_combine(n, _p(e1), _p(e2), _p(out))
    if st != 0:
        raise OracleError(st, 0)
    return out


def costate_combine(e1, e2, n):
    e1, e2 = _f(e1), _f(e2)
    out = np.zeros(n + n * n)
    lib().oracle_costate_combine(n, _p(e1), _p(e2), _p(out))
    return out


def stateprop_combine(e1, e2, n):
    e1, e2 = _f(e1), _f(e2)
    out = np.zeros(n + n * n)
    lib().oracle_stateprop_combine(n, _p(e1), _p(e2), _p(out))
    return out


def lq_adjoint(A, B, c, Q, R, QT, x0, gx, gu, M=None, q=None, r=None, qT=None, *, check=True):
    """Gradients of L(x, u) with dL/dx = gx [T+1,n], dL/du = gu [T,m] through the LQ solution."""
    A, B, c, Q, R, QT, x0, gx, gu, M, q, r, qT = map(_f, (A, B, c, Q, R, QT, x0, gx, gu, M, q, r, qT))
    T, n, m = A.shape[0], A.shape[1], B.shape[2]
    g = {"A": np.zeros((T, n, n)), "B": np.zeros((T, n, m)), "c": np.zeros((T, n)),
         "Q": np.zeros((T, n, n)), "R": np.zeros((T, m, m)), "M": np.zeros((T, n, m)),
         "q": np.zeros((T, n)), "r": np.zeros((T, m)), "QT": np.zeros((n, n)), "qT": np.zeros(n),
         "x0": np.zeros(n)}
    fk = ctypes.c_int(-1)
    st = lib().oracle_lq_adjoint(n, m, T, _p(A), _p(B), _p(c), _p(Q), _p(R), _p(M), _p(q), _p(r),
                                 _p(QT), _p(qT), _p(x0), _p(gx), _p(gu),
                                 *[_p(g[k]) for k in ("A", "B", "c", "Q", "R", "M", "q", "r", "QT", "qT", "x0")],
                                 ctypes.byref(fk))
    if check and st != 0:
        raise OracleError(st, fk.value)
    return g


# ----------------------------------------------------------------------------
# Newton / interior point (tanh network, pendulum, cart-pole)
# ----------------------------------------------------------------------------

def _model(p):
    """(model id, parameter array or None) of a problem (tanh when unset)."""
    model = int(getattr(p, "model", 0))
    prm = getattr(p, "param", None)
    return model, (None if prm is None else _f(np.asarray(prm, np.float64)))


def _wb(p):
    return _f(getattr(p, "W", None)), _f(getattr(p, "Bm", None))


def nmpc_f(p, x, u):
    """Continuous-time right-hand side f(x, u) of the pendulum / cart-pole."""
    model, prm = _model(p)
    x, u = _f(x), _f(u)
    f = np.zeros(p.nx)
    if lib().oracle_nmpc_f(model, _p(prm), p.nx, p.nu, _p(x), _p(u), _p(f)) != 0:
        raise ValueError("nmpc_f: pendulum or cart-pole model expected")
    return f


def _admm(admm):
    """(rho, z, v) of an ADMM augmentation dict, or the barrier's (0, None, None)."""
    if admm is None:
        return 0.0, None, None
    return float(admm["rho"]), _f(admm["z"]), _f(admm["v"])


def nmpc_cost(p, u, mu, admm=None):
    """J_mu(u) (barrier), or J_AD(u) with admm = dict(rho, z, v) ([T, 2 nu] arrays)."""
    model, prm = _model(p)
    u = _f(u)
    W, Bm = _wb(p)
    rho, z, v = _admm(admm)
    Q, R, QT, xref, x0 = map(_f, (p.Q, p.R, p.QT, p.xref, p.x0))
    return lib().oracle_nmpc_cost(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R),
                                  _p(QT), _p(xref), _p(x0), float(p.umin), float(p.umax), rho, _p(z), _p(v),
                                  float(mu), _p(u))


def nmpc_expand(p, x, u, mu, admm=None):
    model, prm = _model(p)
    x, u = _f(x), _f(u)
    W, Bm = _wb(p)
    rho, z, v = _admm(admm)
    Q, R, QT, xref = map(_f, (p.Q, p.R, p.QT, p.xref))
    T, n, m = p.T, p.nx, p.nu
    o = {"A": np.zeros((T, n, n)), "B": np.zeros((T, n, m)), "lam": np.zeros((T + 1, n)),
         "P": np.zeros((T, n, n)), "Rh": np.zeros((T, m, m)), "d": np.zeros((T, m)), "M": np.zeros((T, n, m))}
    lib().oracle_nmpc_expand(n, m, T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R), _p(QT), _p(xref),
                             float(p.umin), float(p.umax), rho, _p(z), _p(v), float(mu), _p(x), _p(u),
                             _p(o["A"]), _p(o["B"]), _p(o["lam"]), _p(o["P"]), _p(o["Rh"]), _p(o["d"]),
                             _p(o["M"]))
    return o


def nmpc_rollout(p, u):
    """Nonlinear rollout x [T+1, nx] of the controls u (no feasibility check)."""
    model, prm = _model(p)
    u = _f(np.asarray(u).reshape(p.T, p.nu))
    W, Bm = _wb(p)
    x = np.zeros((p.T + 1, p.nx))
    if lib().oracle_nmpc_rollout(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(_f(p.x0)),
                                 _p(u), _p(x)) != 0:
        raise ValueError("nmpc_rollout: unknown model")
    return x


def nmpc_newton_step(p, x, u, mu, alpha, nu_lm, *, with_grad=False, admm=None):
    """One Alg. 4 iteration; returns (accepted, x, u, alpha, nu_lm, cost, pred, rho)
    (plus |dJ_mu/du|_inf at the starting nominal when with_grad)."""
    model, prm = _model(p)
    x, u = _f(x).copy(), _f(u).copy()
    W, Bm = _wb(p)
    rho_a, z, v = _admm(admm)
    Q, R, QT, xref, x0 = map(_f, (p.Q, p.R, p.QT, p.xref, p.x0))
    a, nl = ctypes.c_double(alpha), ctypes.c_double(nu_lm)
    cost, pred, rho, grad = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    acc = lib().oracle_nmpc_newton_step(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q),
                                        _p(R), _p(QT), _p(xref), _p(x0), float(p.umin), float(p.umax), rho_a,
                                        _p(z), _p(v), float(mu), ctypes.byref(a), ctypes.byref(nl), _p(x), _p(u),
                                        ctypes.byref(cost), ctypes.byref(pred), ctypes.byref(rho),
                                        ctypes.byref(grad))
    if acc < 0:
        raise ValueError("nmpc_newton_step: unknown model")
    out = (bool(acc), x, u, a.value, nl.value, cost.value, pred.value, rho.value)
    return out + (grad.value,) if with_grad else out


def nmpc_solve(p, mu_levels, iters, alpha0, nu0):
    """IP loop with a fixed iteration count per level; returns dict(u, x, cost, accept, alpha)."""
    model, prm = _model(p)
    W, Bm = _wb(p)
    Q, R, QT, xref, x0 = map(_f, (p.Q, p.R, p.QT, p.xref, p.x0))
    u = _f(p.u0).copy()
    x = np.zeros((p.T + 1, p.nx))
    mus = np.asarray(mu_levels, np.float64)
    n_it = len(mus) * iters
    cost, alph = np.zeros(n_it), np.zeros(n_it)
    acc = np.zeros(n_it, np.int32)
    st = lib().oracle_nmpc_solve(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R), _p(QT),
                                 _p(xref), _p(x0), float(p.umin), float(p.umax), _p(mus), len(mus),
                                 iters, float(alpha0), float(nu0), _p(u), _p(x), _p(cost),
                                 acc.ctypes.data_as(_I), _p(alph))
    if st != 0:
        raise OracleError(st, -1)
    return {"u": u, "x": x, "cost": cost, "accept": acc.astype(bool), "alpha": alph}


def nmpc_ip_solve(p, *, mu0, zeta, mu_min, tol, max_iter, alpha0, nu0, cap=4096):
    """Interior-point method with converged inner Newton loops (Sec. II-B, Alg. 4).

    Returns dict(u, x, iters, level_iters, mu, cost, grad, pred, accept) with
    per-iteration traces (grad: |dJ_mu/du|_inf at the nominal each iteration starts from).
    """
    model, prm = _model(p)
    W, Bm = _wb(p)
    Q, R, QT, xref, x0 = map(_f, (p.Q, p.R, p.QT, p.xref, p.x0))
    u = _f(p.u0).copy()
    x = np.zeros((p.T + 1, p.nx))
    mu_t, cost_t, grad_t, pred_t = np.zeros(cap), np.zeros(cap), np.zeros(cap), np.zeros(cap)
    acc_t = np.zeros(cap, np.int32)
    lv = np.zeros(64, np.int32)
    it = lib().oracle_nmpc_ip_solve(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R),
                                    _p(QT), _p(xref), _p(x0), float(p.umin), float(p.umax), float(mu0),
                                    float(zeta), float(mu_min), float(tol), int(max_iter), float(alpha0),
                                    float(nu0), _p(u), _p(x), cap, _p(mu_t), _p(cost_t), _p(grad_t), _p(pred_t),
                                    acc_t.ctypes.data_as(_I), lv.ctypes.data_as(_I))
    if it < 0:
        raise OracleError(it, -1)
    n_lv = 0
    mu = float(mu0)
    while mu > mu_min:
        n_lv += 1
        mu *= zeta
    return {"u": u, "x": x, "iters": it, "level_iters": lv[:n_lv].copy(), "mu": mu_t[:it].copy(),
            "cost": cost_t[:it].copy(), "grad": grad_t[:it].copy(), "pred": pred_t[:it].copy(),
            "accept": acc_t[:it].astype(bool)}


def nmpc_admm_solve(p, *, rho, eps, tol, max_iter, max_admm, alpha0, nu0):
    """ADMM of Sec. II-C for the control box with Alg. 4 as inner solver.

    Returns dict(u, x, z, v, admm_iters, newton_iters, inner [per ADMM iteration],
    rp, rd [residual norms per ADMM iteration]).
    """
    model, prm = _model(p)
    W, Bm = _wb(p)
    Q, R, QT, xref, x0 = map(_f, (p.Q, p.R, p.QT, p.xref, p.x0))
    u = _f(p.u0).copy()
    x = np.zeros((p.T + 1, p.nx))
    z = np.zeros((p.T, 2 * p.nu))
    v = np.zeros((p.T, 2 * p.nu))
    cap = int(max_admm)
    inner = np.zeros(cap, np.int32)
    rp, rd = np.zeros(cap), np.zeros(cap)
    tot = ctypes.c_int(0)
    it = lib().oracle_nmpc_admm_solve(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R),
                                      _p(QT), _p(xref), _p(x0), float(p.umin), float(p.umax), float(rho),
                                      float(eps), float(tol), int(max_iter), int(max_admm), float(alpha0),
                                      float(nu0), _p(u), _p(x), _p(z), _p(v), cap, inner.ctypes.data_as(_I),
                                      _p(rp), _p(rd), ctypes.byref(tot))
    if it < 0:
        raise OracleError(it, -1)
    return {"u": u, "x": x, "z": z, "v": v, "admm_iters": it, "newton_iters": tot.value,
            "inner": inner[:it].copy(), "rp": rp[:it].copy(), "rd": rd[:it].copy()}


def nmpc_admm_update(p, u, z, v, rho, init):
    """One consensus / multiplier step (eq:admm-step-4, -5); returns (z, v, rp, rd) (new arrays)."""
    u = _f(np.asarray(u).reshape(p.T, p.nu))
    z, v = _f(z).copy(), _f(v).copy()
    rp, rd = ctypes.c_double(0.0), ctypes.c_double(0.0)
    lib().oracle_nmpc_admm_update(p.T, p.nu, float(p.umin), float(p.umax), float(rho), _p(u), _p(z), _p(v),
                                  int(bool(init)), ctypes.byref(rp), ctypes.byref(rd))
    return z, v, rp.value, rd.value


def nmpc_mpc_simulate(p, x_init, *, steps, mu_levels, iters, alpha0, nu0):
    """Receding-horizon simulation of `steps` plant steps (fixed IP budget per solve,
    warm start by shifting); returns dict(x [steps+1, nx], u [steps, nu])."""
    model, prm = _model(p)
    W, Bm = _wb(p)
    Q, R, QT, xref = map(_f, (p.Q, p.R, p.QT, p.xref))
    xi = _f(np.asarray(x_init, np.float64))
    ui = _f(np.asarray(p.u0, np.float64).reshape(p.T, p.nu))
    mus = np.asarray(mu_levels, np.float64)
    x_cl = np.zeros((steps + 1, p.nx))
    u_cl = np.zeros((steps, p.nu))
    st = lib().oracle_nmpc_mpc_simulate(p.nx, p.nu, p.T, float(p.h), model, _p(prm), _p(W), _p(Bm), _p(Q), _p(R),
                                        _p(QT), _p(xref), _p(xi), _p(ui), float(p.umin), float(p.umax), _p(mus),
                                        len(mus), int(iters), float(alpha0), float(nu0), int(steps), _p(x_cl),
                                        _p(u_cl))
    if st != 0:
        raise OracleError(st, -1)
    return {"x": x_cl, "u": u_cl}
