"""FP64 CPU oracle of the differentiable IDM simulator (arXiv 2412.16750).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark.  The product path (``paper_2412_16750_amd``)
never imports it, and the two share no code.

The numerical work is in ``idm_oracle.c`` (plain sequential C, double
precision), which follows Sec. III-A (Eqs. 1-3), Sec. III-B (synchronous
per-frame update) and Sec. III-C (softplus lower bounds) of the paper, plus a
hand-derived adjoint and tangent-linear model of the same equations.  The
MLP oracle for the learned warm start is in ``mlp.py``.

This module only builds/loads that library and marshals NumPy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "idm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_SOFTPLUS = 0
MODE_CLAMP = 1
PARAM_NAMES = ("v0", "T", "a", "b", "s0")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        d, i, pd, pi = ctypes.c_double, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p
        common = [i, d, d, d, d, i, i, pi, i] + [pd] * 6
        L.oracle_forward.restype = ctypes.c_long
        L.oracle_forward.argtypes = common + [pd, pd, pd, pd, pd]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_adjoint.argtypes = common + [pd, pd, pd, pd, pd, pd, pd, pd]
        L.oracle_branch_terms.restype = ctypes.c_int
        L.oracle_branch_terms.argtypes = common + [pd, pd, pd, pd]
        L.oracle_tangent.restype = ctypes.c_int
        L.oracle_tangent.argtypes = common + [pd, pd, pd, pd, pd, pd, pd]
        L.oracle_mse.restype = ctypes.c_double
        L.oracle_mse.argtypes = [i, i, pd, i, pi, pd, pd]
        L.oracle_mae_sum.restype = ctypes.c_double
        L.oracle_mae_sum.argtypes = [i, i, pd, i, pi, pd, pd]
        ego = [i, d, d, d, d, i, i] + [pd] * 7
        L.oracle_ego_forward.restype = ctypes.c_long
        L.oracle_ego_forward.argtypes = ego + [pd, pd, pd, pd]
        L.oracle_ego_adjoint.restype = ctypes.c_int
        L.oracle_ego_adjoint.argtypes = ego + [pd] * 7
        L.oracle_ego_tangent.restype = ctypes.c_int
        L.oracle_ego_tangent.argtypes = ego + [pd] * 7
        L.oracle_ego_mae.restype = ctypes.c_double
        L.oracle_ego_mae.argtypes = [i, i, pd, pi, pi, pd, pd]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Problem:
    """Plain description of one simulation problem in float64."""

    def __init__(self, lane_offsets, params: Dict[str, np.ndarray], p0, v_init, n_steps: int,
                 dt: float = 0.1, delta: float = 4.0, a_min: float = -10.0,
                 gap_floor: float = 1e-3, mode: int = MODE_SOFTPLUS):
        self.lane_offsets = np.ascontiguousarray(np.asarray(lane_offsets, dtype=np.int32))
        self.n = int(self.lane_offsets[-1])
        self.n_lanes = len(self.lane_offsets) - 1
        self.params = {k: _d(params[k]) for k in PARAM_NAMES}
        self.length = _d(params["length"])
        self.p0 = _d(p0)
        self.v_init = _d(v_init)
        self.n_steps = int(n_steps)
        self.dt, self.delta, self.a_min, self.gap_floor = float(dt), float(delta), float(a_min), float(gap_floor)
        self.mode = int(mode)

    @classmethod
    def from_scenario(cls, sc, params=None, mode=None, n_steps=None):
        return cls(sc.lane_offsets, params if params is not None else sc.params, sc.p0, sc.v_init,
                   sc.n_steps if n_steps is None else n_steps, sc.dt, sc.delta, sc.a_min,
                   sc.gap_floor, sc.mode if mode is None else mode)

    def _head(self):
        pr = self.params
        return [self.mode, self.dt, self.delta, self.a_min, self.gap_floor, self.n, self.n_lanes,
                _p(self.lane_offsets), self.n_steps, _p(pr["v0"]), _p(pr["T"]), _p(pr["a"]),
                _p(pr["b"]), _p(pr["s0"]), _p(self.length)]


def forward(pb: Problem, want_acc: bool = False):
    """Returns (P, V, A or None, floor_hits); P, V are [(S+1), N] float64."""
    S, n = pb.n_steps, pb.n
    P = np.empty((S + 1, n), dtype=np.float64)
    V = np.empty((S + 1, n), dtype=np.float64)
    A = np.empty((S, n), dtype=np.float64) if want_acc else None
    hits = lib().oracle_forward(*pb._head(), _p(pb.p0), _p(pb.v_init), _p(P), _p(V), _p(A))
    if hits < 0:
        raise ValueError("oracle_forward: invalid arguments")
    return P, V, A, int(hits)


def adjoint(pb: Problem, P, V, gP, gV=None, magnitude: bool = False):
    """Returns (g_params [5, N] in (v0, T, a, b, s0) order, g_p0 [N], g_v0 [N]),
    plus, with magnitude=True, the [5, N] sums of the absolute per-step terms
    of each parameter gradient."""
    S, n = pb.n_steps, pb.n
    gP = _d(gP).reshape(S + 1, n)
    gV = None if gV is None else _d(gV).reshape(S + 1, n)
    g = np.empty((5, n), dtype=np.float64)
    gp0 = np.empty(n, dtype=np.float64)
    gv0 = np.empty(n, dtype=np.float64)
    gabs = np.empty((5, n), dtype=np.float64) if magnitude else None
    rc = lib().oracle_adjoint(*pb._head(), _p(_d(P)), _p(_d(V)), _p(gP), _p(gV), _p(g), _p(gp0),
                              _p(gv0), _p(gabs))
    if rc != 0:
        raise ValueError("oracle_adjoint: invalid arguments")
    return (g, gp0, gv0, gabs) if magnitude else (g, gp0, gv0)


def branch_terms(pb: Problem, P, V):
    """Per step k < S and vehicle: (AH, GAP) = the IDM acceleration of Eq. 2
    before the Sec. III-C bound / the speed clamp, and the raw gap to the
    leader (+inf for a lane head); [S, N] each."""
    S, n = pb.n_steps, pb.n
    AH = np.empty((S, n), dtype=np.float64)
    GAP = np.empty((S, n), dtype=np.float64)
    rc = lib().oracle_branch_terms(*pb._head(), _p(_d(P)), _p(_d(V)), _p(AH), _p(GAP))
    if rc != 0:
        raise ValueError("oracle_branch_terms: invalid arguments")
    return AH, GAP


def tangent(pb: Problem, P, V, dprm, dp0, dv0):
    S, n = pb.n_steps, pb.n
    dP = np.empty((S + 1, n), dtype=np.float64)
    dV = np.empty((S + 1, n), dtype=np.float64)
    rc = lib().oracle_tangent(*pb._head(), _p(_d(P)), _p(_d(V)), _p(_d(dprm).reshape(5, n)), _p(_d(dp0)),
                              _p(_d(dv0)), _p(dP), _p(dV))
    if rc != 0:
        raise ValueError("oracle_tangent: invalid arguments")
    return dP, dV


def mse(P, steps: Sequence[int], target, want_grad: bool = True):
    """Mean squared error over observed steps; returns (loss, dL/dP or None)."""
    P = _d(P)
    S1, n = P.shape
    steps = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
    target = _d(target).reshape(len(steps), n)
    gP = np.zeros_like(P) if want_grad else None
    loss = lib().oracle_mse(n, S1 - 1, _p(P), len(steps), _p(steps), _p(target), _p(gP))
    return float(loss), gP


def mae_sum(P, steps: Sequence[int], target, want_grad: bool = True):
    """The paper's summed absolute reconstruction error (Sec. IV-A, Eq. 4)."""
    P = _d(P)
    S1, n = P.shape
    steps = np.ascontiguousarray(np.asarray(steps, dtype=np.int32))
    target = _d(target).reshape(len(steps), n)
    gP = np.zeros_like(P) if want_grad else None
    loss = lib().oracle_mae_sum(n, S1 - 1, _p(P), len(steps), _p(steps), _p(target), _p(gP))
    return float(loss), gP


def loss_and_grads(pb: Problem, steps, target, dense_grad=None):
    """Forward + MSE (+ optional dense upstream dL/dP added) + adjoint."""
    P, V, _, hits = forward(pb)
    loss, gP = mse(P, steps, target)
    if dense_grad is not None:
        gP = gP + _d(dense_grad).reshape(gP.shape)
    g, gp0, gv0 = adjoint(pb, P, V, gP)
    return dict(P=P, V=V, loss=loss, g=g, gp0=gp0, gv0=gv0, floor_hits=hits)


# --------------------------------------------------------------------------
# Ego-only reconstruction (Sec. IV-A): one vehicle per trajectory, per-step
# free gap G and speed difference D to an unsimulated leader, p(0) = 0, loss =
# summed absolute error at the observed steps.


class EgoProblem:
    """n trajectories over n_steps steps; params [N] each, G and D [S, N]."""

    def __init__(self, params: Dict[str, np.ndarray], G, D, v_init, n_steps: int,
                 dt: float = 1.0, delta: float = 4.0, a_min: float = -10.0,
                 gap_floor: float = 1e-3, mode: int = MODE_SOFTPLUS):
        self.params = {k: _d(params[k]) for k in PARAM_NAMES}
        self.n = len(self.params["v0"])
        self.n_steps = int(n_steps)
        self.G = _d(G).reshape(self.n_steps, self.n)
        self.D = _d(D).reshape(self.n_steps, self.n)
        self.v_init = _d(v_init)
        self.dt, self.delta, self.a_min, self.gap_floor = float(dt), float(delta), float(a_min), float(gap_floor)
        self.mode = int(mode)

    def _head(self):
        pr = self.params
        return [self.mode, self.dt, self.delta, self.a_min, self.gap_floor, self.n, self.n_steps,
                _p(pr["v0"]), _p(pr["T"]), _p(pr["a"]), _p(pr["b"]), _p(pr["s0"]), _p(self.G),
                _p(self.D)]


def ego_forward(pb: EgoProblem, want_acc: bool = False):
    """Returns (P, V, A or None, floor_hits); P, V [(S+1), N], P(0) = 0."""
    S, n = pb.n_steps, pb.n
    P = np.empty((S + 1, n), dtype=np.float64)
    V = np.empty((S + 1, n), dtype=np.float64)
    A = np.empty((S, n), dtype=np.float64) if want_acc else None
    hits = lib().oracle_ego_forward(*pb._head(), _p(pb.v_init), _p(P), _p(V), _p(A))
    if hits < 0:
        raise ValueError("oracle_ego_forward: invalid arguments")
    return P, V, A, int(hits)


def ego_adjoint(pb: EgoProblem, P, V, gP):
    """Returns (g_params [5, N], g_G [S, N], g_D [S, N], g_v0 [N])."""
    S, n = pb.n_steps, pb.n
    g = np.empty((5, n), dtype=np.float64)
    gG = np.empty((S, n), dtype=np.float64)
    gD = np.empty((S, n), dtype=np.float64)
    gv0 = np.empty(n, dtype=np.float64)
    rc = lib().oracle_ego_adjoint(*pb._head(), _p(_d(P)), _p(_d(V)), _p(_d(gP).reshape(S + 1, n)),
                                  _p(g), _p(gG), _p(gD), _p(gv0))
    if rc != 0:
        raise ValueError("oracle_ego_adjoint: invalid arguments")
    return g, gG, gD, gv0


def ego_tangent(pb: EgoProblem, V, dprm, dG, dD, dv0):
    S, n = pb.n_steps, pb.n
    dP = np.empty((S + 1, n), dtype=np.float64)
    dV = np.empty((S + 1, n), dtype=np.float64)
    rc = lib().oracle_ego_tangent(*pb._head(), _p(_d(V)), _p(_d(dprm).reshape(5, n)),
                                  _p(_d(dG).reshape(S, n)), _p(_d(dD).reshape(S, n)), _p(_d(dv0)),
                                  _p(dP), _p(dV))
    if rc != 0:
        raise ValueError("oracle_ego_tangent: invalid arguments")
    return dP, dV


def ego_mae(P, obs_off, obs_step, obs_pos, want_grad: bool = True):
    """Summed absolute error over each trajectory's observations (CSR by
    trajectory); returns (loss, dL/dP or None)."""
    P = _d(P)
    S1, n = P.shape
    off = np.ascontiguousarray(np.asarray(obs_off, dtype=np.int32))
    st = np.ascontiguousarray(np.asarray(obs_step, dtype=np.int32))
    pos = _d(obs_pos)
    gP = np.zeros_like(P) if want_grad else None
    loss = lib().oracle_ego_mae(n, S1 - 1, _p(P), _p(off), _p(st), _p(pos), _p(gP))
    return float(loss), gP


def reconstruction_metrics(P, A, obs_off, obs_step, obs_pos) -> dict:
    """Plain loops over the paper's evaluation criteria (Sec. V-B4): mean over
    observations of |obs - P[step]| / (last - first observed position of the
    trajectory, at least 1 m); mean and standard deviation of |a| over the
    steps before each trajectory's last observed step; fraction of
    trajectories with |a| > 10 at any of those steps."""
    P, A = _d(P), _d(A)
    n = len(obs_off) - 1
    rel, accs, bad = [], [], 0
    for i in range(n):
        lo, hi = int(obs_off[i]), int(obs_off[i + 1])
        if hi == lo:
            continue
        length = max(abs(float(obs_pos[hi - 1]) - float(obs_pos[lo])), 1.0)
        for j in range(lo, hi):
            rel.append(abs(float(obs_pos[j]) - P[int(obs_step[j]), i]) / length)
        a = np.abs(A[:int(obs_step[hi - 1]), i])
        accs.append(a)
        bad += int(np.any(a > 10.0))
    acc = np.concatenate(accs) if accs else np.zeros(0)
    return {"pos_error": float(np.mean(rel)) if rel else 0.0,
            "acc_mean": float(acc.mean()) if acc.size else 0.0,
            "acc_std": float(acc.std()) if acc.size else 0.0,
            "implausible": bad / n}
