"""Ego-only trajectory reconstruction (Sec. IV-A): each trajectory is one
vehicle starting at p(0) = 0 whose leader is not simulated; the gap G_k and
speed difference D_k to it at every step are fitted together with the five IDM
parameters to sparse observed positions, by Adam on the summed absolute error
(Sec. V-B3: 500 steps, learning rate 0.1 -> 0.01, parameters initialised to
v0 50, T 1, a 10, b 2, s0 5 within boxes, G = 10, D = 0, v(0) = first observed
displacement / time).

Argument marshalling only: forward, loss, gradient, Adam, the step matching and
the initial speed run in libidmx.so's HIP kernels (idm_ego_*).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

from . import _lib, sim
from ._lib import BOUND_SOFTPLUS, IdmEgoFitState, IdmEgoObs, IdmEgoProblem, IdmEgoVars, check
from .sim import _need, _opt, _ptr, _stream

# Sec. IV-A initial values and boxes, in (v0, T, a, b, s0) order
PAPER_INIT = (50.0, 1.0, 10.0, 2.0, 5.0)
PAPER_BOXES = ((20.0, 60.0), (0.1, 5.0), (5.0, 10.0), (0.1, 5.0), (1.0, 10.0))
PAPER_GAP0, PAPER_DV0 = 10.0, 0.0


class EgoPlan:
    """Owns an idm_ego_plan (validated problem, graph of the fit step)."""

    def __init__(self, n_traj: int, n_steps: int, dt: float = 1.0, a_min: float = -10.0,
                 gap_floor: float = 1e-3, bound: int = BOUND_SOFTPLUS, ckpt_every: int = 0,
                 delta: float = 4.0):
        L = _lib.load()
        self._L = L
        self.n, self.n_steps, self.dt = int(n_traj), int(n_steps), float(dt)
        pb = IdmEgoProblem(self.n, self.n_steps, int(ckpt_every), self.dt, float(delta),
                           float(a_min), float(gap_floor), int(bound))
        h = ctypes.c_void_p()
        check(L.idm_ego_plan_create(ctypes.byref(pb), ctypes.byref(h)), "idm_ego_plan_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            self._L.idm_ego_plan_destroy(h)
            self.handle = None

    def workspace_bytes(self) -> int:
        return int(self._L.idm_ego_workspace_bytes(self.handle))

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(), 1), dtype=torch.uint8, device=device)


@dataclass
class EgoObs:
    """Observations, CSR by trajectory: offsets [N+1] int32, step [M] int32
    (nearest simulation step), pos [M] FP32 (p(0) = 0 frame)."""
    offsets: torch.Tensor
    step: torch.Tensor
    pos: torch.Tensor

    @property
    def n_obs(self) -> int:
        return int(self.pos.numel())

    def c(self) -> IdmEgoObs:
        return IdmEgoObs(self.offsets.data_ptr(), self.step.data_ptr(), self.pos.data_ptr(),
                         self.n_obs)


def match_steps(t: torch.Tensor, dt: float, n_steps: int, stream=None) -> torch.Tensor:
    """Nearest simulation step of every timestamp (FP64 seconds), clamped to [0, S]."""
    _need(t, "t", torch.float64, t.numel())
    out = torch.empty(t.numel(), dtype=torch.int32, device=t.device)
    check(_lib.load().idm_ego_match_steps(_ptr(t), int(t.numel()), float(dt), int(n_steps),
                                          _ptr(out), _stream(stream)), "idm_ego_match_steps")
    return out


def initial_speed(offsets: torch.Tensor, t: torch.Tensor, pos: torch.Tensor,
                  stream=None) -> torch.Tensor:
    n = offsets.numel() - 1
    _need(offsets, "offsets", torch.int32, n + 1)
    _need(t, "t", torch.float64, t.numel())
    _need(pos, "pos", torch.float32, t.numel())
    out = torch.empty(n, dtype=torch.float32, device=pos.device)
    check(_lib.load().idm_ego_initial_speed(_ptr(offsets), _ptr(t), _ptr(pos), int(n), _ptr(out),
                                            _stream(stream)), "idm_ego_initial_speed")
    return out


def _vars(plan: EgoPlan, params: torch.Tensor, gap: torch.Tensor, dv: torch.Tensor) -> IdmEgoVars:
    n, sn = plan.n, plan.n * plan.n_steps
    _need(params, "params", torch.float32, 5 * n)
    _need(gap, "gap", torch.float32, sn)
    _need(dv, "dv", torch.float32, sn)
    p = params.data_ptr()
    return IdmEgoVars(p, p + 4 * n, p + 8 * n, p + 12 * n, p + 16 * n, gap.data_ptr(), dv.data_ptr())


def idm_ego_forward(plan: EgoPlan, params, gap, dv, v_init, workspace, traj_p=None, traj_v=None,
                    traj_a=None, stream=None) -> None:
    """Positions / speeds [(S+1), N] and accelerations [S, N] (each nullable)."""
    n, S = plan.n, plan.n_steps
    x = _vars(plan, params, gap, dv)
    _need(v_init, "v_init", torch.float32, n)
    _need(workspace, "workspace", torch.uint8, workspace.numel())
    _opt(traj_p, "traj_p", torch.float32, (S + 1) * n)
    _opt(traj_v, "traj_v", torch.float32, (S + 1) * n)
    _opt(traj_a, "traj_a", torch.float32, S * n)
    check(plan._L.idm_ego_forward(plan.handle, ctypes.byref(x), _ptr(v_init), _ptr(traj_p),
                                  _ptr(traj_v), _ptr(traj_a), _ptr(workspace), _stream(stream)),
          "idm_ego_forward")


def idm_ego_backward(plan: EgoPlan, params, gap, dv, v_init, obs: EgoObs, grad_params, grad_gap,
                     grad_dv, workspace, grad_v0=None, loss_out=None, stream=None) -> None:
    """Gradients of the summed absolute error (after idm_ego_forward on the
    same workspace): grad_params [5, N] FP64, grad_gap / grad_dv [S, N] FP32,
    grad_v0 [N] FP64 and the loss (FP64) where given."""
    n, S = plan.n, plan.n_steps
    x = _vars(plan, params, gap, dv)
    _need(v_init, "v_init", torch.float32, n)
    _need(obs.offsets, "obs.offsets", torch.int32, n + 1)
    _need(obs.step, "obs.step", torch.int32, obs.n_obs)
    _need(obs.pos, "obs.pos", torch.float32, obs.n_obs)
    _need(grad_params, "grad_params", torch.float64, 5 * n)
    _need(grad_gap, "grad_gap", torch.float32, S * n)
    _need(grad_dv, "grad_dv", torch.float32, S * n)
    _opt(grad_v0, "grad_v0", torch.float64, n)
    _opt(loss_out, "loss_out", torch.float64, 1)
    oc = obs.c()
    check(plan._L.idm_ego_backward(plan.handle, ctypes.byref(x), _ptr(v_init), ctypes.byref(oc),
                                   _ptr(grad_params), _ptr(grad_gap), _ptr(grad_dv), _ptr(grad_v0),
                                   _ptr(loss_out), _ptr(workspace), _stream(stream)),
          "idm_ego_backward")


class EgoFitter:
    """Device state of idm_ego_fit_state and the fit loop."""

    def __init__(self, plan: EgoPlan, v_init: torch.Tensor, obs: EgoObs,
                 boxes: Sequence = PAPER_BOXES, lr0: float = 0.1, lr1: float = 0.01,
                 lr_steps: int = 500, hist_len: int = 4096, betas=(0.9, 0.999), eps: float = 1e-8):
        n, S = plan.n, plan.n_steps
        dev = v_init.device
        _need(v_init, "v_init", torch.float32, n)
        self.plan, self.v_init, self.obs = plan, v_init, obs
        self.params = torch.empty(5, n, dtype=torch.float32, device=dev)
        self.gap = torch.empty(S, n, dtype=torch.float32, device=dev)
        self.dv = torch.empty(S, n, dtype=torch.float32, device=dev)
        self.m = torch.empty(5 * n + 2 * S * n, dtype=torch.float32, device=dev)
        self.v = torch.empty_like(self.m)
        self.step_ctr = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss_hist = torch.zeros(int(hist_len), dtype=torch.float64, device=dev)
        self.workspace = plan.workspace(dev)
        st = IdmEgoFitState()
        st.params, st.gap, st.dv = self.params.data_ptr(), self.gap.data_ptr(), self.dv.data_ptr()
        st.m, st.v = self.m.data_ptr(), self.v.data_ptr()
        st.step, st.loss_hist, st.hist_len = self.step_ctr.data_ptr(), self.loss_hist.data_ptr(), int(hist_len)
        for i, (lo, hi) in enumerate(boxes):
            st.lo[i], st.hi[i] = float(lo), float(hi)
        st.lr0, st.lr1, st.lr_steps = float(lr0), float(lr1), int(max(1, lr_steps))
        st.beta1, st.beta2, st.eps = float(betas[0]), float(betas[1]), float(eps)
        self._st = st
        self._obs_c = obs.c()

    def init(self, params5: Sequence[float] = PAPER_INIT, gap0: float = PAPER_GAP0,
             dv0: float = PAPER_DV0, stream=None) -> None:
        arr = (ctypes.c_float * 5)(*[float(x) for x in params5])
        check(self.plan._L.idm_ego_fit_init(self.plan.handle, ctypes.byref(self._st),
                                            ctypes.byref(arr), float(gap0), float(dv0),
                                            _stream(stream)), "idm_ego_fit_init")

    def step(self, stream=None) -> None:
        check(self.plan._L.idm_ego_fit_step(self.plan.handle, ctypes.byref(self._st),
                                            _ptr(self.v_init), ctypes.byref(self._obs_c),
                                            _ptr(self.workspace), _stream(stream)),
              "idm_ego_fit_step")

    def run(self, n_iters: int, stream=None) -> None:
        check(self.plan._L.idm_ego_fit_run(self.plan.handle, ctypes.byref(self._st),
                                           _ptr(self.v_init), ctypes.byref(self._obs_c),
                                           int(n_iters), _ptr(self.workspace), _stream(stream)),
              "idm_ego_fit_run")

    def losses(self) -> torch.Tensor:
        k = int(self.step_ctr.item())
        return self.loss_hist[:min(k, self.loss_hist.numel())].cpu()


def reconstruction_metrics(traj_p: torch.Tensor, traj_a: torch.Tensor, obs: EgoObs) -> dict:
    """The paper's evaluation criteria of a reconstruction (Sec. V-B4),
    evaluated on the device from the forward's positions [(S+1), N] and
    accelerations [S, N]:
      pos_error: mean over observations of |observed - simulated position at the
        nearest step| / the trajectory's length (last minus first observation);
      acc_mean / acc_std: mean and standard deviation of |a| over every step
        inside each trajectory's observed span;
      implausible: fraction of trajectories with |a| > 10 m/s^2 at any such step.
    Evaluation only (not part of the fitted path)."""
    off = obs.offsets.long()
    n = off.numel() - 1
    counts = off[1:] - off[:-1]
    traj = torch.repeat_interleave(torch.arange(n, device=off.device), counts)
    step = obs.step.long()
    sim_p = traj_p[step, traj]
    first = obs.pos[off[:-1].clamp(max=max(obs.n_obs - 1, 0))]
    last = obs.pos[(off[1:] - 1).clamp(min=0)]
    length = (last - first).abs().clamp(min=1.0)
    rel = ((sim_p - obs.pos).abs() / length[traj]).double()
    # steps inside each trajectory's span: k < last observed step
    last_step = torch.zeros(n, dtype=torch.long, device=off.device)
    has = counts > 0
    last_step[has] = step[off[1:][has] - 1]
    S = traj_a.shape[0]
    inside = torch.arange(S, device=off.device)[:, None] < last_step[None, :]
    aa = traj_a.abs().double()
    sel = aa[inside]
    bad = ((aa > 10.0) & inside).any(dim=0)
    return {"pos_error": float(rel.mean().item()) if rel.numel() else 0.0,
            "acc_mean": float(sel.mean().item()) if sel.numel() else 0.0,
            "acc_std": float(sel.std(unbiased=False).item()) if sel.numel() else 0.0,
            "implausible": float(bad.double().mean().item())}
