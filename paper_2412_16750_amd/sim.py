"""Python binding of the C ABI with the same entry-point names.

Every function here checks shapes, dtypes, devices and contiguity on the host
(the C ABI receives raw device pointers and cannot), then forwards the call.
No arithmetic of the method happens in Python: the simulation, the loss and
the gradient all run in libidmx.so's HIP kernels.  torch provides the device
memory and the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import (BOUND_CLAMP, BOUND_SOFTPLUS, IdmFitState, IdmObs, IdmParams, IdmPlanInfo,
                   IdmProblem, IdmStepArgs, IdmTuning, check)

PARAM_NAMES = ("v0", "T", "a", "b", "s0")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, numel: int):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on a HIP device, got %s" % (name, t.device))
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), numel))


def _opt(t, name, dtype, numel):
    if t is not None:
        _need(t, name, dtype, numel)


@dataclass
class Obs:
    """Observed absolute positions target[n_obs, N] (FP32) at steps
    obs_first + j * obs_stride."""
    target: torch.Tensor
    obs_first: int
    obs_stride: int

    @property
    def n_obs(self) -> int:
        return int(self.target.shape[0])

    def c(self) -> IdmObs:
        return IdmObs(self.target.data_ptr(), self.n_obs, int(self.obs_first), int(self.obs_stride))


class Plan:
    """Owns an idm_plan: the validated problem and its work-group bundles."""

    def __init__(self, lane_offsets, n_steps: int, dt: float = 0.1, a_min: float = -10.0,
                 gap_floor: float = 1e-3, bound: int = BOUND_SOFTPLUS, ckpt_every: int = 0,
                 delta: float = 4.0, threads: int = 0, per_thread: int = 0, grid: int = 0,
                 tuning_k: int = 0, block: int = 0, store_states=False, tile_steps: int = 0):
        L = _lib.load()
        self._L = L
        self.offsets = np.ascontiguousarray(np.asarray(lane_offsets, dtype=np.int32))
        self.n = int(self.offsets[-1])
        self.n_lanes = len(self.offsets) - 1
        self.n_steps = int(n_steps)
        self.bound = int(bound)
        pb = IdmProblem(self.n, self.n_lanes, self.n_steps, int(ckpt_every), float(dt), float(delta),
                        float(a_min), float(gap_floor), self.bound,
                        self.offsets.ctypes.data_as(ctypes.c_void_p))
        # store_states: False / True, or "auto" (the autotuner weighs both
        # backwards, and halo tiles); tile_steps > 0: halo tiles advancing that
        # many steps per launch (with store_states=True and explicit threads)
        st = 2 if store_states == "auto" else int(bool(store_states))
        tu = IdmTuning(int(threads), int(per_thread), int(tuning_k), int(grid), int(block), st,
                       int(tile_steps))
        h = ctypes.c_void_p()
        check(L.idm_plan_create(ctypes.byref(pb), ctypes.byref(tu), ctypes.byref(h)), "idm_plan_create")
        self.handle = h

    @classmethod
    def for_scenario(cls, sc, **kw):
        kw.setdefault("ckpt_every", sc.ckpt_every)
        return cls(sc.lane_offsets, sc.n_steps, sc.dt, sc.a_min, sc.gap_floor, sc.mode,
                   delta=sc.delta, **kw)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self._L.idm_plan_destroy(h)
            self.handle = None

    @property
    def workspace_bytes(self) -> int:
        return int(self._L.idm_workspace_bytes(self.handle))

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes, 1), dtype=torch.uint8, device=device)

    def forward_workspace(self, device="cuda") -> Optional[torch.Tensor]:
        """A workspace for forward-only calls: None unless lanes longer than a
        bundle exchange boundary states through it, or halo tiles keep their
        states in it (then one buffer, kept by the plan and reused)."""
        info = self.info()
        if info["n_boundaries"] == 0 and info["tile_steps"] == 0:
            return None
        ws = getattr(self, "_fws", None)
        if ws is None or ws.device != torch.device(device):
            ws = self._fws = self.workspace(device)
        return ws

    def info(self) -> dict:
        o = IdmPlanInfo()
        check(self._L.idm_plan_get_info(self.handle, ctypes.byref(o)), "idm_plan_get_info")
        return {k: getattr(o, k) for k, _ in IdmPlanInfo._fields_}


def _params_c(plan: Plan, prm: torch.Tensor, length: torch.Tensor) -> IdmParams:
    n = plan.n
    _need(prm, "params", torch.float32, 5 * n)
    _need(length, "length", torch.float32, n)
    base = prm.data_ptr()
    return IdmParams(base, base + 4 * n, base + 8 * n, base + 12 * n, base + 16 * n, length.data_ptr())


def _check_ws(plan: Plan, ws: Optional[torch.Tensor], required: bool):
    if ws is None:
        if required:
            raise ValueError("workspace is required")
        return
    if ws.device.type != "cuda" or ws.numel() * ws.element_size() < plan.workspace_bytes:
        raise ValueError("workspace must be a device buffer of at least %d bytes" % plan.workspace_bytes)


def idm_sim_forward(plan: Plan, params: torch.Tensor, length: torch.Tensor, p0: torch.Tensor,
                    v_init: torch.Tensor, traj_d: Optional[torch.Tensor] = None,
                    traj_v: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                    stream=None) -> None:
    """params: [5, N] FP32 (v0, T, a, b, s0); length, v_init: [N] FP32; p0: [N] FP64;
    traj_d / traj_v: [(S+1), N] FP32 outputs (optional)."""
    n, S = plan.n, plan.n_steps
    prm = _params_c(plan, params, length)
    _need(p0, "p0", torch.float64, n)
    _need(v_init, "v_init", torch.float32, n)
    _opt(traj_d, "traj_d", torch.float32, (S + 1) * n)
    _opt(traj_v, "traj_v", torch.float32, (S + 1) * n)
    _check_ws(plan, workspace, False)
    check(plan._L.idm_sim_forward(plan.handle, ctypes.byref(prm), _ptr(p0), _ptr(v_init), _ptr(traj_d),
                                  _ptr(traj_v), _ptr(workspace), _stream(stream)), "idm_sim_forward")


def idm_sim_backward(plan: Plan, params: torch.Tensor, length: torch.Tensor, p0: torch.Tensor,
                     v_init: torch.Tensor, grad_params: torch.Tensor, grad_p0: torch.Tensor,
                     grad_v0: torch.Tensor, workspace: torch.Tensor,
                     grad_traj_d: Optional[torch.Tensor] = None,
                     grad_traj_v: Optional[torch.Tensor] = None, obs: Optional[Obs] = None,
                     loss_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """Gradient of the loss (dense upstream and/or fused MSE) w.r.t. params [5, N],
    p0 [N] and v_init [N], all written in FP64."""
    n, S = plan.n, plan.n_steps
    prm = _params_c(plan, params, length)
    _need(p0, "p0", torch.float64, n)
    _need(v_init, "v_init", torch.float32, n)
    _need(grad_params, "grad_params", torch.float64, 5 * n)
    _need(grad_p0, "grad_p0", torch.float64, n)
    _need(grad_v0, "grad_v0", torch.float64, n)
    _opt(grad_traj_d, "grad_traj_d", torch.float32, (S + 1) * n)
    _opt(grad_traj_v, "grad_traj_v", torch.float32, (S + 1) * n)
    _opt(loss_out, "loss_out", torch.float64, 1)
    _check_ws(plan, workspace, True)
    oc = None
    if obs is not None:
        _need(obs.target, "obs.target", torch.float32, obs.n_obs * n)
        oc = ctypes.byref(obs.c())
    check(plan._L.idm_sim_backward(plan.handle, ctypes.byref(prm), _ptr(p0), _ptr(v_init),
                                   _ptr(grad_traj_d), _ptr(grad_traj_v), oc, _ptr(grad_params),
                                   _ptr(grad_p0), _ptr(grad_v0), _ptr(loss_out), _ptr(workspace),
                                   _stream(stream)), "idm_sim_backward")


def idm_sim_backward_stored(plan: Plan, params: torch.Tensor, length: torch.Tensor,
                            p0: torch.Tensor, traj_d: torch.Tensor, traj_v: torch.Tensor,
                            grad_params: torch.Tensor, grad_p0: torch.Tensor,
                            grad_v0: torch.Tensor, workspace: torch.Tensor,
                            grad_traj_d: Optional[torch.Tensor] = None,
                            grad_traj_v: Optional[torch.Tensor] = None, obs: Optional[Obs] = None,
                            loss_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """idm_sim_backward from the forward's stored trajectory: traj_d and
    traj_v [S+1, N] as idm_sim_forward wrote them (read, not recomputed)."""
    n, S = plan.n, plan.n_steps
    prm = _params_c(plan, params, length)
    _need(p0, "p0", torch.float64, n)
    _need(traj_d, "traj_d", torch.float32, (S + 1) * n)
    _need(traj_v, "traj_v", torch.float32, (S + 1) * n)
    _need(grad_params, "grad_params", torch.float64, 5 * n)
    _need(grad_p0, "grad_p0", torch.float64, n)
    _need(grad_v0, "grad_v0", torch.float64, n)
    _opt(grad_traj_d, "grad_traj_d", torch.float32, (S + 1) * n)
    _opt(grad_traj_v, "grad_traj_v", torch.float32, (S + 1) * n)
    _opt(loss_out, "loss_out", torch.float64, 1)
    _check_ws(plan, workspace, True)
    oc = None
    if obs is not None:
        _need(obs.target, "obs.target", torch.float32, obs.n_obs * n)
        oc = ctypes.byref(obs.c())
    check(plan._L.idm_sim_backward_stored(plan.handle, ctypes.byref(prm), _ptr(p0), _ptr(traj_d),
                                          _ptr(traj_v), _ptr(grad_traj_d), _ptr(grad_traj_v), oc,
                                          _ptr(grad_params), _ptr(grad_p0), _ptr(grad_v0),
                                          _ptr(loss_out), _ptr(workspace), _stream(stream)),
          "idm_sim_backward_stored")


def idm_sim_backward_noalloc(plan: Plan, params: torch.Tensor, length: torch.Tensor,
                             p0: torch.Tensor, v_init: torch.Tensor, grad_params: torch.Tensor,
                             grad_p0: torch.Tensor, grad_v0: torch.Tensor,
                             grad_traj_d: Optional[torch.Tensor] = None,
                             grad_traj_v: Optional[torch.Tensor] = None, obs: Optional[Obs] = None,
                             loss_out: Optional[torch.Tensor] = None, stream=None) -> None:
    """idm_sim_backward with no workspace: the library runs the forward
    (checkpoints) and the backward in its static device scratch array."""
    n, S = plan.n, plan.n_steps
    prm = _params_c(plan, params, length)
    _need(p0, "p0", torch.float64, n)
    _need(v_init, "v_init", torch.float32, n)
    _need(grad_params, "grad_params", torch.float64, 5 * n)
    _need(grad_p0, "grad_p0", torch.float64, n)
    _need(grad_v0, "grad_v0", torch.float64, n)
    _opt(grad_traj_d, "grad_traj_d", torch.float32, (S + 1) * n)
    _opt(grad_traj_v, "grad_traj_v", torch.float32, (S + 1) * n)
    _opt(loss_out, "loss_out", torch.float64, 1)
    oc = None
    if obs is not None:
        _need(obs.target, "obs.target", torch.float32, obs.n_obs * n)
        oc = ctypes.byref(obs.c())
    check(plan._L.idm_sim_backward_noalloc(plan.handle, ctypes.byref(prm), _ptr(p0), _ptr(v_init),
                                           _ptr(grad_traj_d), _ptr(grad_traj_v), oc,
                                           _ptr(grad_params), _ptr(grad_p0), _ptr(grad_v0),
                                           _ptr(loss_out), _stream(stream)),
          "idm_sim_backward_noalloc")


def idm_plan_diagnostics(plan: Plan, workspace: torch.Tensor, out: Optional[torch.Tensor] = None,
                         stream=None) -> torch.Tensor:
    """Anomaly counts of the last forward that wrote `workspace`: a device int64
    tensor [gap-floor evaluations, vehicles with a non-finite state]."""
    _check_ws(plan, workspace, True)
    if out is None:
        out = torch.empty(2, dtype=torch.int64, device=workspace.device)
    _need(out, "out", torch.int64, 2)
    check(plan._L.idm_plan_diagnostics(plan.handle, _ptr(workspace), _ptr(out), _stream(stream)),
          "idm_plan_diagnostics")
    return out


class StepBuffers:
    """Device buffers of one forward + backward pass (used by the graph launch,
    the autotuner and the benchmark)."""

    def __init__(self, plan: Plan, params, length, p0, v_init, traj_d=None, traj_v=None,
                 grad_traj_d=None, grad_traj_v=None, obs: Optional[Obs] = None, device="cuda",
                 workspace_bytes: int = 0):
        """workspace_bytes: room beyond the plan's own need (the autotuner
        only times shapes whose workspace fits, e.g. shorter checkpoint
        intervals when K is left free)."""
        n = plan.n
        self.plan = plan
        self.params, self.length, self.p0, self.v_init = params, length, p0, v_init
        self.traj_d, self.traj_v = traj_d, traj_v
        self.grad_traj_d, self.grad_traj_v = grad_traj_d, grad_traj_v
        self.obs = obs
        self.grad_params = torch.empty(5, n, dtype=torch.float64, device=device)
        self.grad_p0 = torch.empty(n, dtype=torch.float64, device=device)
        self.grad_v0 = torch.empty(n, dtype=torch.float64, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.workspace = torch.empty(max(plan.workspace_bytes, int(workspace_bytes), 1),
                                     dtype=torch.uint8, device=device)
        self._validate()

    def _validate(self):
        p, n, S = self.plan, self.plan.n, self.plan.n_steps
        _params_c(p, self.params, self.length)
        _need(self.p0, "p0", torch.float64, n)
        _need(self.v_init, "v_init", torch.float32, n)
        _opt(self.traj_d, "traj_d", torch.float32, (S + 1) * n)
        _opt(self.traj_v, "traj_v", torch.float32, (S + 1) * n)
        _opt(self.grad_traj_d, "grad_traj_d", torch.float32, (S + 1) * n)
        _opt(self.grad_traj_v, "grad_traj_v", torch.float32, (S + 1) * n)
        if self.obs is not None:
            _need(self.obs.target, "obs.target", torch.float32, self.obs.n_obs * n)
        _check_ws(p, self.workspace, True)

    def args(self) -> IdmStepArgs:
        self._validate()
        a = IdmStepArgs()
        a.prm = _params_c(self.plan, self.params, self.length)
        a.p0 = self.p0.data_ptr()
        a.v_init = self.v_init.data_ptr()
        a.traj_d = self.traj_d.data_ptr() if self.traj_d is not None else None
        a.traj_v = self.traj_v.data_ptr() if self.traj_v is not None else None
        a.grad_traj_d = self.grad_traj_d.data_ptr() if self.grad_traj_d is not None else None
        a.grad_traj_v = self.grad_traj_v.data_ptr() if self.grad_traj_v is not None else None
        if self.obs is not None:
            a.obs_target = self.obs.target.data_ptr()
            a.n_obs, a.obs_first, a.obs_stride = self.obs.n_obs, self.obs.obs_first, self.obs.obs_stride
        else:
            a.obs_target = None
            a.n_obs, a.obs_first, a.obs_stride = 0, 0, 1
        a.grad_params = self.grad_params.data_ptr()
        a.grad_p0 = self.grad_p0.data_ptr()
        a.grad_v0 = self.grad_v0.data_ptr()
        a.loss_out = self.loss.data_ptr()
        a.workspace = self.workspace.data_ptr()
        return a

    def run_eager(self, stream=None):
        idm_sim_forward(self.plan, self.params, self.length, self.p0, self.v_init, self.traj_d,
                        self.traj_v, self.workspace, stream)
        idm_sim_backward(self.plan, self.params, self.length, self.p0, self.v_init, self.grad_params,
                         self.grad_p0, self.grad_v0, self.workspace, self.grad_traj_d,
                         self.grad_traj_v, self.obs, self.loss, stream)

    def realloc_workspace(self):
        if self.workspace.numel() < self.plan.workspace_bytes:
            self.workspace = self.plan.workspace(self.p0.device)


def idm_step_graph_launch(bufs: StepBuffers, stream=None) -> None:
    """Forward + backward as one HIP graph replay (captured on first use)."""
    a = bufs.args()
    check(bufs.plan._L.idm_step_graph_launch(bufs.plan.handle, ctypes.byref(a), _stream(stream)),
          "idm_step_graph_launch")


def idm_plan_autotune(bufs: StepBuffers, reps: int = 3, stream=None) -> dict:
    """Time every launch shape on these buffers and keep the fastest."""
    a = bufs.args()
    ws_bytes = bufs.workspace.numel()
    check(bufs.plan._L.idm_plan_autotune(bufs.plan.handle, ctypes.byref(a), ws_bytes, int(reps),
                                         _stream(stream)), "idm_plan_autotune")
    bufs.realloc_workspace()
    return bufs.plan.info()


def params_tensor(params: dict, device="cuda") -> torch.Tensor:
    """Stack (v0, T, a, b, s0) float32 arrays into a [5, N] device tensor."""
    return torch.from_numpy(np.stack([np.asarray(params[k], dtype=np.float32) for k in PARAM_NAMES])).to(device)


def idm_copy_bytes(dst: torch.Tensor, src: torch.Tensor, stream=None) -> None:
    """Streaming device copy of src into dst (same byte size, 16-byte multiple)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb or src.device.type != "cuda" or dst.device.type != "cuda":
        raise ValueError("idm_copy_bytes: device tensors of equal byte size required")
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("idm_copy_bytes: contiguous tensors required")
    check(_lib.load().idm_copy_bytes(_ptr(dst), _ptr(src), nb, _stream(stream)), "idm_copy_bytes")
