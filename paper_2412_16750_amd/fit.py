"""Trajectory fitting (Sec. IV-A): per-vehicle IDM parameters fitted to
observed positions by Adam with box constraints, every step on the device.

``Fitter`` owns the device state of idm_fit_state (normalised parameters u,
Adam moments, physical parameters, step counter, loss history) and drives
``idm_fit_init`` / ``idm_fit_step`` / ``idm_fit_run`` (the latter replays one
captured fit step as a HIP graph).
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib, sim
from ._lib import IdmFitState, check

PARAM_NAMES = ("v0", "T", "a", "b", "s0")
# Box per parameter kind (v0, T, a, b, s0) for normalised fitting.
DEFAULT_BOXES = ((15.0, 45.0), (0.5, 3.0), (0.5, 3.0), (0.5, 4.0), (0.5, 5.0))


class Fitter:
    def __init__(self, plan: "sim.Plan", length: torch.Tensor, p0: torch.Tensor,
                 v_init: torch.Tensor, obs: "sim.Obs", boxes: Sequence = DEFAULT_BOXES,
                 lr0: float = 1e-2, lr1: Optional[float] = None, lr_steps: int = 1,
                 hist_len: int = 4096, betas=(0.9, 0.999), eps: float = 1e-8,
                 raw_units: bool = False):
        n = plan.n
        dev = p0.device
        sim._need(length, "length", torch.float32, n)
        sim._need(p0, "p0", torch.float64, n)
        sim._need(v_init, "v_init", torch.float32, n)
        sim._need(obs.target, "obs.target", torch.float32, obs.n_obs * n)
        self.plan, self.length, self.p0, self.v_init, self.obs = plan, length, p0, v_init, obs
        self.u = torch.empty(5, n, dtype=torch.float32, device=dev)
        self.m = torch.empty_like(self.u)
        self.v = torch.empty_like(self.u)
        self.params = torch.empty_like(self.u)
        self.step_ctr = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss_hist = torch.zeros(int(hist_len), dtype=torch.float64, device=dev)
        self.workspace = plan.workspace(dev)
        st = IdmFitState()
        st.u, st.m, st.v = self.u.data_ptr(), self.m.data_ptr(), self.v.data_ptr()
        st.params = self.params.data_ptr()
        st.length = length.data_ptr()
        st.step = self.step_ctr.data_ptr()
        st.loss_hist = self.loss_hist.data_ptr()
        st.hist_len = int(hist_len)
        for i, (lo, hi) in enumerate(boxes):
            st.lo[i], st.hi[i] = float(lo), float(hi)
        st.lr0 = float(lr0)
        st.lr1 = float(lr0 if lr1 is None else lr1)
        st.lr_steps = int(max(1, lr_steps))
        st.beta1, st.beta2, st.eps = float(betas[0]), float(betas[1]), float(eps)
        st.raw_units = 1 if raw_units else 0
        self._st = st
        self._obs_c = obs.c()
        self.boxes = np.asarray(boxes, dtype=np.float64)

    def init(self, params: torch.Tensor, stream=None) -> None:
        """Start from physical parameters [5, N] (FP32, device)."""
        sim._need(params, "params", torch.float32, 5 * self.plan.n)
        check(_lib.load().idm_fit_init(self.plan.handle, ctypes.byref(self._st),
                                       sim._ptr(params), sim._stream(stream)), "idm_fit_init")

    def step(self, stream=None) -> None:
        """One eager fit step (forward, fused loss, backward, Adam)."""
        check(_lib.load().idm_fit_step(self.plan.handle, ctypes.byref(self._st), sim._ptr(self.p0),
                                       sim._ptr(self.v_init), ctypes.byref(self._obs_c),
                                       sim._ptr(self.workspace), sim._stream(stream)),
              "idm_fit_step")

    def run(self, n_iters: int, stream=None) -> None:
        """n_iters fit steps as replays of one captured HIP graph."""
        check(_lib.load().idm_fit_run(self.plan.handle, ctypes.byref(self._st), sim._ptr(self.p0),
                                      sim._ptr(self.v_init), ctypes.byref(self._obs_c),
                                      int(n_iters), sim._ptr(self.workspace), sim._stream(stream)),
              "idm_fit_run")

    def steps_done(self) -> int:
        return int(self.step_ctr.item())

    def losses(self) -> np.ndarray:
        k = min(self.steps_done(), self.loss_hist.numel())
        return self.loss_hist[:k].cpu().numpy()
