"""Training-free trajectory forecasting (Sec. V-C): fit every vehicle's IDM
parameters to a short observed history with the lane fit and roll the fitted
lanes out from the starting state.  The fit follows the paper's optimisation
(Sec. IV-A, Sec. V-B3): Adam on the parameters in their own units with the
learning rate falling linearly from 0.1 to 0.01, then projection onto the
boxes.

Argument marshalling and evaluation only: the fit and the rollout are the
library's fit graph and forward kernel.
"""
from __future__ import annotations

from typing import Sequence

import torch

from . import sim
from .fit import DEFAULT_BOXES, Fitter


def fit_and_rollout(plan_history: "sim.Plan", plan_rollout: "sim.Plan", length: torch.Tensor,
                    p0: torch.Tensor, v_init: torch.Tensor, obs: "sim.Obs",
                    init_params: torch.Tensor, iters: int = 500, lr0: float = 0.1,
                    lr1: float = 0.01, boxes: Sequence = DEFAULT_BOXES, raw_units: bool = True):
    """Fit on the history plan's steps, then simulate the rollout plan's steps
    from the same starting state; returns (params [5, N], displacements
    [(S_rollout + 1), N], fitter)."""
    f = Fitter(plan_history, length, p0, v_init, obs, boxes=boxes, lr0=lr0, lr1=lr1,
               lr_steps=iters, raw_units=raw_units)
    f.init(init_params)
    f.run(iters)
    traj = torch.empty(plan_rollout.n_steps + 1, plan_rollout.n, dtype=torch.float32,
                       device=p0.device)
    sim.idm_sim_forward(plan_rollout, f.params, length, p0, v_init, traj, None,
                        plan_rollout.forward_workspace(p0.device))
    return f.params, traj, f


def displacement_errors(traj_pred: torch.Tensor, traj_true: torch.Tensor, first: int, last: int,
                        miss_m: float = 3.6) -> dict:
    """1-D analogues of the forecasting metrics over frames first..last of two
    displacement trajectories from the same starting positions: ADE = mean
    abs error over vehicles and frames, FDE = mean abs error at the last
    frame, miss rate = fraction of vehicles whose last-frame error exceeds
    miss_m (the longitudinal 8 s threshold of the benchmark the paper uses).
    Evaluation only."""
    e = (traj_pred[first:last + 1].double() - traj_true[first:last + 1].double()).abs()
    return {"ade_m": float(e.mean().item()), "fde_m": float(e[-1].mean().item()),
            "miss_rate": float((e[-1] > miss_m).double().mean().item())}
