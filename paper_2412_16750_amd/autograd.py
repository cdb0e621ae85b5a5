"""torch.autograd.Function around the hand-written adjoint.

``simulate(plan, params, p0, v_init, length)`` returns the FP32 displacement
trajectory d [S+1, N] (absolute positions are p0 + d).  Its backward calls
``idm_sim_backward`` with the incoming gradient as the dense upstream dL/dd,
and returns the gradients with respect to params [5, N] (v0, T, a, b, s0),
p0 [N] (through the gaps, Sec. III-A) and v_init [N].  Length is not
differentiated.  Each call allocates its own workspace (the checkpoints of
that forward), so several simulations may be in flight before backward.
"""
from __future__ import annotations

import torch

from . import sim


class IDMSimulate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, p0, v_init, plan, length):
        S, n = plan.n_steps, plan.n
        traj_d = torch.empty(S + 1, n, dtype=torch.float32, device=params.device)
        ws = plan.workspace(params.device)
        sim.idm_sim_forward(plan, params.detach(), length, p0.detach(), v_init.detach(), traj_d,
                            None, ws)
        ctx.plan = plan
        ctx.save_for_backward(params.detach(), p0.detach(), v_init.detach(), length, ws)
        return traj_d

    @staticmethod
    def backward(ctx, grad_d):
        params, p0, v_init, length, ws = ctx.saved_tensors
        plan = ctx.plan
        n = plan.n
        dev = params.device
        gd = grad_d.detach()
        if gd.dtype != torch.float32 or not gd.is_contiguous():
            gd = gd.to(torch.float32).contiguous()
        gp = torch.empty(5, n, dtype=torch.float64, device=dev)
        gp0 = torch.empty(n, dtype=torch.float64, device=dev)
        gv0 = torch.empty(n, dtype=torch.float64, device=dev)
        sim.idm_sim_backward(plan, params, length, p0, v_init, gp, gp0, gv0, ws, grad_traj_d=gd)
        return (gp.to(params.dtype) if ctx.needs_input_grad[0] else None,
                gp0.to(p0.dtype) if ctx.needs_input_grad[1] else None,
                gv0.to(v_init.dtype) if ctx.needs_input_grad[2] else None,
                None, None)


def simulate(plan: "sim.Plan", params: torch.Tensor, p0: torch.Tensor, v_init: torch.Tensor,
             length: torch.Tensor) -> torch.Tensor:
    """Differentiable forward simulation; returns d [S+1, N] (FP32)."""
    return IDMSimulate.apply(params, p0, v_init, plan, length)
