"""Run the HIP path (through the C ABI) on a scenario; used by the GPU tests."""
from __future__ import annotations

import sys

import numpy as np


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def device_inputs(sc, dev="cuda"):
    import torch
    from paper_2412_16750_amd import sim
    return dict(prm=sim.params_tensor(sc.params, dev),
                length=torch.from_numpy(np.ascontiguousarray(sc.params["length"])).to(dev),
                p0=torch.from_numpy(np.ascontiguousarray(sc.p0)).to(dev),
                v=torch.from_numpy(np.ascontiguousarray(sc.v_init)).to(dev))


def gpu_run(sc, steps=None, target=None, dense=None, want_traj=True, want_v=True,
            want_backward=True, **plan_kw):
    """Forward (+ backward with the fused MSE on `target` at `steps` and/or a
    dense upstream gradient) through idm_sim_forward / idm_sim_backward."""
    import torch
    from paper_2412_16750_amd import sim
    dev = "cuda"
    plan = sim.Plan.for_scenario(sc, **plan_kw)
    x = device_inputs(sc, dev)
    S, n = sc.n_steps, sc.n
    traj_d = torch.empty(S + 1, n, dtype=torch.float32, device=dev) if want_traj else None
    traj_v = torch.empty(S + 1, n, dtype=torch.float32, device=dev) if want_v else None
    ws = plan.workspace(dev)
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d, traj_v, ws)
    diag = sim.idm_plan_diagnostics(plan, ws)
    out = dict(info=plan.info(), diag=diag.cpu().numpy().tolist())
    if want_backward:
        obs = None
        if target is not None:
            steps = np.asarray(steps)
            stride = int(steps[1] - steps[0]) if len(steps) > 1 else 1
            assert np.all(np.diff(steps) == stride)
            obs = sim.Obs(torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).to(dev),
                          int(steps[0]), stride)
        gd = None if dense is None else torch.from_numpy(
            np.ascontiguousarray(dense, dtype=np.float32)).to(dev)
        gp = torch.empty(5, n, dtype=torch.float64, device=dev)
        gp0 = torch.empty(n, dtype=torch.float64, device=dev)
        gv0 = torch.empty(n, dtype=torch.float64, device=dev)
        loss = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
        sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, gp0, gv0, ws,
                             grad_traj_d=gd, obs=obs, loss_out=loss)
        torch.cuda.synchronize()
        out.update(g=gp.cpu().numpy(), gp0=gp0.cpu().numpy(), gv0=gv0.cpu().numpy(),
                   loss=float(loss.item()))
    torch.cuda.synchronize()
    if traj_d is not None:
        out["d"] = traj_d.cpu().numpy()
        out["P"] = sc.p0[None, :] + out["d"].astype(np.float64)
    if traj_v is not None:
        out["V"] = traj_v.cpu().numpy()
    return out
