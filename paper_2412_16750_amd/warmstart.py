"""Learned warm start for the trajectory fit.

A 150 -> 256 -> 256 -> 5 MLP (BF16 MFMA kernels, FP32 accumulation, FP32
master weights) maps a vehicle's observed trajectory window to normalised
IDM parameters.  It is trained on (window, parameters) pairs that the
simulator generates, and its predictions initialise the Adam fit of
Sec. IV-A; per lane the fit falls back to the cold start when that gives the
lower observed loss.  Every numeric step (simulation, observation, features,
MLP, per-lane losses and choice, fit) runs in libidmx.so's kernels; torch
holds the buffers and the stream, and shuffles the training rows.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib, sim
from ._lib import MLP_IN_PAD, MLP_OUT, MLP_OUT_PAD, IdmMlpSchedule, IdmMlpState, IdmObs, check
from .fit import DEFAULT_BOXES, Fitter


class MLP:
    """Device state of the warm-start network (idm_mlp_state)."""

    def __init__(self, init_params: np.ndarray, lr: float = 1e-3, betas=(0.9, 0.999),
                 eps: float = 1e-8, device="cuda"):
        L = _lib.load()
        n_p, n_w = int(L.idm_mlp_param_count()), int(L.idm_mlp_weight_bf16_count())
        init_params = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        if init_params.size != n_p:
            raise ValueError("init_params has %d values, expected %d" % (init_params.size, n_p))
        self.params = torch.from_numpy(init_params).to(device)
        self.w16 = torch.empty(n_w, dtype=torch.bfloat16, device=device)
        self.m = torch.zeros(n_p, dtype=torch.float32, device=device)
        self.v = torch.zeros(n_p, dtype=torch.float32, device=device)
        st = IdmMlpState()
        st.params, st.weights_bf16 = self.params.data_ptr(), self.w16.data_ptr()
        st.adam_m, st.adam_v = self.m.data_ptr(), self.v.data_ptr()
        st.lr, st.beta1, st.beta2, st.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        self._st = st
        self.t = 0
        self._ws = {}
        check(L.idm_mlp_sync(ctypes.byref(st), sim._stream()), "idm_mlp_sync")

    def workspace(self, batch: int) -> torch.Tensor:
        if batch not in self._ws:
            nb = int(_lib.load().idm_mlp_workspace_bytes(int(batch)))
            self._ws = {batch: torch.empty(nb, dtype=torch.uint8, device=self.params.device)}
        return self._ws[batch]

    @staticmethod
    def _rows(X, U=None):
        B = X.shape[0]
        sim._need(X, "X", torch.bfloat16, B * MLP_IN_PAD)
        if U is not None:
            sim._need(U, "U", torch.float32, B * MLP_OUT)
        return B

    def forward(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None) -> torch.Tensor:
        B = self._rows(X)
        if Y is None:
            Y = torch.empty(B, MLP_OUT_PAD, dtype=torch.float32, device=X.device)
        sim._need(Y, "Y", torch.float32, B * MLP_OUT_PAD)
        check(_lib.load().idm_mlp_forward(ctypes.byref(self._st), sim._ptr(X), B, sim._ptr(Y),
                                          None, sim._stream()),
              "idm_mlp_forward")
        return Y

    def gradients(self, X, U, grad_out, loss_out=None):
        B = self._rows(X, U)
        sim._need(grad_out, "grad_out", torch.float32, self.params.numel())
        check(_lib.load().idm_mlp_gradients(ctypes.byref(self._st), sim._ptr(X), sim._ptr(U), B,
                                            sim._ptr(grad_out), sim._ptr(loss_out),
                                            sim._ptr(self.workspace(B)), sim._stream()),
              "idm_mlp_gradients")

    def train_step(self, X, U, loss_out=None):
        B = self._rows(X, U)
        self.t += 1
        check(_lib.load().idm_mlp_train_step(ctypes.byref(self._st), sim._ptr(X), sim._ptr(U), B,
                                             self.t, sim._ptr(loss_out),
                                             sim._ptr(self.workspace(B)), sim._stream()),
              "idm_mlp_train_step")


class ScheduledTrainer:
    """Device-side state of a training loop whose steps are all the same call
    (idm_mlp_train_step_scheduled): step counter, learning-rate cosine, the
    epoch's row permutation and fixed batch buffers.  `step()` runs one step
    eagerly; `capture()` records one step in a HIP graph, which `replay()`
    launches (the counter, the rate and the batch rows advance on the device,
    so every replay is the next step)."""

    def __init__(self, mlp: "MLP", data: "Dataset", batch: int, total_steps: int,
                 lr_final: Optional[float] = None):
        dev = data.X.device
        n = int(data.X.shape[0])
        if batch > n:
            raise ValueError("batch larger than the data")
        self.mlp, self.data, self.batch = mlp, data, int(batch)
        self.n_batches = n // self.batch
        self.perm = torch.arange(n, dtype=torch.int64, device=dev)
        self.Xb = torch.empty(self.batch, MLP_IN_PAD, dtype=torch.bfloat16, device=dev)
        self.Ub = torch.empty(self.batch, MLP_OUT, dtype=torch.float32, device=dev)
        self.counter = torch.zeros(1, dtype=torch.int32, device=dev)
        self.loss_hist = torch.zeros(max(self.n_batches, 1), dtype=torch.float64, device=dev)
        self.ws = torch.empty(int(_lib.load().idm_mlp_workspace_bytes(self.batch)),
                              dtype=torch.uint8, device=dev)
        sc = IdmMlpSchedule()
        sc.step, sc.loss_hist = self.counter.data_ptr(), self.loss_hist.data_ptr()
        sc.lr0 = float(mlp._st.lr)
        sc.lr_final = float(mlp._st.lr if lr_final is None else lr_final)
        sc.total_steps = int(max(1, total_steps))
        sc.hist_len = int(self.loss_hist.numel())
        self._sc = sc
        self.graph = None
        self.graph_steps = 0

    def set_permutation(self, perm: torch.Tensor, non_blocking: bool = False) -> None:
        """Rows of the next epoch, copied into the fixed permutation buffer in
        stream order (after the steps already launched)."""
        self.perm.copy_(perm, non_blocking=non_blocking)

    def step(self) -> None:
        check(_lib.load().idm_mlp_train_step_scheduled(
            ctypes.byref(self.mlp._st), sim._ptr(self.data.X), sim._ptr(self.data.U),
            int(self.data.X.shape[0]), sim._ptr(self.perm), self.batch, ctypes.byref(self._sc),
            sim._ptr(self.Xb), sim._ptr(self.Ub), sim._ptr(self.ws), sim._stream()),
            "idm_mlp_train_step_scheduled")

    def capture(self, steps: int = 1) -> None:
        """Record `steps` consecutive steps in one graph (every step is the
        same call; the state that advances lives on the device)."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(int(steps)):
                self.step()
        self.graph = g
        self.graph_steps = int(steps)

    def replay(self) -> None:
        """Launch the captured graph: its `graph_steps` steps."""
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def steps_done(self) -> int:
        return int(self.counter.item())


def train_graph(mlp: "MLP", data: "Dataset", batch: int = 4096, epochs: int = 10, seed: int = 0,
                log=None, lr_final: Optional[float] = None) -> dict:
    """The minibatch Adam loop of `train` as one HIP graph launch per epoch:
    the graph holds the epoch's steps (each the same captured call), a fresh
    row permutation per epoch (the same generator and seed as `train`), the
    learning-rate cosine and the step counter on the device.  The next epoch's
    permutation is drawn on the host while the GPU runs the current one and
    copied in stream order from pinned memory; the epoch losses (mean of the
    steps' losses) are read once at the end."""
    n = data.X.shape[0]
    nb = n // batch
    tr = ScheduledTrainer(mlp, data, batch, max(epochs * nb, 1), lr_final)
    g = torch.Generator(device="cpu").manual_seed(seed)
    dev = data.X.device
    # two pinned host buffers for the permutations, each guarded by the event
    # recorded after its last copy
    pinned = [torch.empty(n, dtype=torch.int64, pin_memory=True) for _ in range(2)]
    copied = [None, None]
    ep_loss = torch.zeros(max(epochs, 1), dtype=torch.float64, device=dev)
    tr.capture(nb)  # records one epoch of steps; nothing runs yet
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = torch.randperm(n, generator=g)
    for ep in range(epochs):
        buf = pinned[ep & 1]
        if copied[ep & 1] is not None:
            copied[ep & 1].synchronize()
        buf.copy_(nxt)
        tr.set_permutation(buf, non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        copied[ep & 1] = ev
        tr.replay()
        ep_loss[ep] = tr.loss_hist[:nb].mean()
        if ep + 1 < epochs:
            nxt = torch.randperm(n, generator=g)  # overlaps the epoch on the GPU
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    losses = ep_loss.cpu().tolist()
    hist = [{"epoch": ep, "train_mse": losses[ep]} for ep in range(epochs)]
    if log:
        for rec in hist:
            log("mlp epoch %d: %s" % (rec["epoch"], rec))
    mlp.t = tr.steps_done()
    return {"history": hist, "seconds": secs, "steps": epochs * nb}


def observe(plan, traj_d, p0, noise, obs_first, obs_stride, n_obs) -> torch.Tensor:
    """Observed absolute positions [n_obs, N] from a simulated trajectory."""
    n = plan.n
    sim._need(traj_d, "traj_d", torch.float32, (plan.n_steps + 1) * n)
    sim._need(p0, "p0", torch.float64, n)
    if noise is not None:
        sim._need(noise, "noise", torch.float32, n_obs * n)
    out = torch.empty(n_obs, n, dtype=torch.float32, device=p0.device)
    check(_lib.load().idm_observe(plan.handle, sim._ptr(traj_d), sim._ptr(p0), sim._ptr(noise),
                                  int(n_obs), int(obs_first), int(obs_stride), sim._ptr(out),
                                  sim._stream()), "idm_observe")
    return out


def features(plan, obs: "sim.Obs", p0, length, X: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Window features [N, 160] (BF16) of every vehicle (into X if given)."""
    n = plan.n
    sim._need(obs.target, "obs.target", torch.float32, obs.n_obs * n)
    if X is None:
        X = torch.empty(n, MLP_IN_PAD, dtype=torch.bfloat16, device=p0.device)
    sim._need(X, "X", torch.bfloat16, n * MLP_IN_PAD)
    check(_lib.load().idm_mlp_features(plan.handle, sim._ptr(obs.target), obs.n_obs, obs.obs_first,
                                       obs.obs_stride, sim._ptr(p0), sim._ptr(length), sim._ptr(X),
                                       sim._stream()), "idm_mlp_features")
    return X


def lane_loss(plan, traj_d, p0, obs: "sim.Obs") -> torch.Tensor:
    out = torch.empty(plan.n_lanes, dtype=torch.float64, device=p0.device)
    oc = obs.c()
    check(_lib.load().idm_lane_loss(plan.handle, sim._ptr(traj_d), sim._ptr(p0), ctypes.byref(oc),
                                    sim._ptr(out), sim._stream()), "idm_lane_loss")
    return out


def select_by_lane(plan, loss_a, loss_b, params_a, params_b):
    out = torch.empty_like(params_a)
    chose = torch.empty(plan.n, dtype=torch.int32, device=params_a.device)
    check(_lib.load().idm_select_by_lane(plan.handle, sim._ptr(loss_a), sim._ptr(loss_b),
                                         sim._ptr(params_a), sim._ptr(params_b), sim._ptr(out),
                                         sim._ptr(chose), sim._stream()), "idm_select_by_lane")
    return out, chose


@dataclass
class Dataset:
    X: torch.Tensor   # [N, 160] BF16 features
    U: torch.Tensor   # [N, 5] FP32 normalised true parameters


def make_pairs(sc, dev="cuda") -> Dataset:
    """Simulate the scenario with its own (true) parameters, observe every
    obs_stride-th step with N(0, 0.5 m) noise, and return (features, u) pairs."""
    import scenarios
    plan = sim.Plan.for_scenario(sc)
    prm = sim.params_tensor(sc.params, dev)
    length = torch.from_numpy(np.ascontiguousarray(sc.params["length"])).to(dev)
    p0 = torch.from_numpy(np.ascontiguousarray(sc.p0)).to(dev)
    v = torch.from_numpy(np.ascontiguousarray(sc.v_init)).to(dev)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device=dev)
    sim.idm_sim_forward(plan, prm, length, p0, v, traj, None, plan.forward_workspace(dev))
    first, stride = int(sc.extra["obs_first"]), int(sc.extra["obs_stride"])
    n_obs = (sc.n_steps - first) // stride + 1
    noise = torch.from_numpy(scenarios.noise((n_obs, sc.n), 5).astype(np.float32)).to(dev)
    tgt = observe(plan, traj, p0, noise, first, stride, n_obs)
    del traj
    X = features(plan, sim.Obs(tgt, first, stride), p0, length)
    U = torch.from_numpy(scenarios.normalized_params(sc.params)).to(dev)
    torch.cuda.synchronize()
    return Dataset(X, U)


def train(mlp: MLP, data: Dataset, batch: int = 4096, epochs: int = 10, seed: int = 0,
          val: Optional[Dataset] = None, log=None, lr_final: Optional[float] = None) -> dict:
    """Minibatch Adam over shuffled rows; returns per-epoch losses and time.
    With `lr_final`, the learning rate follows a cosine from the network's
    initial rate to `lr_final` over all steps; otherwise it stays constant."""
    n = data.X.shape[0]
    nb = n // batch
    g = torch.Generator(device="cpu").manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device=data.X.device)
    hist = []
    lr0, total, step = mlp._st.lr, max(epochs * nb, 1), 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(data.X.device)
        Xs, Us = data.X.index_select(0, perm), data.U.index_select(0, perm)
        acc = torch.zeros(1, dtype=torch.float64, device=data.X.device)
        for b in range(nb):
            if lr_final is not None:
                mlp._st.lr = lr_final + 0.5 * (lr0 - lr_final) * (1.0 + math.cos(math.pi * step / total))
            step += 1
            mlp.train_step(Xs[b * batch:(b + 1) * batch], Us[b * batch:(b + 1) * batch], loss)
            acc += loss
        torch.cuda.synchronize()
        ep_loss = float(acc.item()) / max(nb, 1)
        rec = {"epoch": ep, "train_mse": ep_loss}
        if val is not None:
            rec["val_mse"] = evaluate(mlp, val)
        hist.append(rec)
        if log:
            log("mlp epoch %d: %s" % (ep, rec))
    torch.cuda.synchronize()
    return {"history": hist, "seconds": time.perf_counter() - t0, "steps": epochs * nb}


def evaluate(mlp: MLP, data: Dataset) -> float:
    """Mean squared error of the predicted normalised parameters."""
    Y = mlp.forward(data.X)
    return float(((Y[:, :MLP_OUT] - data.U) ** 2).mean().item())


def warm_init(fitter: Fitter, mlp: MLP, plan, obs, p0, v_init, length, cold_params,
              fallback: bool = True) -> dict:
    """Initialise the fit from the MLP's predictions; with the fallback, lanes
    whose observed loss is lower at the cold start keep the cold start."""
    X = features(plan, obs, p0, length)
    Y = mlp.forward(X)
    check(_lib.load().idm_fit_init_normalized(plan.handle, ctypes.byref(fitter._st), sim._ptr(Y),
                                              MLP_OUT_PAD, sim._stream()), "idm_fit_init_normalized")
    info = {"fallback_lanes": 0}
    if fallback:
        warm = fitter.params.clone()
        traj = torch.empty(plan.n_steps + 1, plan.n, dtype=torch.float32, device=p0.device)
        sim.idm_sim_forward(plan, warm, length, p0, v_init, traj, None, fitter.workspace)
        la = lane_loss(plan, traj, p0, obs)
        sim.idm_sim_forward(plan, cold_params, length, p0, v_init, traj, None, fitter.workspace)
        lb = lane_loss(plan, traj, p0, obs)
        chosen, chose_a = select_by_lane(plan, la, lb, warm, cold_params)
        fitter.init(chosen)
        info["fallback_lanes"] = int((la > lb).sum().item())
    return info


def trajectory_rmse(plan, params, length, p0, v_init, hidden_traj, traj_buf) -> float:
    """RMSE (m) of the simulated trajectory under `params` against the hidden
    trajectory, over every vehicle and steps 1..S (evaluation only)."""
    sim.idm_sim_forward(plan, params, length, p0, v_init, traj_buf, None,
                        plan.forward_workspace(p0.device))
    d = (traj_buf[1:] - hidden_traj[1:]).double()
    return float(torch.sqrt((d * d).mean()).item())


def fit_until(fitter: Fitter, plan, length, p0, v_init, hidden_traj, target_rmse: float = 0.5,
              chunk: int = 10, cap: int = 2000) -> dict:
    """Run the fit in graph replays of `chunk` iterations until the RMSE
    against the hidden trajectory reaches `target_rmse` (or `cap`
    iterations).  Only the fitting is timed (HIP events), not the checks."""
    traj = torch.empty_like(hidden_traj)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fit_ms, it = 0.0, 0
    rmse = trajectory_rmse(plan, fitter.params, length, p0, v_init, hidden_traj, traj)
    curve = [(0, rmse)]
    while rmse > target_rmse and it < cap:
        e0.record()
        fitter.run(chunk)
        e1.record()
        torch.cuda.synchronize()
        fit_ms += e0.elapsed_time(e1)
        it += chunk
        rmse = trajectory_rmse(plan, fitter.params, length, p0, v_init, hidden_traj, traj)
        curve.append((it, rmse))
    return {"iterations": it, "fit_seconds": fit_ms / 1e3, "rmse": rmse,
            "reached": rmse <= target_rmse, "curve": curve}
