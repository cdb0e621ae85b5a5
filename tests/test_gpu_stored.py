"""The backward from the forward's stored trajectory (idm_sim_backward_stored).

It performs the checkpointed backward's arithmetic in the same order and
flushes the FP32 gradient sums at the same K-step block boundaries, so for the
same plan its gradients and loss must equal idm_sim_backward's bit for bit;
beside that, parity with the FP64 oracle at the tolerances of the other
parity tests (positions 1e-4 relative, gradients 1e-3 of each kind's scale).
"""
import numpy as np
import pytest

import scenarios
from scenarios import MODE_CLAMP, MODE_SOFTPLUS

from _util import grad_close, oracle_reference, oracle_targets, ragged_scenario
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _both(sc, steps=None, target=None, dense=None, **plan_kw):
    """Forward with the whole trajectory, then the checkpointed and the
    stored-state backward on the same plan and workspace."""
    import torch
    from paper_2412_16750_amd import sim
    dev = "cuda"
    plan = sim.Plan.for_scenario(sc, **plan_kw)
    x = device_inputs(sc, dev)
    S, n = sc.n_steps, sc.n
    traj_d = torch.empty(S + 1, n, dtype=torch.float32, device=dev)
    traj_v = torch.empty(S + 1, n, dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d, traj_v, ws)
    obs = None
    if target is not None:
        steps = np.asarray(steps)
        stride = int(steps[1] - steps[0]) if len(steps) > 1 else 1
        obs = sim.Obs(torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).to(dev),
                      int(steps[0]), stride)
    gd = None if dense is None else torch.from_numpy(
        np.ascontiguousarray(dense, dtype=np.float32)).to(dev)
    out = {"info": plan.info()}
    for tag in ("ckpt", "stored"):
        gp = torch.full((5, n), float("nan"), dtype=torch.float64, device=dev)
        gp0 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        gv0 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
        loss = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
        if tag == "ckpt":
            sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, gp0, gv0, ws,
                                 grad_traj_d=gd, obs=obs, loss_out=loss)
        else:
            sim.idm_sim_backward_stored(plan, x["prm"], x["length"], x["p0"], traj_d, traj_v,
                                        gp, gp0, gv0, ws, grad_traj_d=gd, obs=obs, loss_out=loss)
        torch.cuda.synchronize()
        out[tag] = dict(g=gp.cpu().numpy(), gp0=gp0.cpu().numpy(), gv0=gv0.cpu().numpy(),
                        loss=float(loss.item()))
    out["P"] = sc.p0[None, :] + traj_d.cpu().numpy().astype(np.float64)
    return out


def _same(out, what):
    a, b = out["ckpt"], out["stored"]
    for k in ("g", "gp0", "gv0"):
        assert np.array_equal(a[k], b[k]), (what, k, np.nanmax(np.abs(a[k] - b[k])))
    assert a["loss"] == b["loss"], (what, a["loss"], b["loss"])


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
@pytest.mark.parametrize("shape", [(1024, 1, 32), (256, 1, 16), (128, 2, 16), (64, 4, 8),
                                   (128, 1, 24), (512, 2, 32)])
def test_stored_backward_bitwise_equals_checkpointed(mode, shape):
    """Lanes of 1..256 vehicles, S = 203 (a ragged last K-step block), fused
    MSE on every 5th step plus a dense upstream gradient; every launch shape
    and K, in both bound modes, and the oracle on the stored result."""
    threads, per, K = shape
    sizes = [1, 2, 3, 63, 64, 65, 100, 127, 31, 256, 0, 17, 200, 5, 90]
    sizes = [s for s in sizes if s <= threads * per]
    sc = ragged_scenario(sizes, 203, mode=mode, ckpt_every=K)
    steps = np.arange(3, sc.n_steps + 1, 5)
    tgt = oracle_targets(sc, steps, c=3)
    dense = np.random.default_rng(11).normal(0, 1e-3, size=(sc.n_steps + 1, sc.n)).astype(
        np.float32)
    out = _both(sc, steps, tgt, dense, threads=threads, per_thread=per, tuning_k=K)
    assert out["info"]["ckpt_every"] == K
    _same(out, "shape %s mode %d" % (shape, mode))
    ref = oracle_reference(sc, steps, tgt, dense)
    s = out["stored"]
    okg, wg = grad_close(s["g"], ref["g"])
    ok0, w0 = grad_close(s["gp0"], ref["gp0"])
    ok1, w1 = grad_close(s["gv0"], ref["gv0"])
    log("stored shape %s mode %d: gradient worst/limit params %.3f p0 %.3f v0 %.3f" %
        (shape, mode, wg, w0, w1))
    assert okg and ok0 and ok1
    assert abs(s["loss"] - ref["loss"]) <= 1e-4 * ref["loss"]


@pytest.mark.parametrize("dense_only", [False, True])
def test_stored_backward_targets_only_and_dense_only(dense_only):
    """The kernel without dense inputs (fused MSE on every step) and with a
    dense upstream only (no targets, loss 0)."""
    sizes = [1000, 24, 512, 3]
    sc = ragged_scenario(sizes, 100, ckpt_every=32)
    if dense_only:
        dense = scenarios.noise((sc.n_steps + 1, sc.n), 17, sigma=1e-2).astype(np.float32)
        out = _both(sc, dense=dense)
        assert out["stored"]["loss"] == 0.0
    else:
        steps = np.arange(1, sc.n_steps + 1)
        out = _both(sc, steps, oracle_targets(sc, steps, c=17))
    log("stored %s: plan %s" % ("dense" if dense_only else "targets", out["info"]))
    _same(out, "dense only" if dense_only else "targets only")


def test_stored_backward_edge_steps():
    """S = 0 (the seed alone), S = 1 and S = 2 (the two-step read-ahead runs
    past step 0), a single vehicle, and K larger than S."""
    for sizes, S, K in (([1], 0, 8), ([3, 1], 0, 8), ([1], 1, 8), ([5, 2], 2, 8), ([1], 400, 16),
                        ([7, 40], 37, 64), ([9], 3, 8)):
        sc = ragged_scenario(sizes, S, ckpt_every=K)
        dense = scenarios.noise((S + 1, sc.n), 5, sigma=1.0).astype(np.float32)
        if S > 0:
            steps = np.arange(1, S + 1)
            out = _both(sc, steps, oracle_targets(sc, steps, c=5), dense, tuning_k=K)
        else:
            out = _both(sc, dense=dense, tuning_k=K)
        _same(out, "sizes %s S %d K %d" % (sizes, S, K))
        if S == 0:
            assert np.all(out["stored"]["g"] == 0.0) and np.all(out["stored"]["gv0"] == 0.0)


def test_stored_backward_rejects_lane_pieces():
    """A lane longer than a bundle is cut into pieces run in several launches;
    the stored-state kernel covers whole lanes only and says so."""
    import torch
    from paper_2412_16750_amd import _lib, sim
    sc = ragged_scenario([150, 20], 10, ckpt_every=8)
    plan = sim.Plan.for_scenario(sc, threads=64, per_thread=1)
    assert plan.info()["n_boundaries"] > 0
    x = device_inputs(sc)
    n, S = sc.n, sc.n_steps
    traj_d = torch.empty(S + 1, n, device="cuda")
    traj_v = torch.empty(S + 1, n, device="cuda")
    ws = plan.workspace()
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d, traj_v, ws)
    gp = torch.empty(5, n, dtype=torch.float64, device="cuda")
    g1 = torch.empty(n, dtype=torch.float64, device="cuda")
    g2 = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.IdmError) as e:
        sim.idm_sim_backward_stored(plan, x["prm"], x["length"], x["p0"], traj_d, traj_v, gp, g1,
                                    g2, ws, grad_traj_d=torch.zeros(S + 1, n, device="cuda"))
    assert "pieces" in str(e.value)


def test_stored_backward_scale_workload_bitwise():
    """The 2000 x 1000 = 2M-vehicle, 100-step workload in the benchmark's
    launch shape (1024 x 1, K = 32): the stored-state gradients equal the
    checkpointed ones element for element (the checkpointed path's own oracle
    parity on this workload is tested on sampled lanes elsewhere)."""
    sc = scenarios.scale()
    steps = np.arange(1, sc.n_steps + 1)
    tgt = scenarios.constant_speed_targets(sc, steps, 2)
    out = _both(sc, steps, tgt)
    log("stored scale: plan %s, loss %.9e" % (out["info"], out["stored"]["loss"]))
    assert (out["info"]["threads"], out["info"]["per_thread"], out["info"]["ckpt_every"]) == \
        (1024, 1, 32)
    _same(out, "scale")


def _plans(sc, **kw):
    from paper_2412_16750_amd import sim
    return (sim.Plan.for_scenario(sc, **kw), sim.Plan.for_scenario(sc, store_states=True, **kw))


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_stored_plan_forward_backward_bitwise(mode):
    """A plan that keeps every step's states (idm_tuning.store_states): its
    forward writes them into the workspace and copies them to the caller's
    trajectory buffers, its idm_sim_backward reads them; trajectories,
    gradients, loss and diagnostics equal the checkpointed plan's."""
    import torch
    from paper_2412_16750_amd import sim
    sc = ragged_scenario([1, 2, 3, 63, 64, 65, 100, 127, 31, 256, 0, 17, 200, 5, 90], 203,
                         mode=mode, ckpt_every=16)
    steps = np.arange(3, sc.n_steps + 1, 5)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=3)).cuda()
    obs = sim.Obs(tgt, 3, 5)
    x = device_inputs(sc)
    S, n = sc.n_steps, sc.n
    res = []
    for plan in _plans(sc, threads=256, per_thread=1):
        d = torch.empty(S + 1, n, device="cuda")
        v = torch.empty(S + 1, n, device="cuda")
        ws = plan.workspace()
        sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], d, v, ws)
        gp = torch.empty(5, n, dtype=torch.float64, device="cuda")
        g0 = torch.empty(n, dtype=torch.float64, device="cuda")
        g1 = torch.empty(n, dtype=torch.float64, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, g0, g1, ws, obs=obs,
                             loss_out=loss)
        diag = sim.idm_plan_diagnostics(plan, ws).cpu().numpy().tolist()
        torch.cuda.synchronize()
        res.append([t.cpu().numpy() for t in (d, v, gp, g0, g1, loss)] + [diag, plan.info()])
    assert res[0][-1]["store_states"] == 0 and res[1][-1]["store_states"] == 1
    log("stored plan: workspace %d vs %d bytes" % (_plans(sc, threads=256, per_thread=1)[0]
                                                   .workspace_bytes,
                                                   _plans(sc, threads=256, per_thread=1)[1]
                                                   .workspace_bytes))
    for i, name in enumerate(("d", "v", "g", "gp0", "gv0", "loss", "diag")):
        if name == "diag":
            assert res[0][i] == res[1][i]
        else:
            assert np.array_equal(res[0][i], res[1][i]), name


def test_stored_plan_fit_graph_and_noalloc():
    """Eight fit steps (one captured graph) and the no-allocation gradient on
    a plan that keeps every step's states equal the checkpointed plan's."""
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd.fit import Fitter
    sc = ragged_scenario([300, 40, 7, 512], 120, ckpt_every=32)
    steps = np.arange(10, sc.n_steps + 1, 10)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=12)).cuda()
    obs = sim.Obs(tgt, 10, 10)
    x = device_inputs(sc)
    cold = sim.params_tensor(scenarios.cold_params(sc))
    outs = []
    for plan in _plans(sc):
        f = Fitter(plan, x["length"], x["p0"], x["v"], obs, lr0=1e-2)
        f.init(cold)
        f.run(8)
        torch.cuda.synchronize()
        n = sc.n
        gp = torch.empty(5, n, dtype=torch.float64, device="cuda")
        g0 = torch.empty(n, dtype=torch.float64, device="cuda")
        g1 = torch.empty(n, dtype=torch.float64, device="cuda")
        sim.idm_sim_backward_noalloc(plan, x["prm"], x["length"], x["p0"], x["v"], gp, g0, g1,
                                     obs=obs)
        torch.cuda.synchronize()
        outs.append((f.losses().copy(), f.params.cpu().numpy(), gp.cpu().numpy(),
                     g0.cpu().numpy(), g1.cpu().numpy()))
    log("stored plan fit: losses %s" % outs[1][0])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_stored_plan_step_graph_autotune_and_autograd():
    """The step graph (forward + backward replayed), the autotuner (it keeps
    the plan's mode and tunes the launch shape) and autograd.simulate on a
    plan that keeps every step's states."""
    import torch
    from paper_2412_16750_amd import autograd, sim
    sc = ragged_scenario([64, 33, 100, 1, 200, 128], 90, ckpt_every=16)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=13)).cuda()
    obs = sim.Obs(tgt, 1, 1)
    x = device_inputs(sc)
    ck, st = _plans(sc)
    res = []
    for plan in (ck, st):
        b = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                            workspace_bytes=4 * plan.workspace_bytes)
        sim.idm_step_graph_launch(b)
        sim.idm_step_graph_launch(b)
        torch.cuda.synchronize()
        res.append((b.grad_params.cpu().numpy(), b.grad_p0.cpu().numpy(), b.loss.item()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    assert res[0][2] == res[1][2]
    b = sim.StepBuffers(st, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                        workspace_bytes=4 * st.workspace_bytes)
    info = sim.idm_plan_autotune(b, reps=1)
    log("stored plan autotuned: %s" % info)
    assert info["store_states"] == 1 and info["ckpt_every"] == 16
    sim.idm_step_graph_launch(b)
    torch.cuda.synchronize()
    assert np.array_equal(b.grad_params.cpu().numpy(), res[0][0])
    grads = []
    for plan in (ck, st):
        prm = x["prm"].clone().requires_grad_(True)
        d = autograd.simulate(plan, prm, x["p0"], x["v"], x["length"])
        (d[-1].double() ** 2).sum().backward()
        grads.append(prm.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])


def test_autotuner_weighs_both_backwards():
    """store_states = 2: the plan starts with checkpoints and idm_plan_autotune
    times both backwards, the kept states only when the workspace it is given
    holds them; with K fixed every choice gives the checkpointed plan's
    gradients bit for bit, and the choice is cached per problem."""
    import torch
    from paper_2412_16750_amd import sim
    sc = ragged_scenario([400, 300, 500, 20], 400, ckpt_every=32)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=21)).cuda()
    obs = sim.Obs(tgt, 1, 1)
    x = device_inputs(sc)
    ref_plan = sim.Plan.for_scenario(sc)
    ref = sim.StepBuffers(ref_plan, x["prm"], x["length"], x["p0"], x["v"], obs=obs)
    sim.idm_step_graph_launch(ref)
    room = sim.Plan.for_scenario(sc, store_states=True).workspace_bytes
    # no room for the states: checkpoints stay
    auto = sim.Plan.for_scenario(sc, store_states="auto")
    assert auto.info()["store_states"] == 0
    b = sim.StepBuffers(auto, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                        workspace_bytes=auto.workspace_bytes)
    info = sim.idm_plan_autotune(b, reps=2)
    assert info["store_states"] == 0
    # room for them: the faster of the two
    auto2 = sim.Plan.for_scenario(sc, store_states="auto", tuning_k=32)
    b2 = sim.StepBuffers(auto2, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                         workspace_bytes=room)
    info2 = sim.idm_plan_autotune(b2, reps=2)
    log("autotune with room for the states: %s" % info2)
    sim.idm_step_graph_launch(b2)
    torch.cuda.synchronize()
    assert np.array_equal(b2.grad_params.cpu().numpy(), ref.grad_params.cpu().numpy())
    assert np.array_equal(b2.grad_v0.cpu().numpy(), ref.grad_v0.cpu().numpy())
    # the same problem again: the cached choice
    auto3 = sim.Plan.for_scenario(sc, store_states="auto", tuning_k=32)
    b3 = sim.StepBuffers(auto3, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                         workspace_bytes=room)
    info3 = sim.idm_plan_autotune(b3, reps=2)
    assert info3["autotune_cached"] == 1 and info3["store_states"] == info2["store_states"]
    sim.idm_step_graph_launch(b3)
    torch.cuda.synchronize()
    assert np.array_equal(b3.grad_params.cpu().numpy(), ref.grad_params.cpu().numpy())


def test_stored_plan_graph_with_trajectory_outputs():
    """A plan that keeps every step's states, captured as a step graph that
    also hands the trajectory to the caller (device-to-device copies out of
    the workspace inside the graph): three replays, each after eager work of
    the program's own, each equal to the eager forward + backward."""
    import torch
    from paper_2412_16750_amd import sim
    sc = ragged_scenario([64, 200, 1, 90], 150, ckpt_every=16)
    steps = np.arange(2, sc.n_steps + 1, 2)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=23)).cuda()
    obs = sim.Obs(tgt, 2, 2)
    x = device_inputs(sc)
    S, n = sc.n_steps, sc.n
    plan = sim.Plan.for_scenario(sc, store_states=True)
    # eager reference on the same plan
    d0 = torch.empty(S + 1, n, device="cuda")
    v0 = torch.empty(S + 1, n, device="cuda")
    ws0 = plan.workspace()
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], d0, v0, ws0)
    g0 = torch.empty(5, n, dtype=torch.float64, device="cuda")
    a0 = torch.empty(n, dtype=torch.float64, device="cuda")
    b0 = torch.empty(n, dtype=torch.float64, device="cuda")
    sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], g0, a0, b0, ws0, obs=obs)
    torch.cuda.synchronize()
    d = torch.full((S + 1, n), float("nan"), device="cuda")
    v = torch.full((S + 1, n), float("nan"), device="cuda")
    b = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d=d, traj_v=v, obs=obs)
    other = torch.empty(S + 1, n, device="cuda")
    for rep in range(3):
        d.fill_(float("nan"))
        v.fill_(float("nan"))
        b.grad_params.zero_()
        sim.idm_step_graph_launch(b)
        torch.cuda.synchronize()
        assert torch.equal(d, d0) and torch.equal(v, v0), rep
        assert torch.equal(b.grad_params, g0) and torch.equal(b.grad_p0, a0), rep
        assert torch.equal(b.grad_v0, b0), rep
        # the program's own eager work between replays
        sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], other, None, None)
        torch.cuda.synchronize()


@pytest.mark.parametrize("seed", range(8))
def test_random_stored_backward_bitwise(seed):
    """Random lane mixes, launch shapes (1, 2 or 4 vehicles per thread), K,
    step counts, observation schedules, bound modes and upstream kinds: the
    backward from stored states equals the checkpointed one bit for bit."""
    rng = np.random.default_rng(500 + seed)
    threads = int(rng.choice([64, 128, 256, 512, 1024]))
    per = int(rng.choice([1, 2, 4]))
    K = int(rng.choice([8, 16] if per == 4 else [8, 16, 32]))
    cap = threads * per
    n = int(rng.integers(2, 30))
    sizes = rng.integers(1, cap + 1, n)
    S = int(rng.integers(1, 120))
    first = int(rng.integers(1, min(S, 6) + 1))
    stride = int(rng.integers(1, 8))
    steps = np.arange(first, S + 1, stride)
    mode = int(rng.integers(0, 2))
    sc = ragged_scenario(sizes, S, mode=mode, seed_c=90 + seed, ckpt_every=K)
    tgt = oracle_targets(sc, steps, c=90 + seed)
    dense = None
    if rng.integers(0, 2):
        dense = np.random.default_rng(seed).normal(0, 1e-3, (S + 1, sc.n)).astype(np.float32)
    out = _both(sc, steps, tgt, dense, threads=threads, per_thread=per, tuning_k=K)
    log("random stored seed %d: %d x %d, K %d, S %d, obs %d:%d, mode %d, dense %s"
        % (seed, threads, per, K, S, first, stride, mode, dense is not None))
    _same(out, "seed %d" % seed)
