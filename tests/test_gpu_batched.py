"""Many independent lanes of uneven length in one launch: bundle packing,
persistent grid, HIP-graph replay of forward + backward, and the autotuner."""
import numpy as np
import pytest

import oracle
import scenarios
from _util import grad_close, oracle_reference, pos_close
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _uneven(n_lanes, hi, S, K=16, c=31):
    sizes = scenarios.lognormal_lane_sizes(n_lanes, 4.0, 1.2, 1, hi, 5000 + c)
    sc = scenarios.make_scenario("uneven_small", scenarios.offsets_from_sizes(sizes), S, c,
                                 ckpt_every=K)
    return sc


def _buffers(sc, steps, tgt, **plan_kw):
    import torch
    from paper_2412_16750_amd import sim
    plan = sim.Plan.for_scenario(sc, **plan_kw)
    x = device_inputs(sc)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), int(steps[0]), int(steps[1] - steps[0]))
    b = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d=traj, obs=obs)
    return plan, b


def _snapshot(b):
    return [t.clone() for t in (b.traj_d, b.grad_params, b.grad_p0, b.grad_v0, b.loss)]


def test_uneven_lanes_graph_replay_and_parity():
    import torch
    from paper_2412_16750_amd import sim
    sc = _uneven(300, 600, 120)
    steps = np.arange(2, sc.n_steps + 1, 2)
    P2, _, _, _ = oracle.forward(oracle.Problem.from_scenario(sc, params=scenarios.second_params(sc, 31)))
    tgt = (P2[steps] + scenarios.noise((len(steps), sc.n), 31)).astype(np.float32)
    plan, b = _buffers(sc, steps, tgt, grid=200)
    info = plan.info()
    log("uneven: N=%d lanes=%d plan %s" % (sc.n, sc.n_lanes, info))
    assert info["grid"] == min(200, info["n_bundles"])
    b.run_eager()
    torch.cuda.synchronize()
    eager = _snapshot(b)
    for rep in range(3):
        for t in (b.traj_d, b.grad_params, b.grad_p0, b.grad_v0, b.loss):
            t.zero_()
        sim.idm_step_graph_launch(b)
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").square().sum()
        torch.cuda.synchronize()
        for a, e in zip(_snapshot(b), eager):
            assert torch.equal(a, e), rep
        del junk
    ref = oracle_reference(sc, steps, tgt)
    d = eager[0].cpu().numpy()
    ok, err, w = pos_close(sc.p0[None, :] + d.astype(np.float64), ref["P"])
    log("uneven: positions max|err| %.3e worst/limit %.3f" % (err, w))
    assert ok
    okg, wg = grad_close(eager[1].cpu().numpy(), ref["g"])
    ok0, w0 = grad_close(eager[2].cpu().numpy(), ref["gp0"])
    ok1, w1 = grad_close(eager[3].cpu().numpy(), ref["gv0"])
    log("uneven: gradient worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1
    assert abs(eager[4].item() - ref["loss"]) <= 1e-4 * ref["loss"]


def test_autotuner_keeps_results():
    """The autotuner times launch shapes on the real inputs and keeps the
    fastest; with the checkpoint interval fixed the trajectory and gradients
    are bitwise those of the default shape."""
    import torch
    from paper_2412_16750_amd import sim
    sc = _uneven(400, 1024, 64, K=16, c=32)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = scenarios.constant_speed_targets(sc, steps, 32)
    plan, b = _buffers(sc, steps, tgt)
    b.run_eager()
    torch.cuda.synchronize()
    before = _snapshot(b)
    info = sim.idm_plan_autotune(b, reps=2)
    log("autotuner chose %s" % info)
    assert info["ckpt_every"] == 16 and info["threads"] * info["per_thread"] >= info["max_lane"]
    b.run_eager()
    torch.cuda.synchronize()
    after = _snapshot(b)
    for a, e in zip(after[:4], before[:4]):
        assert torch.equal(a, e)
    assert abs(after[4].item() - before[4].item()) <= 1e-12 * before[4].item()
    sim.idm_step_graph_launch(b)
    torch.cuda.synchronize()
    assert torch.equal(b.grad_params, before[1])


@pytest.mark.parametrize("shape", [{}, {"ckpt_every": 16, "grid": 256}])
def test_uneven_workload_full_size_sampled_lanes(shape):
    """The 10,000-lane workload (lognormal(5, 1.2) sizes clipped to [10, 4096],
    about 3.0M vehicles, 300 steps) as one graph, in the default plan (K = 32,
    one work-group per bundle) and in the shape the autotuner picks for it on
    the benchmark (K = 16, a persistent grid of 256 work-groups); 8 lanes
    (including the longest) are recomputed by the oracle."""
    import torch
    from paper_2412_16750_amd import sim
    sc = scenarios.uneven()
    sizes = np.diff(sc.lane_offsets)
    log("uneven full: N=%d lanes=%d max lane %d, shape %s" % (sc.n, sc.n_lanes, sizes.max(), shape))
    steps = np.arange(10, sc.n_steps + 1, 10)
    tgt = scenarios.constant_speed_targets(sc, steps, 3)
    plan, b = _buffers(sc, steps, tgt, **shape)
    log("uneven full: plan %s" % plan.info())
    sim.idm_step_graph_launch(b)
    torch.cuda.synchronize()
    lanes = [int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 1, 4999, 7777, 9998, 9999]
    sub = scenarios.subset_lanes(sc, lanes)
    idx = sub.extra["vehicle_index"]
    ref = oracle_reference(sub, steps, tgt[:, idx])
    fac = sub.n / sc.n  # the MSE is normalised over all N vehicles
    it = torch.from_numpy(idx).cuda()
    d = b.traj_d[:, it].cpu().numpy()
    ok, err, w = pos_close(sc.p0[idx][None, :] + d.astype(np.float64), ref["P"])
    log("uneven full: positions max|err| %.3e worst/limit %.3f" % (err, w))
    assert ok
    okg, wg = grad_close(b.grad_params[:, it].cpu().numpy(), ref["g"] * fac)
    ok0, w0 = grad_close(b.grad_p0[it].cpu().numpy(), ref["gp0"] * fac)
    ok1, w1 = grad_close(b.grad_v0[it].cpu().numpy(), ref["gv0"] * fac)
    log("uneven full: gradient worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1


def test_autotuner_chooses_k_and_caches_the_choice():
    """With the checkpoint interval left free the autotuner also picks K (KB
    or 2 KB of each candidate's backward block) from the shapes whose
    workspace fits: the tuned plan's trajectory is bitwise the default's (the
    forward does not depend on K), its gradients match the oracle and the
    default's to within the FP32 block sums' regrouping; a second plan for the
    same problem takes the cached shape without timing."""
    import torch
    from paper_2412_16750_amd import sim
    sc = _uneven(400, 1024, 64, K=0, c=33)
    steps = np.arange(1, sc.n_steps + 1)
    P2, _, _, _ = oracle.forward(oracle.Problem.from_scenario(sc, params=scenarios.second_params(sc, 33)))
    tgt = (P2[steps] + scenarios.noise((len(steps), sc.n), 33)).astype(np.float32)
    # room for the shortest checkpoint interval a candidate can take (K = 8)
    room = sim.Plan.for_scenario(sc, ckpt_every=8, threads=1024, per_thread=1).workspace_bytes
    plan, b = _buffers(sc, steps, tgt)
    b = sim.StepBuffers(plan, b.params, b.length, b.p0, b.v_init, traj_d=b.traj_d, obs=b.obs,
                        workspace_bytes=room)
    default = plan.info()
    b.run_eager()
    torch.cuda.synchronize()
    before = _snapshot(b)
    info = sim.idm_plan_autotune(b, reps=2)
    log("autotuner, free K: default %s -> chose %s" % (default, info))
    assert info["autotune_cached"] == 0
    assert info["ckpt_every"] in (8, 16, 32, 64) and info["ckpt_every"] % info["block"] == 0
    b.run_eager()
    torch.cuda.synchronize()
    after = _snapshot(b)
    assert torch.equal(after[0], before[0])
    ref = oracle_reference(sc, steps, tgt)
    for name, a_, e_, r_ in (("params", after[1], before[1], ref["g"]),
                             ("p0", after[2], before[2], ref["gp0"]),
                             ("v0", after[3], before[3], ref["gv0"])):
        ok, w = grad_close(a_.cpu().numpy(), r_)
        rel = float((a_ - e_).abs().max() / e_.abs().max())
        log("autotuned K=%d: %s gradient worst/limit %.3f vs oracle, max |diff| / max |g| %.2e "
            "vs the default K" % (info["ckpt_every"], name, w, rel))
        assert ok and rel <= 1e-5
    assert abs(after[4].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    # a second plan for the same problem: the cached choice, no timing
    plan2, b2 = _buffers(sc, steps, tgt)
    b2 = sim.StepBuffers(plan2, b2.params, b2.length, b2.p0, b2.v_init, traj_d=b2.traj_d,
                         obs=b2.obs, workspace_bytes=room)
    info2 = sim.idm_plan_autotune(b2, reps=2)
    log("autotuner, second plan: %s" % info2)
    assert info2["autotune_cached"] == 1
    keep = ("threads", "per_thread", "ckpt_every", "block", "grid", "n_bundles")
    assert {k: info2[k] for k in keep} == {k: info[k] for k in keep}
    b2.run_eager()
    torch.cuda.synchronize()
    assert torch.equal(b2.grad_params, after[1]) and torch.equal(b2.traj_d, after[0])
