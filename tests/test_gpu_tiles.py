"""Halo tiles: lanes cut across several work-groups, steps run in blocks of J.

A step moves information one vehicle along the lane (Sec. III-B: every
vehicle reacts to its leader's state of the previous step), so a tile that
also simulates the J vehicles ahead of its owned ones (forward) or behind
them (backward) gets its owned vehicles exactly right for J steps.  The
per-vehicle arithmetic is the whole-lane kernels', and the FP32 gradient sums
are flushed into FP64 at the same K-step boundaries, so trajectories,
gradients and anomaly counts must equal a whole-lane plan's with the same K
bit for bit; the loss is summed over other work-groups and may differ in its
last bits.  Beside that, parity with the FP64 oracle at the tolerances of
the other parity tests.
"""
import numpy as np
import pytest

import scenarios
from scenarios import MODE_CLAMP, MODE_SOFTPLUS

from _util import grad_close, oracle_reference, oracle_targets, pos_close, ragged_scenario
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _run(sc, steps=None, target=None, dense=None, with_ws_forward=True, **plan_kw):
    """Forward (trajectories, anomaly counts) and backward through the plan's
    own entry points."""
    import torch
    from paper_2412_16750_amd import sim
    dev = "cuda"
    plan = sim.Plan.for_scenario(sc, **plan_kw)
    x = device_inputs(sc, dev)
    S, n = sc.n_steps, sc.n
    traj_d = torch.full((S + 1, n), float("nan"), dtype=torch.float32, device=dev)
    traj_v = torch.full((S + 1, n), float("nan"), dtype=torch.float32, device=dev)
    ws = plan.workspace(dev)
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d, traj_v,
                        ws if with_ws_forward else None)
    diag = sim.idm_plan_diagnostics(plan, ws).cpu().tolist() if with_ws_forward else None
    obs = None
    if target is not None:
        steps = np.asarray(steps)
        stride = int(steps[1] - steps[0]) if len(steps) > 1 else 1
        obs = sim.Obs(torch.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).to(dev),
                      int(steps[0]), stride)
    gd = None if dense is None else torch.from_numpy(
        np.ascontiguousarray(dense, dtype=np.float32)).to(dev)
    gp = torch.full((5, n), float("nan"), dtype=torch.float64, device=dev)
    gp0 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    gv0 = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    loss = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    if with_ws_forward:
        sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, gp0, gv0, ws,
                             grad_traj_d=gd, obs=obs, loss_out=loss)
    else:
        sim.idm_sim_backward_stored(plan, x["prm"], x["length"], x["p0"], traj_d, traj_v, gp, gp0,
                                    gv0, ws, grad_traj_d=gd, obs=obs, loss_out=loss)
    torch.cuda.synchronize()
    return dict(info=plan.info(), d=traj_d.cpu().numpy(), v=traj_v.cpu().numpy(),
                g=gp.cpu().numpy(), gp0=gp0.cpu().numpy(), gv0=gv0.cpu().numpy(),
                loss=float(loss.item()), diag=diag)


def _same(a, b, what, diag=True):
    for k in ("d", "v", "g", "gp0", "gv0"):
        assert np.array_equal(a[k], b[k]), (what, k, np.nanmax(np.abs(a[k] - b[k])))
    assert abs(a["loss"] - b["loss"]) <= 1e-12 * max(abs(b["loss"]), 1e-300), (what, a["loss"],
                                                                               b["loss"])
    if diag:
        assert a["diag"] == b["diag"], (what, a["diag"], b["diag"])


def _tiled(threads, J, K):
    return dict(threads=threads, per_thread=1, tuning_k=K, store_states=True, tile_steps=J)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
@pytest.mark.parametrize("shape", [(256, 64, 16), (512, 128, 32), (256, 32, 32),
                                   (1024, 256, 32), (768, 256, 32), (640, 256, 32),
                                   (576, 128, 32)])
def test_tiles_bitwise_equal_whole_lanes(mode, shape):
    """Lanes of 1 to 3000 vehicles (exactly a work-group, one more, a
    work-group less the halo, several tiles, a lane whose even split would
    fill every tile), S = 203 (a ragged last block of J and of K),
    fused MSE on every 5th step plus a dense upstream gradient: equal to the
    default plan (whole lanes, lanes above 1024 cut into pieces) with the
    same K; the oracle on the tiled result."""
    threads, J, K = shape
    # 3 T - 2 J: three tiles of exactly T slots without the T - 1 cap, the
    # backward's tail tile then ending on the lane tail at the last thread
    sizes = [1, 2, threads - J, threads, threads + 1, 600, 1000, 3000, 63, 0, 17, 2 * threads + 5,
             3 * threads - 2 * J]
    sc = ragged_scenario(sizes, 203, mode=mode, ckpt_every=K)
    steps = np.arange(3, sc.n_steps + 1, 5)
    tgt = oracle_targets(sc, steps, c=3)
    dense = np.random.default_rng(11).normal(0, 1e-3, size=(sc.n_steps + 1, sc.n)).astype(
        np.float32)
    t = _run(sc, steps, tgt, dense, **_tiled(threads, J, K))
    info = t["info"]
    log("tiles shape %s mode %d: %d tiles, plan %s" % (shape, mode, info["n_bundles"], info))
    assert info["tile_steps"] == J and info["ckpt_every"] == K and info["n_bundles"] > len(sizes)
    ref = _run(sc, steps, tgt, dense, tuning_k=K)
    _same(t, ref, "shape %s mode %d" % (shape, mode))
    o = oracle_reference(sc, steps, tgt, dense)
    P = sc.p0[None, :] + t["d"].astype(np.float64)
    okp, errp, _ = pos_close(P, o["P"])
    okg, wg = grad_close(t["g"], o["g"])
    ok0, w0 = grad_close(t["gp0"], o["gp0"])
    ok1, w1 = grad_close(t["gv0"], o["gv0"])
    log("tiles shape %s mode %d: position err %.2e, gradient worst/limit params %.3f p0 %.3f "
        "v0 %.3f" % (shape, mode, errp, wg, w0, w1))
    assert okp and okg and ok0 and ok1
    assert abs(t["loss"] - o["loss"]) <= 1e-4 * o["loss"]


@pytest.mark.parametrize("dense_only", [False, True])
def test_tiles_targets_only_and_dense_only(dense_only):
    """The backward without dense inputs (fused MSE on every step) and with a
    dense upstream only (no targets, loss 0)."""
    sizes = [1000, 24, 700, 3]
    sc = ragged_scenario(sizes, 100, ckpt_every=32)
    kw = _tiled(256, 64, 32)
    if dense_only:
        dense = scenarios.noise((sc.n_steps + 1, sc.n), 17, sigma=1e-2).astype(np.float32)
        t, ref = _run(sc, dense=dense, **kw), _run(sc, dense=dense, ckpt_every=32)
        assert t["loss"] == 0.0
    else:
        steps = np.arange(1, sc.n_steps + 1)
        tgt = oracle_targets(sc, steps, c=17)
        t, ref = _run(sc, steps, tgt, **kw), _run(sc, steps, tgt, ckpt_every=32)
    _same(t, ref, "dense only" if dense_only else "targets only")


def test_tiles_edge_steps():
    """S = 0 (one launch writing the initial row), S = 1, S below, at and just
    above one block of J, two blocks; single vehicles, lanes just longer than
    a tile, and two short lanes sharing a tile they fill exactly (its last
    thread, a lane tail, gathers from thread 0, the other lane's head)."""
    for sizes, S, threads, J, K in (([1, 300], 0, 256, 64, 16), ([300, 1], 1, 256, 64, 16),
                                    ([700], 63, 256, 64, 16), ([700, 2], 64, 256, 64, 16),
                                    ([257, 9], 65, 256, 32, 8), ([900], 128, 512, 128, 32),
                                    ([1, 513, 40], 129, 512, 128, 64),
                                    ([128, 700, 128, 2, 1], 70, 256, 64, 16)):
        sc = ragged_scenario(sizes, S, ckpt_every=K)
        dense = scenarios.noise((S + 1, sc.n), 5, sigma=1.0).astype(np.float32)
        if S > 0:
            steps = np.arange(1, S + 1)
            tgt = oracle_targets(sc, steps, c=5)
            t = _run(sc, steps, tgt, dense, **_tiled(threads, J, K))
            ref = _run(sc, steps, tgt, dense, tuning_k=K)
        else:
            t = _run(sc, dense=dense, **_tiled(threads, J, K))
            ref = _run(sc, dense=dense, tuning_k=K)
        _same(t, ref, "sizes %s S %d J %d K %d" % (sizes, S, J, K))


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_tiles_stop_and_go_counts(mode):
    """Stop-and-go lanes (Sec. III-C bounds active, speeds reaching 0) of 600
    vehicles, and lanes whose followers overlap their leaders (the gap floor
    from the first step): equal to whole lanes, anomaly counts included."""
    sc = scenarios.congested(n_lanes=6, lane_len=600, n_steps=150, mode=mode)
    sc.ckpt_every = 16
    steps = np.arange(1, sc.n_steps + 1)
    tgt = oracle_targets(sc, steps, c=9)
    t = _run(sc, steps, tgt, **_tiled(256, 64, 16))
    ref = _run(sc, steps, tgt, ckpt_every=16)
    log("tiles stop-and-go mode %d: counts %s, min speed %.3f" % (mode, t["diag"],
                                                                  float(np.min(t["v"]))))
    _same(t, ref, "stop-and-go mode %d" % mode)
    # overlapping vehicles (negative gaps) on three 700-vehicle lanes, each cut
    # into tiles
    n_lanes, lane_len = 3, 700
    off = scenarios.uniform_lanes(n_lanes, lane_len)
    n = int(off[-1])
    params = scenarios.draw_params(np.random.default_rng(1014), n)
    rng = np.random.default_rng(3014)
    gaps = np.where(rng.uniform(size=n) < 0.35, rng.uniform(-3.0, -0.5, n), rng.uniform(0.5, 20.0, n))
    v = rng.uniform(5.0, 20.0, n).astype(np.float32)
    p0 = np.zeros(n)
    for l in range(n_lanes):
        lo, hi = int(off[l]), int(off[l + 1])
        p0[hi - 1] = 0.0
        for i in range(hi - 2, lo - 1, -1):
            p0[i] = p0[i + 1] + params["length"][i] + gaps[i + 1]
    sc2 = scenarios.Scenario("overlap", off, params, p0, v, 3, mode=mode, ckpt_every=8)
    steps2 = np.arange(1, 4)
    tgt2 = oracle_targets(sc2, steps2, c=14)
    t2 = _run(sc2, steps2, tgt2, **_tiled(256, 32, 8))
    ref2 = _run(sc2, steps2, tgt2, ckpt_every=8)
    log("tiles overlap mode %d: counts %s" % (mode, t2["diag"]))
    assert t2["diag"][0] > 100
    _same(t2, ref2, "overlap mode %d" % mode)


def test_tiles_forward_into_caller_rows_and_stored_entry():
    """Without a workspace the tiled forward keeps its states in the caller's
    two trajectory outputs; idm_sim_backward_stored reads them from there;
    with neither, the forward says what it needs."""
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd._lib import IdmError
    sizes = [800, 5, 300]
    sc = ragged_scenario(sizes, 90, ckpt_every=16)
    steps = np.arange(2, sc.n_steps + 1, 4)
    tgt = oracle_targets(sc, steps, c=21)
    t = _run(sc, steps, tgt, with_ws_forward=False, **_tiled(256, 64, 16))
    ref = _run(sc, steps, tgt, ckpt_every=16)
    _same(t, ref, "caller rows", diag=False)
    plan = sim.Plan.for_scenario(sc, **_tiled(256, 64, 16))
    x = device_inputs(sc)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    with pytest.raises(IdmError) as e:
        sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None, None)
    assert "trajectory" in str(e.value)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_tiles_fit_graph_bitwise(mode):
    """Fit steps replayed as one captured graph (several launches per pass)
    on a tiled plan: the parameters equal those of a whole-lane plan that
    keeps its states, iteration for iteration; the loss history agrees to
    rounding."""
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd.fit import Fitter
    sc = scenarios.make_scenario("fittile", scenarios.uniform_lanes(6, 1000), 200, 4, mode=mode,
                                 ckpt_every=32)
    steps = scenarios.obs_steps(sc.n_steps, 10, 10)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=4)).cuda()
    x = device_inputs(sc)
    cold = sim.params_tensor(scenarios.cold_params(sc), "cuda")
    res = {}
    for tag, kw in (("tiles", _tiled(512, 128, 32)), ("lanes", dict(store_states=True))):
        plan = sim.Plan.for_scenario(sc, **kw)
        f = Fitter(plan, x["length"], x["p0"], x["v"], sim.Obs(tgt, 10, 10))
        f.init(cold)
        f.run(4)
        f.step()
        f.run(3)
        torch.cuda.synchronize()
        res[tag] = (f.params.cpu().numpy(), f.losses(), plan.info())
    log("tiles fit mode %d: plans %s / %s, losses %s" % (mode, res["tiles"][2], res["lanes"][2],
                                                       res["tiles"][1][:3]))
    assert res["tiles"][2]["tile_steps"] == 128
    assert np.array_equal(res["tiles"][0], res["lanes"][0])
    np.testing.assert_allclose(res["tiles"][1], res["lanes"][1], rtol=1e-12)


def test_tiles_autotune_and_full_fit_workload():
    """The fit workload at full size (100 lanes x 1000 vehicles, 500 steps,
    observed every 10th step): a tiled plan equals the whole-lane plan that
    keeps its states, and the autotuner, asked to weigh the backwards
    (store_states "auto"), picks a shape whose results are equal too."""
    import torch
    from paper_2412_16750_amd import sim
    sc = scenarios.fit()
    steps = scenarios.obs_steps(sc.n_steps, 10, 10)
    tgt = scenarios.constant_speed_targets(sc, steps, 4)
    t = _run(sc, steps, tgt, **_tiled(512, 128, 32))
    ref = _run(sc, steps, tgt, store_states=True)
    _same(t, ref, "fit workload 512 x 128")
    plan = sim.Plan.for_scenario(sc, store_states="auto")
    x = device_inputs(sc)
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), 10, 10)
    room = sim.Plan.for_scenario(sc, **_tiled(256, 64, 32)).workspace_bytes
    tb = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], obs=obs,
                         workspace_bytes=room)
    tuned = sim.idm_plan_autotune(tb, reps=2)
    log("tiles autotune on the fit workload: %s" % tuned)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    gp = torch.empty(5, sc.n, dtype=torch.float64, device="cuda")
    g0 = torch.empty(sc.n, dtype=torch.float64, device="cuda")
    g1 = torch.empty_like(g0)
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None, ws)
    sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, g0, g1, ws, obs=obs)
    torch.cuda.synchronize()
    assert np.array_equal(traj.cpu().numpy(), ref["d"])
    assert np.array_equal(gp.cpu().numpy(), ref["g"])
    assert np.array_equal(g0.cpu().numpy(), ref["gp0"])
    assert np.array_equal(g1.cpu().numpy(), ref["gv0"])


def test_tiles_step_graph_autograd_noalloc_and_forward_helper():
    """A tiled plan under the other entry points: the step graph with
    trajectory outputs (several launches inside one graph, the kept states
    written straight into the outputs and read back from them) replayed three
    times with eager work in between, the step graph with only the
    displacement output (speeds kept in the workspace), also on a whole-lane
    plan keeping states, autograd, the no-allocation gradient and a
    forward-only call through the plan's forward workspace all equal the
    whole-lane plan's results."""
    import torch
    from paper_2412_16750_amd import autograd, sim
    sc = ragged_scenario([900, 33, 700, 1, 300], 150, ckpt_every=16)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = torch.from_numpy(oracle_targets(sc, steps, c=23)).cuda()
    obs = sim.Obs(tgt, 1, 1)
    x = device_inputs(sc)
    S, n = sc.n_steps, sc.n
    tiled = sim.Plan.for_scenario(sc, **_tiled(256, 64, 16))
    whole = sim.Plan.for_scenario(sc, ckpt_every=16)
    ref = sim.StepBuffers(whole, x["prm"], x["length"], x["p0"], x["v"],
                          traj_d=torch.empty(S + 1, n, device="cuda"),
                          traj_v=torch.empty(S + 1, n, device="cuda"), obs=obs)
    ref.run_eager()
    torch.cuda.synchronize()
    b = sim.StepBuffers(tiled, x["prm"], x["length"], x["p0"], x["v"],
                        traj_d=torch.empty(S + 1, n, device="cuda"),
                        traj_v=torch.empty(S + 1, n, device="cuda"), obs=obs)
    for rep in range(3):
        for t in (b.traj_d, b.traj_v, b.grad_params, b.grad_p0, b.grad_v0):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        sim.idm_step_graph_launch(b)
        torch.cuda.synchronize()
        for k in ("traj_d", "traj_v", "grad_params", "grad_p0", "grad_v0"):
            assert torch.equal(getattr(b, k), getattr(ref, k)), (rep, k)
        assert abs(b.loss.item() - ref.loss.item()) <= 1e-12 * ref.loss.item()
    kept = sim.Plan.for_scenario(sc, ckpt_every=16, store_states=True)
    for plan in (tiled, kept):
        bd = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"],
                             traj_d=torch.full((S + 1, n), float("nan"), device="cuda"), obs=obs)
        for rep in range(2):
            bd.grad_params.fill_(float("nan"))
            torch.cuda.synchronize()
            sim.idm_step_graph_launch(bd)
            torch.cuda.synchronize()
            for k in ("traj_d", "grad_params", "grad_p0", "grad_v0"):
                assert torch.equal(getattr(bd, k), getattr(ref, k)), (plan.info()["tile_steps"], k)
            assert abs(bd.loss.item() - ref.loss.item()) <= 1e-12 * ref.loss.item()
        del bd
    grads = []
    for plan in (whole, tiled):
        prm = x["prm"].clone().requires_grad_(True)
        d = autograd.simulate(plan, prm, x["p0"], x["v"], x["length"])
        (d[-1].double() ** 2).sum().backward()
        grads.append(prm.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1])
    outs = []
    for plan in (whole, tiled):
        gp = torch.empty(5, n, dtype=torch.float64, device="cuda")
        g0 = torch.empty(n, dtype=torch.float64, device="cuda")
        g1 = torch.empty(n, dtype=torch.float64, device="cuda")
        sim.idm_sim_backward_noalloc(plan, x["prm"], x["length"], x["p0"], x["v"], gp, g0, g1,
                                     obs=obs)
        traj = torch.empty(S + 1, n, device="cuda")
        sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None,
                            plan.forward_workspace())
        torch.cuda.synchronize()
        outs.append((gp.cpu().numpy(), g0.cpu().numpy(), g1.cpu().numpy(), traj.cpu().numpy()))
    for a, c in zip(outs[0], outs[1]):
        assert np.array_equal(a, c)
    assert np.array_equal(outs[1][3], ref.traj_d.cpu().numpy())


@pytest.mark.parametrize("seed", range(8))
def test_random_tiles_bitwise(seed):
    """Random lane mixes, tile widths, halo lengths, step counts, checkpoint
    intervals, bound modes and upstream kinds: halo tiles give the
    trajectories, gradients and anomaly counts of the whole-lane plan with
    the same K, bit for bit."""
    rng = np.random.default_rng(300 + seed)
    K = int(rng.choice([8, 16, 32]))
    threads = int(rng.choice([256, 512, 576, 640, 768, 1024]))
    Js = [j for j in range(K, threads, K) if j % 2 == 0 and j <= 256]
    J = int(rng.choice(Js))
    n = int(rng.integers(3, 20))
    sizes = rng.integers(1, 3 * threads + 1, n)
    sizes[rng.integers(0, n)] = int(2.5 * threads)       # at least one lane cut several times
    S = int(rng.integers(1, 3 * J + 2))
    mode = int(rng.integers(0, 2))
    sc = ragged_scenario(sizes, S, mode=mode, seed_c=80 + seed, ckpt_every=K)
    steps = np.arange(1, S + 1)
    tgt = oracle_targets(sc, steps, c=80 + seed)
    dense = None
    if rng.integers(0, 2):
        dense = np.random.default_rng(seed).normal(0, 1e-3, (S + 1, sc.n)).astype(np.float32)
    t = _run(sc, steps, tgt, dense, **_tiled(threads, J, K))
    ref = _run(sc, steps, tgt, dense, tuning_k=K)
    log("random tiles seed %d: %d x J %d, K %d, S %d, mode %d, dense %s, %d tiles"
        % (seed, threads, J, K, S, mode, dense is not None, t["info"]["n_bundles"]))
    assert t["info"]["n_bundles"] > n
    _same(t, ref, "seed %d" % seed)
