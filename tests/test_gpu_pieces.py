"""Lanes longer than a work-group bundle: cut into pieces that run in
successive launches and exchange the boundary vehicle's state (forward) and
adjoint contribution (backward) through the workspace.

The cut changes no arithmetic: trajectories and per-vehicle gradients are
bitwise those of the same lanes run whole in a larger bundle, and both match
the FP64 oracle to the usual tolerances (positions 1e-4 relative, gradients
1e-3 relative)."""
import numpy as np
import pytest

import scenarios
from scenarios import MODE_CLAMP, MODE_SOFTPLUS

from _util import grad_close, oracle_reference, oracle_targets, pos_close, ragged_scenario
from gpu_run import gpu_run, log

pytestmark = pytest.mark.gpu

KEYS = ("d", "V", "g", "gp0", "gv0")


def _sizes(n, hi, seed, extra=()):
    s = scenarios.lognormal_lane_sizes(n, np.log(hi) - 1.0, 1.0, 1, hi, seed)
    return np.concatenate([np.asarray(extra, dtype=s.dtype), s])


def _same(a, b, what):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), (what, k)
    assert abs(a["loss"] - b["loss"]) <= 1e-12 * abs(b["loss"]), what


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
@pytest.mark.parametrize("dense", [False, True])
def test_pieces_bitwise_equal_to_whole_lanes(mode, dense):
    """Lanes up to 400 vehicles (with sizes at and around multiples of 64) in
    64-slot bundles (up to 7 pieces, 7 launch levels) against 512-slot
    bundles holding every lane whole; fused MSE or a dense upstream."""
    sizes = _sizes(60, 400, 41, extra=(64, 65, 128, 129, 191, 192, 1, 400))
    sc = ragged_scenario(sizes, 48, mode=mode, seed_c=41, ckpt_every=16)
    steps = np.arange(2, sc.n_steps + 1, 2)
    tgt = oracle_targets(sc, steps, c=41)
    gd = None
    if dense:
        gd = scenarios.noise((sc.n_steps + 1, sc.n), 43, sigma=1e-3).astype(np.float32)
    whole = gpu_run(sc, steps, tgt, dense=gd, threads=512, per_thread=1, block=16)
    cut = gpu_run(sc, steps, tgt, dense=gd, threads=64, per_thread=1, block=16)
    log("pieces: whole %s / cut %s" % (whole["info"], cut["info"]))
    assert whole["info"]["n_levels"] == 1 and cut["info"]["n_levels"] == 7
    assert cut["info"]["n_boundaries"] == int(np.sum(np.maximum(-(-sizes // 64) - 1, 0)))
    _same(cut, whole, "64-slot pieces vs whole lanes")
    # a persistent grid walks every level's bundles
    pers = gpu_run(sc, steps, tgt, dense=gd, threads=64, per_thread=1, block=16, grid=3)
    _same(pers, whole, "persistent grid")


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_long_lanes_default_shape_oracle_parity(mode):
    """Lanes of 2500, 1100, 1025 and 1024 vehicles among short ones: the
    default shape (1024 threads x 1, K = 32 with the LDS stash) cuts them into
    up to 3 pieces; parity with the oracle, and bitwise equality with the
    register-only backward (block 32)."""
    sizes = _sizes(40, 300, 42, extra=(2500, 1100, 1025, 1024, 3))
    sc = ragged_scenario(sizes, 64, mode=mode, seed_c=42, ckpt_every=32)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = oracle_targets(sc, steps, c=42)
    out = gpu_run(sc, steps, tgt)
    info = out["info"]
    log("long lanes: plan %s" % info)
    assert (info["threads"], info["per_thread"], info["block"]) == (1024, 1, 16)
    assert info["n_levels"] == 3 and info["n_boundaries"] == 2 + 1 + 1
    ref = oracle_reference(sc, steps, tgt)
    ok, err, w = pos_close(out["P"], ref["P"])
    log("long lanes: positions max|err| %.3e m, worst/limit %.3f" % (err, w))
    assert ok
    okv, _, wv = pos_close(out["V"].astype(np.float64), ref["V"])
    assert okv, wv
    okg, wg = grad_close(out["g"], ref["g"])
    ok0, w0 = grad_close(out["gp0"], ref["gp0"])
    ok1, w1 = grad_close(out["gv0"], ref["gv0"])
    log("long lanes: gradient worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1
    assert abs(out["loss"] - ref["loss"]) <= 1e-4 * ref["loss"]
    reg = gpu_run(sc, steps, tgt, block=32)
    assert reg["info"]["block"] == 32
    _same(out, reg, "stash vs register backward")


@pytest.mark.parametrize("S", [0, 1, 5])
def test_pieces_few_steps(S):
    """Zero, one and a few steps (a partial checkpoint block) with pieces."""
    sizes = _sizes(10, 200, 44, extra=(300, 130))
    sc = ragged_scenario(sizes, S, seed_c=44, ckpt_every=8)
    steps = np.arange(0, S + 1)
    tgt = oracle_targets(sc, steps, c=44)
    whole = gpu_run(sc, steps, tgt, threads=512, per_thread=1, block=8)
    cut = gpu_run(sc, steps, tgt, threads=64, per_thread=1, block=8)
    assert cut["info"]["n_levels"] == 5
    _same(cut, whole, "S=%d" % S)
    ref = oracle_reference(sc, steps, tgt)
    assert pos_close(cut["P"], ref["P"])[0]
    assert grad_close(cut["g"], ref["g"])[0] and grad_close(cut["gv0"], ref["gv0"])[0]


def test_forward_without_workspace_is_rejected_with_pieces():
    import torch
    from paper_2412_16750_amd import _lib, sim
    from gpu_run import device_inputs
    sc = ragged_scenario([100, 30], 10, seed_c=45)
    plan = sim.Plan.for_scenario(sc, threads=64, per_thread=1)
    assert plan.info()["n_boundaries"] == 1
    x = device_inputs(sc)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.IdmError):
        sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None, None)
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None,
                        plan.workspace())
    torch.cuda.synchronize()


def test_graph_and_fit_with_pieces():
    """Forward + backward as one replayed graph, and the graph-captured fit,
    on a plan with pieces: bitwise the eager results / the whole-lane fit."""
    import torch
    from paper_2412_16750_amd import fit, sim
    from gpu_run import device_inputs
    sizes = _sizes(30, 300, 46, extra=(700, 260))
    sc = ragged_scenario(sizes, 40, seed_c=46, ckpt_every=16)
    steps = np.arange(4, sc.n_steps + 1, 4)
    tgt = oracle_targets(sc, steps, c=46)
    x = device_inputs(sc)
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), int(steps[0]), 4)
    plan = sim.Plan.for_scenario(sc, threads=128, per_thread=1, block=16)
    assert plan.info()["n_levels"] == 6
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    b = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d=traj, obs=obs)
    b.run_eager()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (b.traj_d, b.grad_params, b.grad_p0, b.grad_v0, b.loss)]
    for rep in range(3):
        for t in (b.traj_d, b.grad_params, b.grad_p0, b.grad_v0, b.loss):
            t.zero_()
        sim.idm_step_graph_launch(b)
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").square().sum()
        torch.cuda.synchronize()
        for a, e in zip((b.traj_d, b.grad_params, b.grad_p0, b.grad_v0, b.loss), eager):
            assert torch.equal(a, e), rep
        del junk
    cold = sim.params_tensor(scenarios.cold_params(sc), "cuda")
    res = []
    for kw in (dict(threads=128, per_thread=1, block=16), dict(threads=1024, per_thread=1, block=16)):
        p = sim.Plan.for_scenario(sc, **kw)
        f = fit.Fitter(p, x["length"], x["p0"], x["v"], obs, lr0=0.05)
        f.init(cold)
        f.run(6)
        torch.cuda.synchronize()
        res.append((f.params.clone(), np.asarray(f.losses())))
    assert torch.equal(res[0][0], res[1][0])
    assert np.allclose(res[0][1], res[1][1], rtol=1e-12, atol=0)


def test_autograd_with_pieces():
    """torch.autograd through a plan with pieces: the dense upstream reaches
    every piece, and two simulations in flight keep their own boundary rows."""
    import torch
    from paper_2412_16750_amd import autograd, sim
    from gpu_run import device_inputs
    sizes = _sizes(20, 300, 47, extra=(500, 129))
    sc = ragged_scenario(sizes, 30, seed_c=47, ckpt_every=16)
    x = device_inputs(sc)
    w = torch.from_numpy(scenarios.noise((sc.n_steps + 1, sc.n), 48, sigma=1.0)).cuda()
    grads = []
    for kw in (dict(threads=64, per_thread=1, block=16), dict(threads=512, per_thread=1, block=16)):
        plan = sim.Plan.for_scenario(sc, **kw)
        prm = x["prm"].clone().requires_grad_(True)
        v0 = x["v"].clone().requires_grad_(True)
        d1 = autograd.simulate(plan, prm, x["p0"], v0, x["length"])
        d2 = autograd.simulate(plan, prm * 1.01, x["p0"], v0, x["length"])  # second in flight
        loss = (w * d1.double()).sum() + 0.5 * (w * d2.double()).sum()
        loss.backward()
        torch.cuda.synchronize()
        grads.append((prm.grad.clone(), v0.grad.clone(), plan.info()["n_levels"]))
    assert grads[0][2] == 8 and grads[1][2] == 1
    # FP64 gradients rounded to FP32 by the wrapper: bitwise equal across the cut
    assert torch.equal(grads[0][0], grads[1][0]) and torch.equal(grads[0][1], grads[1][1])


def test_autotuner_with_pieces():
    """The autotuner on lanes up to 2500 vehicles (K fixed at 32): it may pick
    any shape whose workspace fits; trajectories and gradients stay bitwise
    those of the default plan."""
    import torch
    from paper_2412_16750_amd import sim
    from gpu_run import device_inputs
    sizes = _sizes(60, 400, 49, extra=(2500, 1500, 700))
    sc = ragged_scenario(sizes, 40, seed_c=49, ckpt_every=32)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = oracle_targets(sc, steps, c=49)
    x = device_inputs(sc)
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), 1, 1)
    plan = sim.Plan.for_scenario(sc)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    b = sim.StepBuffers(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d=traj, obs=obs)
    # room for the shapes that cut lanes into more pieces
    b.workspace = torch.empty(4 * plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    b.run_eager()
    torch.cuda.synchronize()
    before = [t.clone() for t in (b.traj_d, b.grad_params, b.grad_p0, b.grad_v0)]
    info = sim.idm_plan_autotune(b, reps=1)
    log("autotune with pieces chose %s" % info)
    assert info["ckpt_every"] == 32 and info["per_thread"] == 1
    b.run_eager()
    torch.cuda.synchronize()
    for a, e in zip((b.traj_d, b.grad_params, b.grad_p0, b.grad_v0), before):
        assert torch.equal(a, e)


@pytest.mark.parametrize("seed", range(10))
def test_random_cuts_bitwise(seed):
    """Random lane mixes, bundle sizes, step counts, checkpoint intervals,
    bound modes and upstream kinds (targets, or targets and a dense upstream
    gradient from seed 6 on): lanes cut into pieces give the trajectories
    and gradients of the same lanes held whole by 1024-slot bundles, bit for
    bit."""
    rng = np.random.default_rng(100 + seed)
    cap = int(rng.choice([64, 128, 256]))
    n = int(rng.integers(5, 40))
    sizes = rng.integers(1, 3 * cap + 1, n)
    sizes[rng.integers(0, n)] = 3 * cap            # at least three pieces somewhere
    S = int(rng.integers(1, 41))
    K = int(rng.choice([8, 16]))
    mode = int(rng.integers(0, 2))
    sc = ragged_scenario(sizes, S, mode=mode, seed_c=60 + seed, ckpt_every=K)
    steps = np.arange(1, S + 1)
    tgt = oracle_targets(sc, steps, c=60 + seed)
    dense = None
    if seed >= 6:
        dense = np.random.default_rng(seed).normal(0, 1e-3, (S + 1, sc.n)).astype(np.float32)
    whole = gpu_run(sc, steps, tgt, dense, threads=1024, per_thread=1, block=8)
    cut = gpu_run(sc, steps, tgt, dense, threads=cap, per_thread=1, block=8)
    log("random cut seed %d: cap %d, S %d, K %d, mode %d, dense %s, levels %d" %
        (seed, cap, S, K, mode, dense is not None, cut["info"]["n_levels"]))
    assert cut["info"]["n_levels"] >= 3
    _same(cut, whole, "seed %d" % seed)
