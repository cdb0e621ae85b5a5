"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Positions: |p_gpu - p_oracle| <= 1e-4 * max(|p_oracle|, 1 m) at every step.
Gradients: |g_gpu - g_oracle| <= 1e-3 * max(|g_oracle|, 1e-2 * max|g_oracle|)
per parameter kind and for both initial-state gradients.
The GPU simulates in FP32 and sums gradients in FP64; the oracle is FP64.
"""
import numpy as np
import pytest

import scenarios
from scenarios import MODE_CLAMP, MODE_SOFTPLUS

from _util import (disp_close, grad_close, oracle_reference, oracle_targets, pos_close,
                   ragged_scenario)
from gpu_run import gpu_run, log

pytestmark = pytest.mark.gpu


def _check(sc, ref, out, what, pos_rtol=1e-4, grad_rtol=1e-3, check_v=True):
    ok, maxerr, worst = pos_close(out["P"], ref["P"], rtol=pos_rtol)
    log("%s: positions max|err| = %.3e m, worst/limit = %.3f" % (what, maxerr, worst))
    assert ok, (what, maxerr, worst)
    okd, maxd, worstd = disp_close(out["d"], ref["P"], sc.p0, rtol=pos_rtol)
    log("%s: displacements max|err| = %.3e m, worst/limit = %.3f" % (what, maxd, worstd))
    assert okd, (what, maxd, worstd)
    # the gap floor never triggers on these lanes, and no state is non-finite
    assert out["diag"] == [ref["floor_hits"], 0], (what, out["diag"], ref["floor_hits"])
    if check_v:
        okv, maxv, worstv = pos_close(out["V"].astype(np.float64), ref["V"], rtol=pos_rtol)
        log("%s: speeds max|err| = %.3e m/s" % (what, maxv))
        assert okv, (what, maxv, worstv)
    if "g" in out:
        where = []
        okg, wg = grad_close(out["g"], ref["g"], rtol=grad_rtol, where=where)
        ok0, w0 = grad_close(out["gp0"], ref["gp0"], rtol=grad_rtol)
        ok1, w1 = grad_close(out["gv0"], ref["gv0"], rtol=grad_rtol)
        log("%s: gradient worst/limit params %.3f p0 %.3f v0 %.3f (worst param element "
            "(kind, vehicle, gpu, oracle, limit) = %s)" % (what, wg, w0, w1, where))
        assert okg and ok0 and ok1, (what, wg, w0, w1)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_single_lane_1000_steps(mode):
    """1 lane x 100 vehicles, 1000 steps; MSE against targets from a second
    parameter draw plus N(0, 0.5 m) noise, observed at every step 1..1000."""
    sc = scenarios.single_lane(mode=mode, ckpt_every=32)
    steps = np.arange(1, sc.n_steps + 1)
    tgt = oracle_targets(sc, steps)
    ref = oracle_reference(sc, steps, tgt)
    log("single_lane mode=%d: oracle loss %.6e, floor hits %d" % (mode, ref["loss"], ref["floor_hits"]))
    out = gpu_run(sc, steps, tgt)
    _check(sc, ref, out, "single_lane mode=%d" % mode)
    assert abs(out["loss"] - ref["loss"]) <= 1e-4 * ref["loss"], (out["loss"], ref["loss"])


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
@pytest.mark.parametrize("shape", [(64, 1, 8, 8), (128, 2, 8, 8), (64, 4, 4, 4), (256, 1, 32, 32),
                                   (256, 1, 32, 16), (128, 1, 32, 8), (128, 2, 16, 16),
                                   (64, 4, 8, 8), (64, 4, 24, 4), (1024, 1, 32, 16),
                                   (512, 1, 32, 16), (512, 2, 32, 16), (256, 4, 16, 8)])
def test_ragged_lanes_several_tiles(mode, shape):
    """Lanes of 1..256 vehicles (several work-group tiles, ragged bundle tails),
    S = 203 (ragged last checkpoint block and sub-block), checkpoint interval K
    with a backward register block KB dividing it (1 to 6 sub-blocks per
    checkpoint block; K = 2 KB on the shapes with an LDS stash of the lower
    sub-block), dense upstream gradient + fused MSE."""
    threads, per, K, KB = shape
    sizes = [1, 2, 3, 63, 64, 65, 100, 127, 31, 256, 0, 17, 200, 5, 90]
    cap = threads * per
    sizes = [s for s in sizes if s <= cap]
    sc = ragged_scenario(sizes, 203, mode=mode, ckpt_every=K)
    rng = np.random.default_rng(11)
    steps = np.arange(3, sc.n_steps + 1, 5)
    tgt = oracle_targets(sc, steps, c=3)
    dense = rng.normal(0, 1e-3, size=(sc.n_steps + 1, sc.n)).astype(np.float32)
    ref = oracle_reference(sc, steps, tgt, dense)
    out = gpu_run(sc, steps, tgt, dense, threads=threads, per_thread=per, tuning_k=K, block=KB)
    assert out["info"]["threads"] == threads and out["info"]["per_thread"] == per
    assert out["info"]["ckpt_every"] == K and out["info"]["block"] == KB
    _check(sc, ref, out, "ragged mode=%d shape=%s" % (mode, shape))


def test_forward_bitwise_independent_of_launch_shape():
    """The per-vehicle arithmetic does not depend on where the leader's state
    comes from (register or LDS), so trajectories are bitwise identical for
    every launch shape and checkpoint interval; gradients are bitwise identical
    across shapes with the same K.  Only the FP64 loss sum depends on how lanes
    are grouped into bundles (summation order).""" 
    sizes = [50, 64, 1, 120, 33, 7, 128]
    sc = ragged_scenario(sizes, 150, ckpt_every=8)
    steps = np.arange(1, 151)
    tgt = oracle_targets(sc, steps, c=5)
    base = gpu_run(sc, steps, tgt, threads=128, per_thread=1, tuning_k=8)
    for shape in [(64, 2, 8), (64, 4, 8), (256, 1, 8), (128, 2, 8)]:
        o = gpu_run(sc, steps, tgt, threads=shape[0], per_thread=shape[1], tuning_k=shape[2])
        assert np.array_equal(o["d"], base["d"]) and np.array_equal(o["V"], base["V"]), shape
        assert np.array_equal(o["g"], base["g"]), shape
        assert np.array_equal(o["gp0"], base["gp0"]) and np.array_equal(o["gv0"], base["gv0"])
        # the loss is summed per bundle, and bundles differ between shapes
        assert abs(o["loss"] - base["loss"]) <= 1e-13 * base["loss"]
    for K, KB in ((16, 16), (32, 32), (32, 8), (24, 8)):
        o = gpu_run(sc, steps, tgt, threads=128, per_thread=1, tuning_k=K, block=KB)
        assert np.array_equal(o["d"], base["d"]) and np.array_equal(o["V"], base["V"])
        okg, w = grad_close(o["g"], base["g"], rtol=1e-5)
        assert okg, (K, KB, w)
    # with K fixed, the register block only changes where states are recomputed:
    # the arithmetic of every step is the same, so gradients are bitwise equal
    a32 = gpu_run(sc, steps, tgt, threads=128, per_thread=1, tuning_k=32, block=32)
    b32 = gpu_run(sc, steps, tgt, threads=128, per_thread=1, tuning_k=32, block=8)
    for k in ("g", "gp0", "gv0"):
        assert np.array_equal(a32[k], b32[k]), k


def test_persistent_grid_matches_one_group_per_bundle():
    sizes = [30, 64, 2, 64, 64, 17, 9, 50, 64, 1] * 6
    sc = ragged_scenario(sizes, 64, ckpt_every=8)
    steps = np.arange(2, 65, 2)
    tgt = oracle_targets(sc, steps, c=6)
    a = gpu_run(sc, steps, tgt, threads=64, per_thread=1, tuning_k=8, grid=0)
    b = gpu_run(sc, steps, tgt, threads=64, per_thread=1, tuning_k=8, grid=3)
    assert b["info"]["grid"] == 3 and a["info"]["grid"] == a["info"]["n_bundles"]
    for k in ("d", "V", "g", "gp0", "gv0"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loss"] == b["loss"]


def test_repeat_runs_are_bitwise_identical():
    sc = scenarios.single_lane(n_vehicles=300, n_steps=300, ckpt_every=16)
    steps = np.arange(1, 301)
    tgt = oracle_targets(sc, steps, c=2)
    a = gpu_run(sc, steps, tgt)
    b = gpu_run(sc, steps, tgt)
    for k in ("d", "V", "g", "gp0", "gv0"):
        assert np.array_equal(a[k], b[k]), k
    assert a["loss"] == b["loss"]


def test_zero_steps_and_single_vehicle():
    sc = ragged_scenario([1], 0, ckpt_every=8)
    dense = np.array([[0.7]], dtype=np.float32)
    out = gpu_run(sc, dense=dense, tuning_k=8)
    assert out["d"].shape == (1, 1) and out["d"][0, 0] == 0.0
    # d_0 = 0 does not depend on p0 or v_init
    assert out["gp0"][0] == 0.0 and out["gv0"][0] == 0.0
    assert np.all(out["g"] == 0.0)
    sc1 = ragged_scenario([1], 400, ckpt_every=16)
    steps = np.arange(1, 401)
    tgt = oracle_targets(sc1, steps, c=4)
    ref = oracle_reference(sc1, steps, tgt)
    out1 = gpu_run(sc1, steps, tgt)
    _check(sc1, ref, out1, "single vehicle")


def test_full_capacity_lanes():
    """Lanes that fill a bundle exactly (1024 = 1024 x 1 and 256 x 4)."""
    for threads, per, K in [(1024, 1, 32), (256, 4, 4)]:
        sc = ragged_scenario([1024, 1023], 120, ckpt_every=K)
        steps = np.arange(1, 121)
        tgt = oracle_targets(sc, steps, c=8)
        ref = oracle_reference(sc, steps, tgt)
        out = gpu_run(sc, steps, tgt, threads=threads, per_thread=per, tuning_k=K)
        _check(sc, ref, out, "full capacity %s" % ((threads, per, K),))


def test_lanes_far_from_origin():
    """Lanes 250 km from the origin (an FP32 position step there is 1.6 cm): the
    residual p0 + d - target is formed from a two-float split of p0, so loss and
    gradients keep the oracle's accuracy although positions alone could not."""
    sizes = [100, 37, 64, 1]
    sc = ragged_scenario(sizes, 300, ckpt_every=32)
    sc.p0 = sc.p0 + 2.5e5
    steps = np.arange(2, sc.n_steps + 1, 2)
    tgt = oracle_targets(sc, steps, c=9)
    ref = oracle_reference(sc, steps, tgt)
    out = gpu_run(sc, steps, tgt, threads=128, per_thread=1, tuning_k=32, block=16)
    log("far lanes: loss %.9e vs oracle %.9e" % (out["loss"], ref["loss"]))
    assert abs(out["loss"] - ref["loss"]) <= 1e-4 * ref["loss"]
    _check(sc, ref, out, "far from origin")


@pytest.mark.parametrize("mode", [MODE_CLAMP, MODE_SOFTPLUS])
def test_equilibrium_platoon_on_gpu(mode):
    """An open-lane platoon at its equilibrium gaps (Eqs. 1-2 with dv = 0)
    stays at the head's fixed-point speed in FP32 too."""
    import math
    n = 64
    rng = np.random.default_rng(7)
    v0 = rng.uniform(32, 40, n); v0[0] = 24.0
    T = rng.uniform(1, 2, n); a = rng.uniform(1, 2, n); b = rng.uniform(1.5, 3, n)
    s0 = rng.uniform(1.5, 3, n); length = rng.uniform(3.5, 12.0, n)
    prm = {k: np.asarray(x, dtype=np.float32) for k, x in
           dict(v0=v0, T=T, a=a, b=b, s0=s0, length=length).items()}
    f = {k: prm[k].astype(np.float64) for k in prm}
    cm = math.log(1.0 - math.exp(-10.0))
    V = f["v0"][0] if mode == MODE_CLAMP else f["v0"][0] * (1.0 - cm / f["a"][0]) ** 0.25
    p = np.zeros(n)
    for i in range(1, n):
        x4 = (V / f["v0"][i]) ** 4
        sopt = f["s0"][i] + V * f["T"][i]
        if mode == MODE_CLAMP:
            s_e = sopt / math.sqrt(1.0 - x4)
        else:
            s_e = (sopt + math.log1p(math.exp(-sopt))) / math.sqrt(1.0 - x4 - cm / f["a"][i])
        p[i] = p[i - 1] - f["length"][i - 1] - s_e
    p -= p[-1]
    sc = scenarios.Scenario("platoon", np.array([0, n], np.int32), prm, p,
                            np.full(n, V, np.float32), 1000, mode=mode, ckpt_every=16)
    out = gpu_run(sc, want_backward=False)
    assert np.max(np.abs(out["V"] - V)) < 2e-4
    gaps = out["P"][:, :-1] - out["P"][:, 1:]
    assert np.max(np.abs(gaps - gaps[0])) < 5e-3


def test_scale_config_sampled_lanes():
    """The 2000 x 1000 = 2M-vehicle workload, 100 steps, checkpoints every 32,
    in the launch shape the benchmark uses; the oracle recomputes 6 sampled
    lanes (lanes are independent, so a lane subset is an exact reference)."""
    import torch
    from paper_2412_16750_amd import sim
    from gpu_run import device_inputs
    sc = scenarios.scale()
    log("scale: N=%d S=%d" % (sc.n, sc.n_steps))
    steps = np.arange(1, sc.n_steps + 1)
    tgt = scenarios.constant_speed_targets(sc, steps, 2)
    plan = sim.Plan.for_scenario(sc)
    x = device_inputs(sc)
    S, n = sc.n_steps, sc.n
    traj_d = torch.empty(S + 1, n, dtype=torch.float32, device="cuda")
    ws = plan.workspace()
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), 1, 1)
    gp = torch.empty(5, n, dtype=torch.float64, device="cuda")
    gp0 = torch.empty(n, dtype=torch.float64, device="cuda")
    gv0 = torch.empty(n, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj_d, None, ws)
    sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], gp, gp0, gv0, ws, obs=obs,
                         loss_out=loss)
    torch.cuda.synchronize()
    log("scale: plan %s" % plan.info())
    lanes = [0, 1, 777, 1000, 1998, 1999]
    sub = scenarios.subset_lanes(sc, lanes)
    idx = sub.extra["vehicle_index"]
    # the MSE normalisation is over ALL N vehicles: scale the subset's gradient
    ref = oracle_reference(sub, steps, tgt[:, idx])
    fac = sub.n / sc.n
    d = traj_d[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    ok, maxerr, worst = pos_close(sc.p0[idx][None, :] + d.astype(np.float64), ref["P"])
    log("scale sampled: positions max|err| %.3e worst/limit %.3f" % (maxerr, worst))
    assert ok
    okd, maxd, worstd = disp_close(d, ref["P"], sc.p0[idx])
    log("scale sampled: displacements max|err| %.3e worst/limit %.3f" % (maxd, worstd))
    assert okd
    diag = sim.idm_plan_diagnostics(plan, ws).cpu().numpy().tolist()
    log("scale: diagnostics (gap-floor evaluations, non-finite vehicles) = %s" % diag)
    assert diag == [0, 0]
    g = gp.cpu().numpy()[:, idx]
    okg, wg = grad_close(g, ref["g"] * fac)
    ok0, w0 = grad_close(gp0.cpu().numpy()[idx], ref["gp0"] * fac)
    ok1, w1 = grad_close(gv0.cpu().numpy()[idx], ref["gv0"] * fac)
    log("scale sampled: gradient worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1
    assert np.isfinite(loss.item()) and loss.item() > 0
