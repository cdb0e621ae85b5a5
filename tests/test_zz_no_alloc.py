"""The entry point that allocates nothing: idm_sim_backward_noalloc (forward
checkpoints + backward in the library's static device scratch) against
idm_sim_forward + idm_sim_backward on a caller workspace, through the C ABI.
The same kernels run on the same inputs, so every output is bitwise equal;
two calls in a row, the second on a smaller problem, show that the array's
leftover contents from the first call do not leak into the second."""
import numpy as np
import pytest

import scenarios
from _util import oracle_targets, ragged_scenario
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _both(sc, steps, tgt, dense, **plan_kw):
    import torch
    from paper_2412_16750_amd import sim
    plan = sim.Plan.for_scenario(sc, **plan_kw)
    x = device_inputs(sc)
    n, S = sc.n, sc.n_steps
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), int(steps[0]), int(steps[1] - steps[0]))
    gd = torch.from_numpy(dense).cuda()

    def outs():
        return (torch.full((5, n), np.nan, dtype=torch.float64, device="cuda"),
                torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
                torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
                torch.full((1,), np.nan, dtype=torch.float64, device="cuda"))
    ref = outs()
    ws = plan.workspace("cuda")
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], None, None, ws)
    sim.idm_sim_backward(plan, x["prm"], x["length"], x["p0"], x["v"], *ref[:3], ws,
                         grad_traj_d=gd, obs=obs, loss_out=ref[3])
    got = outs()
    sim.idm_sim_backward_noalloc(plan, x["prm"], x["length"], x["p0"], x["v"], *got[:3],
                                 grad_traj_d=gd, obs=obs, loss_out=got[3])
    torch.cuda.synchronize()
    info = plan.info()
    return [r.cpu().numpy() for r in ref], [g.cpu().numpy() for g in got], info


def _case(sizes, n_steps, c, **plan_kw):
    sc = ragged_scenario(sizes, n_steps, seed_c=c, ckpt_every=plan_kw.pop("ckpt_every", 16))
    steps = np.arange(1, n_steps + 1)
    tgt = oracle_targets(sc, steps, c=c)
    dense = np.random.default_rng(c).normal(0, 1e-3, (n_steps + 1, sc.n)).astype(np.float32)
    return sc, steps, tgt, dense, plan_kw


def test_noalloc_matches_workspace_path_twice():
    names = ("grad_params", "grad_p0", "grad_v0", "loss")
    # first call: lanes longer than a bundle (pieces exchange boundary states
    # through the scratch), several checkpoint blocks and a ragged last block
    big = _case([700, 1, 64, 300, 129, 2000], 150, 21, threads=256, per_thread=1, ckpt_every=32)
    # second call: a smaller problem on a different plan
    small = _case([40, 3, 17], 37, 22, threads=64, per_thread=1, ckpt_every=8)
    for what, (sc, steps, tgt, dense, kw) in (("large", big), ("small", small)):
        log("no-alloc %s: N=%d S=%d %s" % (what, sc.n, sc.n_steps, kw))
        ref, got, info = _both(sc, steps, tgt, dense, **kw)
        if what == "large":
            assert info["n_boundaries"] > 0
        for nm, r, g in zip(names, ref, got):
            assert np.all(np.isfinite(r)), (what, nm)
            assert np.array_equal(r, g), (what, nm, float(np.max(np.abs(r - g))))


def test_noalloc_rejects_a_problem_larger_than_the_scratch():
    import torch
    from paper_2412_16750_amd import _lib, sim
    # 1000 lanes x 1000 vehicles, 1000 steps, K = 32: 32 checkpoint blocks of
    # 2 x 4 B per vehicle (256 MB) already exceed the 256 MiB array
    sc = scenarios.make_scenario("big", scenarios.uniform_lanes(1000, 1000), 1000, 2, ckpt_every=32)
    plan = sim.Plan.for_scenario(sc)
    need = plan.workspace_bytes
    log("no-alloc reject: workspace %d bytes" % need)
    assert need > (256 << 20)
    x = device_inputs(sc)
    g = torch.empty(5, sc.n, dtype=torch.float64, device="cuda")
    g0 = torch.empty(sc.n, dtype=torch.float64, device="cuda")
    g1 = torch.empty(sc.n, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.IdmError) as e:
        sim.idm_sim_backward_noalloc(plan, x["prm"], x["length"], x["p0"], x["v"], g, g0, g1)
    assert e.value.status == -4 and "static scratch" in str(e.value)
