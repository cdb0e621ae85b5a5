"""The device-side trajectory fit (idm_fit_init / idm_fit_step / idm_fit_run)
against the oracle's gradient + Adam step, graph replay against eager steps,
and convergence on a small problem."""
import functools

import numpy as np
import pytest

import oracle
import scenarios
from oracle.fit import adam_box_step
from _util import grad_close, ragged_scenario
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu

BOX_LO = np.array([15.0, 0.5, 0.5, 0.5, 0.5])
BOX_HI = np.array([45.0, 3.0, 3.0, 4.0, 5.0])
MID = (BOX_LO + BOX_HI) / 2  # exactly representable, u = 0.5 exactly


def _problem(sizes=(30, 20, 1, 12), S=200, every=10, seed_c=4):
    sc = ragged_scenario(list(sizes), S, ckpt_every=16, seed_c=seed_c)
    steps = np.arange(every, S + 1, every)
    P, _, _, _ = oracle.forward(oracle.Problem.from_scenario(sc))  # hidden parameters
    tgt = (P[steps] + scenarios.noise((len(steps), sc.n), seed_c)).astype(np.float32)
    return sc, steps, tgt


def _fitter(sc, steps, tgt, lr=1e-2, plan_kw=None, **kw):
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd.fit import Fitter
    plan = sim.Plan.for_scenario(sc, **(plan_kw or {}))
    x = device_inputs(sc)
    obs = sim.Obs(torch.from_numpy(tgt).cuda(), int(steps[0]), int(steps[1] - steps[0]))
    f = Fitter(plan, x["length"], x["p0"], x["v"], obs, lr0=lr, **kw)
    return f, x


def _cold(n, values):
    import torch
    return torch.from_numpy(np.repeat(np.asarray(values, np.float32)[:, None], n, axis=1)).cuda()


def test_first_fit_step_matches_oracle_gradient_and_adam():
    sc, steps, tgt = _problem()
    f, x = _fitter(sc, steps, tgt)
    f.init(_cold(sc.n, MID))
    f.step()
    import torch
    torch.cuda.synchronize()
    # oracle: loss and gradient at the box midpoints, then one Adam step
    prm = {k: np.full(sc.n, MID[i], np.float32) for i, k in enumerate(oracle.PARAM_NAMES)}
    prm["length"] = sc.params["length"]
    pb = oracle.Problem.from_scenario(sc, params=prm)
    P, V, _, _ = oracle.forward(pb)
    loss, gP = oracle.mse(P, steps, tgt.astype(np.float64))
    g, _, _ = oracle.adjoint(pb, P, V, gP)
    u0 = np.full((5, sc.n), 0.5)
    u1, m1, v1, th1 = adam_box_step(u0, np.zeros_like(u0), np.zeros_like(u0), g,
                                    BOX_LO[:, None], BOX_HI[:, None], 1, 1e-2)
    l_gpu = f.losses()[0]
    log("fit step 1: loss gpu %.9e oracle %.9e" % (l_gpu, loss))
    assert abs(l_gpu - loss) <= 1e-4 * loss
    ok, w = grad_close(f.m.double().cpu().numpy(), m1)
    log("fit step 1: Adam first moment worst/limit %.3f" % w)
    assert ok
    assert np.max(np.abs(f.u.double().cpu().numpy() - u1)) < 1e-5
    assert np.max(np.abs(f.params.double().cpu().numpy() - th1) / (BOX_HI - BOX_LO)[:, None]) < 1e-5
    assert f.steps_done() == 1


def test_fit_graph_replay_matches_eager_steps():
    """Each replay of the captured fit step is checked against the eager step,
    with eager work and synchronisations between the replays."""
    import torch
    sc, steps, tgt = _problem(seed_c=5)
    f, x = _fitter(sc, steps, tgt)
    cold = _cold(sc.n, [scenarios.COLD_START[k] for k in oracle.PARAM_NAMES])
    f.init(cold)
    eager = []
    for _ in range(6):
        f.step()
        torch.cuda.synchronize()
        eager.append([t.clone() for t in (f.u, f.m, f.v, f.params)] + [f.losses().copy()])
    f.init(cold)
    for i in range(6):
        f.run(1)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        got = [f.u, f.m, f.v, f.params]
        for a, b in zip(got, eager[i][:4]):
            assert torch.equal(a, b), i
        assert np.array_equal(f.losses(), eager[i][4]), i
        del junk
    f.init(cold)
    f.run(6)
    torch.cuda.synchronize()
    assert torch.equal(f.u, eager[-1][0]) and f.steps_done() == 6


def test_fit_reduces_the_loss_within_the_boxes():
    import torch
    sc, steps, tgt = _problem(sizes=(60, 40), S=300, seed_c=6)
    f, x = _fitter(sc, steps, tgt)
    f.init(_cold(sc.n, [scenarios.COLD_START[k] for k in oracle.PARAM_NAMES]))
    f.run(150)
    torch.cuda.synchronize()
    L = f.losses()
    log("fit: loss %.4e -> %.4e over %d steps" % (L[0], L[-1], len(L)))
    assert len(L) == 150 and L[-1] < 0.3 * L[0]
    prm = f.params.double().cpu().numpy()
    assert np.all(prm >= BOX_LO[:, None] - 1e-6) and np.all(prm <= BOX_HI[:, None] + 1e-6)
    u = f.u.cpu().numpy()
    assert u.min() >= 0.0 and u.max() <= 1.0


@pytest.mark.parametrize("raw_units", [False, True])
def test_scheduled_fit_matches_oracle_over_eight_steps(raw_units):
    """Eight fit steps with the learning rate falling linearly from 0.1 to
    0.01 (the schedule of Sec. V-B3) against the oracle's own eight steps from
    the same start: oracle.fit.lr_at for the rate, adam_box_step (Adam on the
    normalised parameters) or adam_raw_step (Adam on the parameters in their
    own units, Sec. IV-A) for the update, the oracle's loss and adjoint for
    the gradient.  The loss history agrees step by step, and the first step's
    moments element by element."""
    import torch
    from oracle.fit import adam_raw_step, lr_at
    sc, steps, tgt = _problem(seed_c=7)
    lr0, lr1, n = 0.1, 0.01, 8
    f, x = _fitter(sc, steps, tgt, lr=lr0, lr1=lr1, lr_steps=n, raw_units=raw_units)
    f.init(_cold(sc.n, MID))
    moments = None
    for t in range(n):
        f.step()
        if t == 0:
            torch.cuda.synchronize()
            moments = (f.m.double().cpu().numpy(), f.v.double().cpu().numpy(),
                       f.params.double().cpu().numpy())
    torch.cuda.synchronize()
    L_gpu = f.losses()
    lo, hi = BOX_LO[:, None], BOX_HI[:, None]
    th = np.repeat(MID[:, None], sc.n, axis=1).astype(np.float64)
    u = (th - lo) / (hi - lo)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L_or = []
    for t in range(1, n + 1):
        prm = {k: th[i] for i, k in enumerate(oracle.PARAM_NAMES)}
        prm["length"] = sc.params["length"]
        pb = oracle.Problem.from_scenario(sc, params=prm)
        P, V, _, _ = oracle.forward(pb)
        loss, gP = oracle.mse(P, steps, tgt.astype(np.float64))
        g, _, _ = oracle.adjoint(pb, P, V, gP)
        L_or.append(loss)
        lr = lr_at(t, lr0, lr1, n)
        if raw_units:
            th, m, v = adam_raw_step(th, m, v, g, lo, hi, t, lr)
        else:
            u, m, v, th = adam_box_step(u, m, v, g, lo, hi, t, lr)
        if t == 1:
            ok_m, w_m = grad_close(moments[0], m)
            ok_v, w_v = grad_close(moments[1], v)
            d_th = float(np.max(np.abs(moments[2] - th) / (hi - lo)))
            log("scheduled fit raw=%s step 1: moments worst/limit %.3f %.3f, params %.2e of the box"
                % (raw_units, w_m, w_v, d_th))
            assert ok_m and ok_v and d_th < 1e-5
    L_or = np.asarray(L_or)
    rel = np.abs(L_gpu - L_or) / L_or
    log("scheduled fit raw=%s: loss gpu %s oracle %s, max rel %.2e"
        % (raw_units, np.array2string(L_gpu, precision=5), np.array2string(L_or, precision=5),
           rel.max()))
    assert len(L_gpu) == n and rel.max() <= 1e-3
    assert L_or[-1] < L_or[0]
    # the rate really falls: the oracle's schedule reaches lr1 on the last step
    assert lr_at(n + 1, lr0, lr1, n) == pytest.approx(lr1) and lr_at(1, lr0, lr1, n) == lr0


@functools.lru_cache(maxsize=1)
def _full_fit_reference():
    """The oracle's side of the full fit workload test: the Adam first moment
    after one step from the box midpoints on three sampled lanes, and the loss
    over all 100,000 vehicles."""
    sc = scenarios.fit()
    steps = scenarios.obs_steps(sc.n_steps, sc.extra["obs_first"], sc.extra["obs_stride"])
    tgt = scenarios.constant_speed_targets(sc, steps, 44)
    lanes = [0, 57, 99]
    sub = scenarios.subset_lanes(sc, lanes)
    idx = sub.extra["vehicle_index"]
    prm = {k: np.full(sub.n, MID[i], np.float32) for i, k in enumerate(oracle.PARAM_NAMES)}
    prm["length"] = sub.params["length"]
    pb = oracle.Problem.from_scenario(sub, params=prm)
    P, V, _, _ = oracle.forward(pb)
    _, gP = oracle.mse(P, steps, tgt[:, idx].astype(np.float64))
    g, _, _ = oracle.adjoint(pb, P, V, gP)
    fac = sub.n / sc.n  # the loss is normalised over all N vehicles
    m_ref = 0.1 * g * fac * (BOX_HI - BOX_LO)[:, None]
    prm_all = {k: np.full(sc.n, MID[i], np.float32) for i, k in enumerate(oracle.PARAM_NAMES)}
    prm_all["length"] = sc.params["length"]
    P_all, _, _, _ = oracle.forward(oracle.Problem.from_scenario(sc, params=prm_all))
    loss_all, _ = oracle.mse(P_all, steps, tgt.astype(np.float64))
    return sc, steps, tgt, lanes, idx, m_ref, loss_all


@pytest.mark.parametrize("plan_kw", [
    {},
    dict(store_states=True, threads=640, per_thread=1, tile_steps=256),
    dict(store_states=True, threads=256, per_thread=1, tile_steps=64)],
    ids=["checkpoints", "tiles640x256", "tiles256x64"])
def test_first_fit_step_on_the_full_fit_workload_sampled_lanes(plan_kw):
    """The fit workload at full size (100 lanes x 1000 vehicles, 500 steps,
    observed every 10th step) in the launch configurations the benchmark times
    (the default plan, and the halo tiles its autotuner picks among): after
    one fit step from the box midpoints, the Adam first moment of three
    sampled lanes equals (1 - beta1) times the oracle's gradient of the same
    loss (normalised over all 100,000 vehicles), element by element, and the
    loss matches."""
    import torch
    sc, steps, tgt, lanes, idx, m_ref, loss_all = _full_fit_reference()
    f, x = _fitter(sc, steps, tgt, plan_kw=plan_kw)
    f.init(_cold(sc.n, MID))
    f.step()
    torch.cuda.synchronize()
    m_gpu = f.m.double().cpu().numpy()[:, idx]
    ok, w = grad_close(m_gpu, m_ref)
    log("full fit workload %s, step 1: Adam first moment on lanes %s worst/limit %.3f"
        % (plan_kw, lanes, w))
    assert ok
    log("full fit workload %s, step 1: loss gpu %.9e oracle %.9e" % (plan_kw, f.losses()[0],
                                                                    loss_all))
    assert abs(f.losses()[0] - loss_all) <= 1e-4 * loss_all
