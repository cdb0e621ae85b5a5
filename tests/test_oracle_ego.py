"""Pins of the ego-only reconstruction oracle (Sec. IV-A): per-step free gap
G and speed difference D, p(0) = 0, summed absolute error.  Each test checks
the oracle against something other than itself: central differences, the
tangent-linear model, a closed-form equilibrium, the lane model's head and
two-vehicle lanes, and hand-computed losses."""
import numpy as np
import pytest

import oracle

MODES = [oracle.MODE_SOFTPLUS, oracle.MODE_CLAMP]


def _problem(n=3, S=40, mode=oracle.MODE_SOFTPLUS, seed=0, dt=0.5):
    rng = np.random.default_rng(seed)
    pr = dict(v0=rng.uniform(25, 35, n), T=rng.uniform(1, 2, n), a=rng.uniform(1, 2, n),
              b=rng.uniform(1.5, 3, n), s0=rng.uniform(1.5, 3, n))
    G = rng.uniform(15, 40, (S, n))
    D = rng.normal(0, 1.5, (S, n))
    v = rng.uniform(12, 22, n)
    return oracle.EgoProblem(pr, G, D, v, S, dt=dt, mode=mode)


def _loss(pb, W):
    P, _, _, _ = oracle.ego_forward(pb)
    return float(np.sum(W * P))


def _perturbed(pb, what, idx, h):
    pr = {k: v.copy() for k, v in pb.params.items()}
    G, D, v = pb.G.copy(), pb.D.copy(), pb.v_init.copy()
    if what in pr:
        pr[what][idx] += h
    elif what == "G":
        G[idx] += h
    elif what == "D":
        D[idx] += h
    else:
        v[idx] += h
    return oracle.EgoProblem(pr, G, D, v, pb.n_steps, pb.dt, pb.delta, pb.a_min, pb.gap_floor, pb.mode)


@pytest.mark.parametrize("mode", MODES)
def test_ego_adjoint_matches_central_differences(mode):
    pb = _problem(mode=mode)
    rng = np.random.default_rng(1)
    W = rng.normal(0, 1, (pb.n_steps + 1, pb.n))
    P, V, _, hits = oracle.ego_forward(pb)
    assert hits == 0 and V.min() > 0.5   # smooth region: no floor, no clamp
    g, gG, gD, gv0 = oracle.ego_adjoint(pb, P, V, W)
    checks = [(k, i, g[j, i]) for j, k in enumerate(oracle.PARAM_NAMES) for i in range(pb.n)]
    for (k, i) in [(0, 0), (5, 1), (17, 2), (39, 0), (22, 1)]:
        checks.append(("G", (k, i), gG[k, i]))
        checks.append(("D", (k, i), gD[k, i]))
    checks += [("v", i, gv0[i]) for i in range(pb.n)]
    for what, idx, got in checks:
        base = pb.params[what][idx] if what in pb.params else (
            pb.G[idx] if what == "G" else pb.D[idx] if what == "D" else pb.v_init[idx])
        h = 1e-6 * max(abs(base), 1.0)
        fd = (_loss(_perturbed(pb, what, idx, h), W) - _loss(_perturbed(pb, what, idx, -h), W)) / (2 * h)
        assert abs(got - fd) <= 1e-6 * max(abs(fd), 1.0), (what, idx, got, fd)


@pytest.mark.parametrize("mode", MODES)
def test_ego_adjoint_is_transpose_of_tangent(mode):
    pb = _problem(n=4, S=60, mode=mode, seed=3)
    rng = np.random.default_rng(4)
    P, V, _, _ = oracle.ego_forward(pb)
    W = rng.normal(0, 1, P.shape)
    dprm = rng.normal(0, 1, (5, pb.n))
    dG = rng.normal(0, 1, pb.G.shape)
    dD = rng.normal(0, 1, pb.D.shape)
    dv0 = rng.normal(0, 1, pb.n)
    dP, _ = oracle.ego_tangent(pb, V, dprm, dG, dD, dv0)
    g, gG, gD, gv0 = oracle.ego_adjoint(pb, P, V, W)
    lhs = float(np.sum(W * dP))
    rhs = float(np.sum(g * dprm) + np.sum(gG * dG) + np.sum(gD * dD) + np.sum(gv0 * dv0))
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("mode", MODES)
def test_ego_equilibrium_gap_is_stationary(mode):
    """With D = 0 and the gap at which the bounded acceleration vanishes, the
    speed stays put and the position grows linearly.  CLAMP: G = (s0 + V T) /
    sqrt(1 - (V/v0)^4); SOFTPLUS: G = softplus(s0 + V T) /
    sqrt(1 - (V/v0)^4 - ln(1 - e^a_min) / a) (a_min binds while V/dt > -a_min)."""
    n, S, dt = 4, 100, 1.0
    v0, T, a, b, s0 = np.full(n, 30.0), np.array([1.0, 1.3, 1.7, 2.0]), np.full(n, 1.5), \
        np.full(n, 2.0), np.full(n, 2.0)
    V0 = np.array([12.0, 16.0, 20.0, 25.0])
    x4 = (V0 / v0) ** 4
    s = s0 + V0 * T
    if mode == oracle.MODE_CLAMP:
        gap = s / np.sqrt(1 - x4)
    else:
        s = np.log1p(np.exp(s))
        gap = s / np.sqrt(1 - x4 - np.log1p(-np.exp(-10.0)) / a)
    pb = oracle.EgoProblem(dict(v0=v0, T=T, a=a, b=b, s0=s0), np.tile(gap, (S, 1)),
                           np.zeros((S, n)), V0, S, dt=dt, mode=mode)
    P, V, A, _ = oracle.ego_forward(pb, want_acc=True)
    assert np.max(np.abs(V - V0)) < 1e-9
    assert np.max(np.abs(A)) < 1e-10
    assert np.allclose(P, np.arange(S + 1)[:, None] * dt * V0, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("mode", MODES)
def test_ego_without_leader_influence_is_the_lane_head(mode):
    """A gap of 1e12 m removes the interaction term up to rounding: the ego
    trajectory is the lane model's free-road head."""
    pb = _problem(n=5, S=80, mode=mode, seed=7)
    G = np.full_like(pb.G, 1e12)
    ego = oracle.EgoProblem(pb.params, G, pb.D, pb.v_init, pb.n_steps, pb.dt, mode=mode)
    P, V, _, _ = oracle.ego_forward(ego)
    params = dict(pb.params, length=np.full(pb.n, 5.0))
    lane = oracle.Problem(np.arange(pb.n + 1), params, np.zeros(pb.n), pb.v_init, pb.n_steps,
                          dt=pb.dt, mode=mode)
    P2, V2, _, _ = oracle.forward(lane)
    assert np.allclose(V, V2, rtol=1e-12, atol=1e-12)
    assert np.allclose(P, P2, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("mode", MODES)
def test_ego_step_is_the_follower_of_a_two_vehicle_lane(mode):
    """One step: the ego with gap G and speed difference D accelerates like the
    follower of a lane whose leader (length 5 m) stands G + 5 m ahead with
    speed v - D."""
    rng = np.random.default_rng(9)
    n = 6
    pr = dict(v0=rng.uniform(25, 35, n), T=rng.uniform(1, 2, n), a=rng.uniform(1, 2, n),
              b=rng.uniform(1.5, 3, n), s0=rng.uniform(1.5, 3, n))
    G = rng.uniform(3, 40, (1, n))
    D = rng.normal(0, 3, (1, n))
    v = rng.uniform(5, 25, n)
    P, V, _, _ = oracle.ego_forward(oracle.EgoProblem(pr, G, D, v, 1, dt=0.1, mode=mode))
    # lanes of two: leader first (its own parameters are irrelevant to the follower)
    off = np.arange(0, 2 * n + 1, 2)
    lp = {k: np.repeat(pr[k], 2) for k in pr}
    lp["length"] = np.full(2 * n, 5.0)
    p0 = np.zeros(2 * n)
    p0[0::2] = G[0] + 5.0
    vi = np.zeros(2 * n)
    vi[0::2] = v - D[0]
    vi[1::2] = v
    P2, V2, _, _ = oracle.forward(oracle.Problem(off, lp, p0, vi, 1, dt=0.1, mode=mode))
    assert np.allclose(V[1], V2[1, 1::2], rtol=1e-13, atol=1e-13)


def test_ego_mae_hand_example():
    P = np.array([[0.0, 0.0], [1.0, 2.0], [3.0, 5.0]])  # [S+1 = 3, N = 2]
    off = [0, 3, 5]
    steps = [1, 2, 2, 0, 2]            # trajectory 0: steps 1, 2, 2; trajectory 1: 0, 2
    pos = [1.5, 3.0, 2.0, -1.0, 6.5]
    loss, gP = oracle.ego_mae(P, off, steps, pos)
    # |1-1.5| + |3-3| + |3-2| + |0-(-1)| + |5-6.5| = 0.5 + 0 + 1 + 1 + 1.5
    assert loss == pytest.approx(4.0, abs=1e-15)
    expect = np.zeros_like(P)
    expect[1, 0] = -1.0      # 1 < 1.5
    expect[2, 0] = 0.0 + 1.0  # tie contributes 0, 3 > 2 contributes +1
    expect[0, 1] = 1.0       # 0 > -1
    expect[2, 1] = -1.0      # 5 < 6.5
    assert np.array_equal(gP, expect)


def test_ego_mae_gradient_is_the_derivative_away_from_ties():
    rng = np.random.default_rng(2)
    S, n = 30, 5
    P = rng.normal(0, 10, (S + 1, n))
    counts = rng.integers(0, 6, n)
    off = np.concatenate([[0], np.cumsum(counts)])
    steps = np.concatenate([np.sort(rng.integers(0, S + 1, c)) for c in counts]).astype(np.int32)
    pos = rng.normal(0, 10, len(steps))
    loss, gP = oracle.ego_mae(P, off, steps, pos)
    h = 1e-7
    for k in range(S + 1):
        for i in range(n):
            Pp, Pm = P.copy(), P.copy()
            Pp[k, i] += h
            Pm[k, i] -= h
            fd = (oracle.ego_mae(Pp, off, steps, pos, False)[0] -
                  oracle.ego_mae(Pm, off, steps, pos, False)[0]) / (2 * h)
            assert abs(fd - gP[k, i]) < 1e-6


def test_raw_adam_first_step_projection_and_quadratic():
    from oracle.fit import adam_raw_step, lr_at
    x = np.array([1.0, 5.0, -3.0])
    g = np.array([2.0, -0.5, 1e3])
    lo, hi = np.array([0.0, -np.inf, -3.05]), np.array([10.0, 5.02, np.inf])
    x1, m, v = adam_raw_step(x, np.zeros(3), np.zeros(3), g, lo, hi, 1, 0.1)
    # first step moves every coordinate by lr against the gradient's sign ...
    assert np.allclose(x1[:1], [0.9], rtol=0, atol=1e-7)
    # ... then projects: 5.1 -> 5.02 and -3.1 -> -3.05
    assert x1[1] == 5.02 and x1[2] == -3.05
    # the schedule: 0.1 at step 1, 0.01 from step 501 on
    assert lr_at(1, 0.1, 0.01, 500) == 0.1 and lr_at(501, 0.1, 0.01, 500) == pytest.approx(0.01)
    # minimises a box-constrained quadratic: argmin of (x - 3)^2 on [0, 2] is 2
    x, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        x, m, v = adam_raw_step(x, m, v, 2 * (x - 3.0), 0.0, 2.0, t, lr_at(t, 0.1, 0.01, 500))
    assert x[0] == 2.0


def test_reconstruction_metrics_hand_example():
    # two trajectories, S = 4; trajectory 1 has no observation
    P = np.zeros((5, 2))
    P[:, 0] = [0.0, 10.0, 20.0, 30.0, 40.0]
    A = np.zeros((4, 2))
    A[:, 0] = [1.0, -3.0, 11.0, 2.0]
    A[:, 1] = [50.0, 50.0, 50.0, 50.0]
    off = [0, 3, 3]
    steps = [0, 2, 3]
    pos = [0.0, 21.0, 28.0]
    m = oracle.reconstruction_metrics(P, A, off, steps, pos)
    # length 28 - 0 = 28 m; errors 0, 1, 2 -> mean 3 / (3 * 28)
    assert m["pos_error"] == pytest.approx(3.0 / 84.0)
    # steps before the last observed step (3): |a| = 1, 3, 11
    assert m["acc_mean"] == pytest.approx(5.0)
    assert m["acc_std"] == pytest.approx(np.std([1.0, 3.0, 11.0]))
    # trajectory 0 exceeds 10 m/s^2 once; trajectory 1 has no observed span
    assert m["implausible"] == pytest.approx(0.5)
