"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the mathematical fact) it checks,
and is built so that a plausible slip in the oracle (a dropped term, a wrong
sign or index, the follower's length instead of the leader's, a semi-implicit
Euler step) makes at least one of them fail.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from oracle import MODE_CLAMP, MODE_SOFTPLUS, Problem

pytestmark = pytest.mark.usefixtures("oracle_lib")


def lane_problem(n_steps, v0, T, a, b, s0, length, p0, v_init, mode, dt=0.1, delta=4.0,
                 a_min=-10.0, gap_floor=1e-3, lane_offsets=None):
    n = len(v0)
    off = [0, n] if lane_offsets is None else lane_offsets
    prm = dict(v0=v0, T=T, a=a, b=b, s0=s0, length=length)
    return Problem(off, prm, p0, v_init, n_steps, dt, delta, a_min, gap_floor, mode)


def single(n_steps, v0, a, v_init, mode, dt=0.1, delta=4.0, **kw):
    return lane_problem(n_steps, [v0], [1.5], [a], [2.0], [2.0], [5.0], [0.0], [v_init], mode,
                        dt=dt, delta=delta, **kw)


# ---------------------------------------------------------------- free road

def test_free_road_delta1_matches_discrete_closed_form():
    """Eq. 2 with no leader and delta = 1 plus Eq. 3 is the linear recursion
    v' = v (1 - a dt / v0) + a dt, whose exact solution is
    v_k = v0 + (v_init - v0) r^k, r = 1 - a dt / v0, and
    p_k = p_0 + dt * sum_{j<k} v_j (closed-form geometric sum)."""
    v0, a, vi, dt, S = 30.0, 1.7, 12.0, 0.1, 400
    pb = single(S, v0, a, vi, MODE_CLAMP, dt=dt, delta=1.0)
    P, V, _, _ = oracle.forward(pb)
    r = 1.0 - a * dt / v0
    k = np.arange(S + 1)
    v_exact = v0 + (vi - v0) * r ** k
    p_exact = dt * (k * v0 + (vi - v0) * (1.0 - r ** k) / (1.0 - r))
    np.testing.assert_allclose(V[:, 0], v_exact, rtol=1e-12)
    np.testing.assert_allclose(P[:, 0], p_exact, rtol=1e-11, atol=1e-10)


def _ode_time(v, vi, v0, a):
    """Closed-form time to go from vi to v under dv/dt = a (1 - (v/v0)^4):
    t = v0 / (2a) * [artanh(u) + arctan(u)] between u0 = vi/v0 and u = v/v0."""
    F = lambda u: math.atanh(u) + math.atan(u)
    return v0 / (2 * a) * (F(v / v0) - F(vi / v0))


def test_free_road_delta4_converges_to_ode_at_first_order():
    """Explicit Euler (Eq. 3) on the free-road IDM (Eq. 2, delta = 4) is a
    first-order method: halving dt halves the error against the ODE solution."""
    v0, a, vi, t_end = 30.0, 1.5, 10.0, 20.0
    v_true = brentq(lambda v: _ode_time(v, vi, v0, a) - t_end, vi, v0 * (1 - 1e-15))
    errs, finals = [], []
    for dt in (0.1, 0.05, 0.025, 0.0125):
        S = int(round(t_end / dt))
        P, V, _, _ = oracle.forward(single(S, v0, a, vi, MODE_CLAMP, dt=dt))
        finals.append(V[-1, 0])
        errs.append(abs(V[-1, 0] - v_true))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(1.9 < r < 2.1 for r in ratios), (errs, ratios)
    # Richardson extrapolation removes the O(dt) term: what is left is O(dt^2)
    rich = 2 * finals[-1] - finals[-2]
    assert abs(rich - v_true) < 0.02 * errs[-1]


def test_free_road_clamp_fixed_point_is_v0_bitwise():
    """At v = v0 the free-road acceleration of Eq. 2 is exactly zero."""
    P, V, _, _ = oracle.forward(single(500, 27.25, 1.3, 27.25, MODE_CLAMP))
    assert np.all(V[:, 0] == 27.25)
    np.testing.assert_allclose(P[-1, 0], 500 * 0.1 * 27.25, rtol=1e-14)


@pytest.mark.parametrize("a", [1.0, 2.0])
def test_free_road_softplus_fixed_point(a):
    """Sec. III-C: with a_lb = a_min (v > -a_min dt), a* = 0 needs
    softplus(ahat - a_min) = -a_min, i.e. ahat = ln(1 - e^{a_min}), so the free
    road speed settles at v* = v0 (1 - ln(1 - e^{a_min}) / a)^{1/4}."""
    v0, a_min = 30.0, -10.0
    v_star = v0 * (1.0 - math.log(1.0 - math.exp(a_min)) / a) ** 0.25
    P, V, _, _ = oracle.forward(single(6000, v0, a, 20.0, MODE_SOFTPLUS))
    assert abs(V[-1, 0] - v_star) < 1e-9 * v_star
    assert v_star > v0  # the softplus bound lets the head exceed v0 slightly


# ---------------------------------------------------------------- platoons

def _platoon(mode, n=8, S=1000):
    """Open lane whose head drives at its fixed-point speed V and whose
    followers sit at the equilibrium gap for speed V (Eqs. 1-2 with dv = 0):
      CLAMP:    s_e = (s0 + V T) / sqrt(1 - (V/v0)^4)
      SOFTPLUS: s_e = softplus(s0 + V T) / sqrt(1 - (V/v0)^4 - ln(1 - e^{a_min}) / a)
    Lengths differ per vehicle: the gap is measured to the LEADER's rear,
    p_h - p_i - length_h (Sec. III-A)."""
    rng = np.random.default_rng(7)
    v0 = rng.uniform(32, 40, n)
    v0[0] = 24.0
    T = rng.uniform(1, 2, n)
    a = rng.uniform(1, 2, n)
    b = rng.uniform(1.5, 3, n)
    s0 = rng.uniform(1.5, 3, n)
    length = rng.uniform(3.5, 12.0, n)
    a_min = -10.0
    cm = math.log(1.0 - math.exp(a_min))
    if mode == MODE_CLAMP:
        V = v0[0]
    else:
        V = v0[0] * (1.0 - cm / a[0]) ** 0.25
    p = np.zeros(n)
    for i in range(1, n):
        x4 = (V / v0[i]) ** 4
        if mode == MODE_CLAMP:
            s_e = (s0[i] + V * T[i]) / math.sqrt(1.0 - x4)
        else:
            sopt = s0[i] + V * T[i]
            sp = sopt + math.log1p(math.exp(-sopt))
            s_e = sp / math.sqrt(1.0 - x4 - cm / a[i])
        p[i] = p[i - 1] - length[i - 1] - s_e
    p -= p[-1]
    pb = lane_problem(S, v0, T, a, b, s0, length, p, np.full(n, V), mode, a_min=a_min)
    return pb, V


@pytest.mark.parametrize("mode", [MODE_CLAMP, MODE_SOFTPLUS])
def test_equilibrium_platoon_is_stationary(mode):
    pb, V = _platoon(mode)
    P, Vt, _, _ = oracle.forward(pb)
    assert np.max(np.abs(Vt - V)) < 1e-9
    gaps0 = P[0, :-1] - P[0, 1:]
    gapsS = P[-1, :-1] - P[-1, 1:]
    np.testing.assert_allclose(gapsS, gaps0, atol=1e-8)


def test_equilibrium_breaks_with_follower_length():
    """Control for the test above: measuring the gap with the follower's own
    length (a plausible slip) gives a platoon that is NOT stationary."""
    pb, V = _platoon(MODE_CLAMP)
    n = pb.n
    # shift every follower so that the gap would be right if own length were used
    p = pb.p0.copy()
    for i in range(1, n):
        p[i:] += pb.length[i - 1] - pb.length[i]
    pb2 = Problem(pb.lane_offsets, dict(pb.params, length=pb.length), p, pb.v_init, pb.n_steps,
                  mode=MODE_CLAMP)
    _, Vt, _, _ = oracle.forward(pb2)
    assert np.max(np.abs(Vt - V)) > 1e-3


# ---------------------------------------------------------------- one-step cases

@pytest.mark.parametrize("gap_factor, expected_ahat", [(1.0, 0.0), (2.0, 0.75), (0.5, -3.0)])
def test_matched_gap_interaction(gap_factor, expected_ahat):
    """Eqs. 1-2 with v0 -> infinity: if the gap is gap_factor * s_opt, then
    ahat = a (1 - 1/gap_factor^2).  Numbers: follower v = 10, leader speed 4
    (dv = +6, closing), a = 1, b = 4 (sqrt(ab) = 2), s0 = 2, T = 1, so
    s_opt = 2 + 10 + 10*6/(2*2) = 27.  The leader is 5 m long, the follower
    7 m.  A sign slip in dv gives s_opt = -3, a dropped 2 gives 42, the
    follower's length shifts the gap by 2 m: each changes the result."""
    s_opt = 27.0
    gap = gap_factor * s_opt
    v0 = [1e9, 1e9]
    p = [gap + 5.0, 0.0]
    pb = lane_problem(1, v0, [1.0, 1.0], [1.0, 1.0], [4.0, 4.0], [2.0, 2.0], [5.0, 7.0], p,
                      [4.0, 10.0], MODE_CLAMP)
    P, V, A, _ = oracle.forward(pb, want_acc=True)
    assert abs(A[0, 1] - expected_ahat) < 1e-9
    assert abs(V[1, 1] - (10.0 + 0.1 * expected_ahat)) < 1e-10
    assert P[1, 1] == 0.0 + 0.1 * 10.0          # position uses the OLD speed (Eq. 3)


def test_softplus_bound_offsets_zero_acceleration():
    """Sec. III-C: a* = a_lb + softplus(ahat - a_lb).  With ahat = 0 and
    a_lb = a_min = -10 this is ln(1 + e^{-10}) (the bound never returns
    exactly zero), and for very negative ahat a* tends to a_min."""
    p = [27.0 + 5.0, 0.0]
    pb = lane_problem(1, [1e9, 1e9], [1.0, 1.0], [1.0, 1.0], [4.0, 4.0], [2.0, 2.0],
                      [5.0, 7.0], p, [4.0, 10.0], MODE_SOFTPLUS)
    _, _, A, _ = oracle.forward(pb, want_acc=True)
    # softplus(27) differs from 27 by ~1.9e-12: its effect on ahat is below 1e-10
    assert abs(A[0, 1] - math.log1p(math.exp(-10.0))) < 1e-10
    # hard braking: tiny gap, fast follower
    pb2 = lane_problem(1, [30, 30], [1.5, 1.5], [1.5, 1.5], [2, 2], [2, 2], [5, 5],
                       [7.0, 0.0], [0.0, 30.0], MODE_SOFTPLUS)
    _, _, A2, _ = oracle.forward(pb2, want_acc=True)
    assert -10.0 <= A2[0, 1] < -10.0 + 1e-9


def test_lower_bound_switches_to_minus_v_over_dt():
    """Sec. III-C: a_lb = max(-v/dt, a_min): a slow vehicle (v = 0.3 m/s,
    dt = 0.1, so -v/dt = -3 > -10) facing a wall cannot decelerate below
    -v/dt, so its next speed is dt * softplus(ahat + 3) > 0."""
    pb = lane_problem(1, [30, 30], [1.5, 1.5], [1.5, 1.5], [2, 2], [2, 2], [5, 5],
                      [5.5, 0.0], [0.0, 0.3], MODE_SOFTPLUS)
    P, V, A, _ = oracle.forward(pb, want_acc=True)
    assert -3.0 < A[0, 1] < -3.0 + 1e-6
    assert 0.0 < V[1, 1] < 1e-6


def test_dimensional_scaling_clamp_bitwise():
    """IDM is dimensionally consistent: scaling lengths by 2 and times by 2
    (speeds unchanged, accelerations halved) maps every trajectory to twice
    itself.  Powers of two make this exact, so the check is bitwise; a term
    with the wrong dimension (e.g. a*b instead of sqrt(a*b)) breaks it."""
    rng = np.random.default_rng(3)
    n, S = 12, 300
    v0 = rng.uniform(25, 35, n); T = rng.uniform(1, 2, n); a = rng.uniform(1, 2, n)
    b = rng.uniform(1.5, 3, n); s0 = rng.uniform(1.5, 3, n); ln = rng.uniform(4, 6, n)
    gaps = rng.uniform(8, 30, n); vi = rng.uniform(5, 25, n)
    p = np.zeros(n)
    for i in range(n - 2, -1, -1):
        p[i] = p[i + 1] + gaps[i + 1] + ln[i]
    pb = lane_problem(S, v0, T, a, b, s0, ln, p, vi, MODE_CLAMP)
    pb2 = lane_problem(S, v0, 2 * T, a / 2, b / 2, 2 * s0, 2 * ln, 2 * p, vi, MODE_CLAMP,
                       dt=0.2, gap_floor=2e-3)
    P, V, _, _ = oracle.forward(pb)
    P2, V2, _, _ = oracle.forward(pb2)
    assert np.array_equal(P2, 2 * P)
    assert np.array_equal(V2, V)


# ---------------------------------------------------------------- invariants

def _harsh(mode, n=40, S=300, seed=11):
    rng = np.random.default_rng(seed)
    v0 = rng.uniform(25, 35, n); T = rng.uniform(1, 2, n); a = rng.uniform(1, 2, n)
    b = rng.uniform(1.5, 3, n); s0 = rng.uniform(1.5, 3, n); ln = np.full(n, 5.0)
    gaps = rng.uniform(3, 12, n); vi = rng.uniform(0, 30, n)
    vi[0] = 0.0  # a stopped head
    p = np.zeros(n)
    for i in range(n - 2, -1, -1):
        p[i] = p[i + 1] + gaps[i + 1] + ln[i]
    return lane_problem(S, v0, T, a, b, s0, ln, p, vi, mode)


def test_softplus_keeps_speed_nonnegative_and_accel_bounded():
    """Sec. III-C: v >= 0 by construction, and a* >= a_lb >= a_min = -10; and
    a* <= a + ln 2 < 10 (a_max <= 2 here), so every |a| <= 10 (Sec. V-B's
    physical-validity criterion)."""
    pb = _harsh(MODE_SOFTPLUS)
    P, V, A, _ = oracle.forward(pb, want_acc=True)
    assert V.min() >= -1e-12
    assert A.min() >= -10.0 - 1e-12
    assert A.max() <= 2.0 + math.log(2.0)


def test_clamp_keeps_speed_nonnegative():
    pb = _harsh(MODE_CLAMP)
    _, V, _, _ = oracle.forward(pb)
    assert V.min() == 0.0 or V.min() > 0.0


def test_kinematic_identity():
    """Eq. 3: p_S = p_0 + dt * sum_{k<S} v_k (positions use the old speed)."""
    for mode in (MODE_SOFTPLUS, MODE_CLAMP):
        pb = _harsh(mode)
        P, V, _, _ = oracle.forward(pb)
        np.testing.assert_allclose(P[-1], P[0] + pb.dt * V[:-1].sum(axis=0), rtol=1e-12, atol=1e-9)


def test_causality_bitwise():
    """Sec. III-A: a vehicle reacts only to the vehicle directly ahead, so
    perturbing vehicle j's parameters leaves vehicles 0..j-1 bitwise unchanged,
    and changes vehicle j."""
    for mode in (MODE_SOFTPLUS, MODE_CLAMP):
        pb = _harsh(mode)
        P, V, _, _ = oracle.forward(pb)
        j = 17
        pb.params["T"][j] *= 1.3
        pb.params["v0"][j] *= 0.9
        P2, V2, _, _ = oracle.forward(pb)
        assert np.array_equal(P2[:, :j], P[:, :j])
        assert np.array_equal(V2[:, :j], V[:, :j])
        assert not np.array_equal(P2[:, j], P[:, j])


def _sub_lane(pb, P, V, first, last, k0, steps):
    """Vehicles first..last-1 of a one-lane problem as a lane of their own
    (the first one driving on a free road), started from the full run's
    exact states at step k0."""
    idx = np.arange(first, last)
    prm = {k: pb.params[k][idx] for k in pb.params}
    prm["length"] = pb.length[idx]
    return Problem([0, len(idx)], prm, P[k0, idx], V[k0, idx], steps, pb.dt, pb.delta, pb.a_min,
                   pb.gap_floor, pb.mode)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
@pytest.mark.parametrize("J", [1, 2, 3, 6])
def test_information_moves_one_vehicle_per_step(mode, J):
    """Sec. III-B's synchronous update (each vehicle's next state from its own
    and its leader's current state, Eqs. 1-3) moves information one vehicle
    per step: the reading the halo tiles rest on.  Forward: a sub-lane started
    from the exact states at step k0 with J vehicles ahead of the owned ones
    keeps the owned ones bitwise exact for J steps; with J - 1 the first owned
    vehicle is exact through step J - 1 and wrong at step J.  Backward (the
    last J steps, upstream gradients on every step's positions and speeds):
    with J + 1 vehicles ahead and J behind, the owned vehicles' adjoints at k0
    and parameter gradients equal the full lane's bit for bit; with J - 1
    behind the last owned vehicle's do not (a follower reaches its leader
    through its speed adjoint, so the speed upstream makes the bound tight)."""
    import scenarios
    # free flow (the single-lane workload's draws: gaps 20-40 m), where every
    # coupling is far from vanishing in FP64; a stop-and-go queue braking at
    # the bound has speed derivatives below FP64 resolution
    pb = Problem.from_scenario(scenarios.single_lane(n_vehicles=40, n_steps=30, mode=mode))
    P, V, _, _ = oracle.forward(pb)
    a, b, k0 = 18, 24, 12
    Ps, Vs, _, _ = oracle.forward(_sub_lane(pb, P, V, a - J, b, k0, J))
    assert np.array_equal(Ps[:, J:], P[k0:k0 + J + 1, a:b])
    assert np.array_equal(Vs[:, J:], V[k0:k0 + J + 1, a:b])
    Ps, Vs, _, _ = oracle.forward(_sub_lane(pb, P, V, a - J + 1, b, k0, J))
    assert np.array_equal(Vs[:J, J - 1], V[k0:k0 + J, a])
    assert Vs[J, J - 1] != V[k0 + J, a]
    # backward over the last J steps of the run
    S = pb.n_steps
    k1 = S - J
    rng = np.random.default_rng(5)
    gP = rng.normal(0.0, 1.0, (J + 1, pb.n))
    gV = rng.normal(0.0, 1.0, (J + 1, pb.n))
    tail = _sub_lane(pb, P, V, 0, pb.n, k1, J)
    g, gp0, gv0 = oracle.adjoint(tail, P[k1:], V[k1:], gP, gV)

    def sub_adjoint(behind):
        lo, hi = a - J - 1, min(pb.n, b + behind)
        sp = _sub_lane(pb, P, V, lo, hi, k1, J)
        Ps, Vs, _, _ = oracle.forward(sp)
        return oracle.adjoint(sp, Ps, Vs, gP[:, lo:hi], gV[:, lo:hi]), a - lo

    (gs, gp0s, gv0s), off = sub_adjoint(J)
    own = slice(off, off + b - a)
    assert np.array_equal(gp0s[own], gp0[a:b]) and np.array_equal(gv0s[own], gv0[a:b])
    assert np.array_equal(gs[:, own], g[:, a:b])
    (gs, gp0s, gv0s), off = sub_adjoint(J - 1)
    assert gv0s[off + b - a - 1] != gv0[b - 1]


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_halo_tiles_reproduce_the_lane_oracle(mode):
    """The halo-tile scheme carried out on the oracle itself (R25): one lane
    of 70 vehicles cut into tiles owning [0, 25), [25, 50), [50, 70), the 37
    steps into blocks of J = 8.  Forward: each block restarts every tile from
    the states its owners reached at the block's first step, simulating J
    vehicles ahead of the owned ones (the first of them as a free-road head).
    Adjoint, blocks from the last to the first: each tile runs the oracle's
    adjoint on the exact states of its owned vehicles, their leader and J
    followers, seeded at the block's last step with the adjoints the owners
    carried out of the block above (the upstream of the block's steps below
    it as given).  The owned states and the initial-state adjoints equal the
    whole-lane oracle's bit for bit, the parameter gradients (summed over the
    blocks in another association) to 1e-12."""
    import scenarios
    pb = Problem.from_scenario(scenarios.single_lane(n_vehicles=70, n_steps=37, mode=mode))
    P, V, _, _ = oracle.forward(pb)
    n, S, J = pb.n, pb.n_steps, 8
    rng = np.random.default_rng(7)
    gP = rng.normal(0.0, 1.0, (S + 1, n))
    gV = rng.normal(0.0, 1.0, (S + 1, n))
    g, gp0, gv0 = oracle.adjoint(pb, P, V, gP, gV)
    owned = [(0, 25), (25, 50), (50, 70)]
    blocks = [(k, min(S, k + J)) for k in range(0, S, J)]
    # forward, block by block
    Pt = np.full_like(P, np.nan)
    Vt = np.full_like(V, np.nan)
    Pt[0], Vt[0] = P[0], V[0]
    for k0, k1 in blocks:
        for lo, hi in owned:
            first = max(0, lo - J)
            sub = _sub_lane(pb, Pt, Vt, first, hi, k0, k1 - k0)
            Ps, Vs, _, _ = oracle.forward(sub)
            Pt[k0 + 1:k1 + 1, lo:hi] = Ps[1:, lo - first:]
            Vt[k0 + 1:k1 + 1, lo:hi] = Vs[1:, lo - first:]
    assert np.array_equal(Pt, P) and np.array_equal(Vt, V)
    # adjoint, from the last block to the first; lam holds every vehicle's
    # adjoint of (p, v) at the current block boundary
    lam_p, lam_v = gP[S].copy(), gV[S].copy()
    gt = np.zeros_like(g)
    for k0, k1 in reversed(blocks):
        new_p, new_v = np.full(n, np.nan), np.full(n, np.nan)
        for lo, hi in owned:
            first, last = max(0, lo - 1), min(n, hi + J)
            idx = np.arange(first, last)
            sub = _sub_lane(pb, P, V, first, last, k0, k1 - k0)
            up_p = gP[k0:k1 + 1, idx].copy()
            up_v = gV[k0:k1 + 1, idx].copy()
            up_p[-1], up_v[-1] = lam_p[idx], lam_v[idx]   # carried out of the block above
            gs, ps, vs = oracle.adjoint(sub, P[k0:k1 + 1, idx], V[k0:k1 + 1, idx], up_p, up_v)
            own = slice(lo - first, hi - first)
            new_p[lo:hi], new_v[lo:hi] = ps[own], vs[own]
            gt[:, lo:hi] += gs[:, own]
        lam_p, lam_v = new_p, new_v
    assert np.array_equal(lam_p, gp0) and np.array_equal(lam_v, gv0)
    np.testing.assert_allclose(gt, g, rtol=1e-12, atol=1e-12 * np.abs(g).max())


def test_lanes_are_independent_bitwise():
    """Two lanes simulated together equal each simulated alone."""
    a = _harsh(MODE_SOFTPLUS, n=10, seed=1)
    b = _harsh(MODE_SOFTPLUS, n=7, seed=2)
    cat = lambda x, y: np.concatenate([x, y])
    prm = {k: cat(a.params[k], b.params[k]) for k in a.params}
    prm["length"] = cat(a.length, b.length)
    both = Problem([0, 10, 17], prm, cat(a.p0, b.p0), cat(a.v_init, b.v_init), a.n_steps)
    P, V, _, _ = oracle.forward(both)
    Pa, _, _, _ = oracle.forward(a)
    Pb, _, _, _ = oracle.forward(b)
    assert np.array_equal(P[:, :10], Pa) and np.array_equal(P[:, 10:], Pb)


def test_softplus_floor_makes_accel_monotone_in_leader_speed():
    """Sec. III-C motivates the floor s* = softplus(s_opt): without it a leader
    pulling away fast (s_opt < 0) would make (s_opt/gap)^2 grow again and the
    follower brake.  With the floor, acceleration never decreases as the
    leader speeds up; with the plain IDM (CLAMP mode) it does."""
    def accel(mode, vh):
        pb = lane_problem(1, [1e9, 30.0], [1.0, 1.0], [1.5, 1.5], [2.0, 2.0], [2.0, 2.0],
                          [5.0, 5.0], [25.0, 0.0], [vh, 10.0], mode)
        _, _, A, _ = oracle.forward(pb, want_acc=True)
        return A[0, 1]
    vh = np.linspace(0.0, 60.0, 241)
    sp = np.array([accel(MODE_SOFTPLUS, x) for x in vh])
    cl = np.array([accel(MODE_CLAMP, x) for x in vh])
    assert np.all(np.diff(sp) >= -1e-12)
    assert np.any(np.diff(cl) < -1e-3)


def test_gap_floor_is_counted():
    pb = lane_problem(1, [30, 30], [1.5, 1.5], [1.5, 1.5], [2, 2], [2, 2], [5, 5],
                      [4.0, 0.0], [0.0, 10.0], MODE_SOFTPLUS)  # overlapping vehicles
    _, _, _, hits = oracle.forward(pb)
    assert hits == 1


# ---------------------------------------------------------------- gradients

def _small(mode, n=6, S=150, seed=5):
    rng = np.random.default_rng(seed)
    v0 = rng.uniform(25, 35, n); T = rng.uniform(1, 2, n); a = rng.uniform(1, 2, n)
    b = rng.uniform(1.5, 3, n); s0 = rng.uniform(1.5, 3, n); ln = rng.uniform(4.5, 5.5, n)
    gaps = rng.uniform(12, 30, n); vi = rng.uniform(10, 25, n)
    p = np.zeros(n)
    for i in range(n - 2, -1, -1):
        p[i] = p[i + 1] + gaps[i + 1] + ln[i]
    return lane_problem(S, v0, T, a, b, s0, ln, p, vi, mode, lane_offsets=[0, 4, n])


def _loss_fn(pb, W):
    P, V, _, _ = oracle.forward(pb)
    return float(np.sum(W * P))


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_adjoint_matches_central_differences(mode):
    """Central differences of a linear functional of the trajectory against the
    hand-derived adjoint, for every parameter of every vehicle and both initial
    states (<= 10 vehicles, two lanes)."""
    pb = _small(mode)
    rng = np.random.default_rng(0)
    W = rng.normal(size=(pb.n_steps + 1, pb.n))
    P, V, _, hits = oracle.forward(pb)
    assert hits == 0
    g, gp0, gv0 = oracle.adjoint(pb, P, V, W)
    names = ["v0", "T", "a", "b", "s0"]
    for j, name in enumerate(names):
        for i in range(pb.n):
            base = pb.params[name][i]
            h = 1e-6 * max(1.0, abs(base))
            pb.params[name][i] = base + h
            lp = _loss_fn(pb, W)
            pb.params[name][i] = base - h
            lm = _loss_fn(pb, W)
            pb.params[name][i] = base
            fd = (lp - lm) / (2 * h)
            scale = max(1.0, np.max(np.abs(g[j])))
            assert abs(fd - g[j, i]) <= 1e-6 * scale, (name, i, fd, g[j, i])
    for arr, grad in ((pb.p0, gp0), (pb.v_init, gv0)):
        for i in range(pb.n):
            base = arr[i]
            h = 1e-6 * max(1.0, abs(base))
            arr[i] = base + h
            lp = _loss_fn(pb, W)
            arr[i] = base - h
            lm = _loss_fn(pb, W)
            arr[i] = base
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[i]) <= 1e-6 * max(1.0, np.max(np.abs(grad)))


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_adjoint_is_transpose_of_tangent(mode):
    """Dot-product test: <J u, w> = <u, J^T w> for random u (parameters and
    initial state) and w (trajectory weights)."""
    pb = _small(mode, n=9, S=300, seed=9)
    rng = np.random.default_rng(1)
    P, V, _, _ = oracle.forward(pb)
    du = rng.normal(size=(5, pb.n)); dp0 = rng.normal(size=pb.n); dv0 = rng.normal(size=pb.n)
    wP = rng.normal(size=P.shape); wV = rng.normal(size=V.shape)
    dP, dV = oracle.tangent(pb, P, V, du, dp0, dv0)
    lhs = np.sum(wP * dP) + np.sum(wV * dV)
    g, gp0, gv0 = oracle.adjoint(pb, P, V, wP, wV)
    rhs = np.sum(g * du) + np.sum(gp0 * dp0) + np.sum(gv0 * dv0)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_head_has_zero_interaction_gradients():
    """The lane head drives on a free road (no leader): its loss does not
    depend on T, b, s0 (they only enter Eq. 1)."""
    pb = _small(MODE_SOFTPLUS)
    P, V, _, _ = oracle.forward(pb)
    W = np.zeros_like(P); W[:, 0] = 1.0; W[:, 4] = 1.0   # heads of both lanes
    g, _, _ = oracle.adjoint(pb, P, V, W)
    for j in (1, 3, 4):
        assert g[j, 0] == 0.0 and g[j, 4] == 0.0
    assert np.all(g[:, 1:4] == 0.0) and np.all(g[:, 5:] == 0.0)   # followers do not affect heads


def test_mse_and_gradient():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(11, 5))
    steps = [2, 5, 10]
    tgt = P[steps] + 0.25
    loss, gP = oracle.mse(P, steps, tgt)
    assert abs(loss - 0.0625) < 1e-15
    expect = np.zeros_like(P); expect[steps] = 2 * (-0.25) / 15
    np.testing.assert_allclose(gP, expect, rtol=1e-14)
    loss0, _ = oracle.mse(P, steps, P[steps])
    assert loss0 == 0.0
    s, g = oracle.mae_sum(P, steps, tgt)
    assert abs(s - 0.25 * 15) < 1e-12 and np.all(g[steps] == -1.0)


# ---------------------------------------------------------------- fit (Adam + box)

def test_adam_first_step_is_signed_learning_rate():
    """With zero moments the bias-corrected first Adam step is
    -lr * g / (|g| + eps): a step of (almost exactly) lr against the sign of
    the gradient, whatever its scale."""
    from oracle.fit import adam_box_step
    u = np.full((5, 4), 0.5)
    g = np.array([[3.0, -2e-3, 1e5, -7.0]] * 5)
    lo = np.zeros((5, 1)); hi = np.ones((5, 1))
    u1, m, v, th = adam_box_step(u, np.zeros_like(u), np.zeros_like(u), g, lo, hi, 1, 0.01)
    np.testing.assert_allclose(u1, 0.5 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(th, u1)


def test_adam_projection_and_chain_rule():
    """The box is enforced after every step, and a box of width w scales the
    gradient seen by u by w (theta = lo + u w)."""
    from oracle.fit import adam_box_step, lr_at
    lo = np.array([[15.0]]); hi = np.array([[45.0]])
    u = np.array([[0.995]]); m = np.zeros((1, 1)); v = np.zeros((1, 1))
    for t in range(1, 50):
        u, m, v, th = adam_box_step(u, m, v, np.array([[-1.0]]), lo, hi, t, 0.01)
        assert 0.0 <= u[0, 0] <= 1.0
    assert u[0, 0] == 1.0 and th[0, 0] == 45.0
    _, m1, _, _ = adam_box_step(np.array([[0.5]]), np.zeros((1, 1)), np.zeros((1, 1)),
                                np.array([[2.0]]), lo, hi, 1, 0.1)
    assert abs(m1[0, 0] - 0.1 * 2.0 * 30.0) < 1e-12
    assert lr_at(1, 0.1, 0.01, 500) == 0.1 and abs(lr_at(501, 0.1, 0.01, 500) - 0.01) < 1e-15
    assert abs(lr_at(251, 0.1, 0.01, 500) - 0.055) < 1e-15


def test_adam_minimises_a_box_constrained_quadratic():
    """Adam on f(theta) = (theta - c)^2 reaches c inside the box and the
    nearest bound when c is outside."""
    from oracle.fit import adam_box_step
    lo = np.array([[0.5], [0.5]]); hi = np.array([[3.0], [3.0]])
    c = np.array([[1.7], [5.0]])
    u = np.array([[0.9], [0.1]]); m = np.zeros_like(u); v = np.zeros_like(u)
    th = lo + u * (hi - lo)
    for t in range(1, 3000):
        u, m, v, th = adam_box_step(u, m, v, 2 * (th - c), lo, hi, t, 0.01)
    assert abs(th[0, 0] - 1.7) < 5e-3 and th[1, 0] == 3.0


# ---------------------------------------------------------------- warm-start MLP

def test_bf16_rounding_matches_torch():
    """The oracle's BF16 rounding (nearest, ties to even) equals torch's
    float32 -> bfloat16 conversion, including exact ties."""
    import torch
    from oracle.mlp import bf16
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 20000), rng.normal(0, 1e-3, 1000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 0.0, -0.0])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16(x32), ref)


def test_mlp_gradient_matches_central_differences():
    """FP64 network (no BF16 rounding): the hand-written backward against
    central differences on 60 random parameters, every block included."""
    from oracle import mlp
    import scenarios
    rng = np.random.default_rng(1)
    theta = scenarios.mlp_init_params(3).astype(np.float64)
    theta += rng.normal(0, 0.05, theta.shape)  # non-zero biases and padding
    X = rng.normal(0, 1, (12, mlp.IN_PAD))
    U = rng.uniform(0, 1, (12, mlp.OUT))
    L, g = mlp.loss_and_grad(theta, X, U, mirror=False)
    sizes = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    idx = np.concatenate([rng.integers(sizes[b], sizes[b + 1], 10) for b in range(6)])
    for i in idx:
        h = 1e-6
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, U, False)[0] - mlp.loss_and_grad(tm, X, U, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mlp_bf16_mirror_is_close_to_fp64():
    from oracle import mlp
    import scenarios
    rng = np.random.default_rng(2)
    theta = scenarios.mlp_init_params(4).astype(np.float64)
    X = rng.normal(0, 1, (64, mlp.IN_PAD)); X[:, mlp.IN:] = 0
    U = rng.uniform(0, 1, (64, mlp.OUT))
    La, ga = mlp.loss_and_grad(theta, X, U, mirror=True)
    Lb, gb = mlp.loss_and_grad(theta, X, U, mirror=False)
    assert abs(La - Lb) < 2e-2 * Lb
    assert np.linalg.norm(ga - gb) < 5e-2 * np.linalg.norm(gb)


def test_window_features_hand_computed():
    """The warm-start window (per observation: offset from p0 / 1000 m,
    finite-difference speed / 30 m/s from p0 at t = 0, gap to the observed
    leader / 50 m with 200 m for a lane head) on a case small enough to work
    out by hand: lane 0 = vehicles 0 (head) and 1, lane 1 = vehicle 2 (head),
    an empty lane between them, observations at steps 5, 15, 25 of 0.2 s
    (t = 1, 3, 5 s: a first interval of 1 s and then 2 s, so the time of the
    first observation and the stride are told apart).  Vehicle 1's leader is 4 m
    long and vehicle 1 itself 5 m, so using the follower's own length, the
    follower as leader or a sign flip changes a gap value."""
    from oracle import mlp
    tgt = np.array([[110.0, 88.0, 30.0],
                    [125.0, 101.0, 60.0],
                    [145.0, 118.0, 90.0]])
    p0 = np.array([100.0, 80.0, 0.0])
    length = np.array([4.0, 5.0, 6.0])
    F = mlp.features(tgt, 5, 10, 0.2, p0, length, np.array([0, 2, 2, 3]))
    expect = np.zeros((3, mlp.IN_PAD))
    # offsets (p_j - p0) / 1000
    expect[0, 0:3] = [10 / 1000, 25 / 1000, 45 / 1000]
    expect[1, 0:3] = [8 / 1000, 21 / 1000, 38 / 1000]
    expect[2, 0:3] = [30 / 1000, 60 / 1000, 90 / 1000]
    # speeds: (110 - 100) / 1 s, (125 - 110) / 2 s, (145 - 125) / 2 s, all / 30
    expect[0, 3:6] = [10 / 30, 7.5 / 30, 10 / 30]
    expect[1, 3:6] = [8 / 30, 6.5 / 30, 8.5 / 30]
    expect[2, 3:6] = [30 / 30, 15 / 30, 15 / 30]
    # gaps: heads 200 / 50; vehicle 1: 110 - 88 - 4, 125 - 101 - 4, 145 - 118 - 4
    expect[0, 6:9] = [4.0, 4.0, 4.0]
    expect[1, 6:9] = [18 / 50, 20 / 50, 23 / 50]
    expect[2, 6:9] = [4.0, 4.0, 4.0]
    np.testing.assert_allclose(F, expect, rtol=1e-15, atol=0)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_branch_terms_agree_with_the_forward(mode):
    """oracle.branch_terms (the test helper that measures distances to the
    kinks) reports what the forward used: the raw gap is the leader's position
    minus the own position minus the LEADER's length (+inf for a head); in
    CLAMP mode an unclamped speed update is v + dt ahat; in SOFTPLUS mode the
    acceleration is a_lb + softplus(ahat - a_lb) with a_lb = max(-v/dt, a_min)."""
    import scenarios
    sc = scenarios.congested(n_lanes=4, lane_len=12, n_steps=60, mode=mode)
    pb = Problem.from_scenario(sc)
    P, V, A, _ = oracle.forward(pb, want_acc=True)
    AH, GAP = oracle.branch_terms(pb, P, V)
    off = sc.lane_offsets
    for l in range(sc.n_lanes):
        lo, hi = int(off[l]), int(off[l + 1])
        assert np.all(np.isinf(GAP[:, lo]))
        want = P[:-1, lo:hi - 1] - P[:-1, lo + 1:hi] - sc.params["length"][lo:hi - 1].astype(np.float64)
        np.testing.assert_allclose(GAP[:, lo + 1:hi], want, rtol=0, atol=1e-9)
    if mode == MODE_CLAMP:
        moving = V[1:] > 0
        assert np.array_equal(V[1:][moving], (V[:-1] + sc.dt * AH)[moving])
        assert np.all(V[:-1][~moving] + sc.dt * AH[~moving] <= 0)
    else:
        a_lb = np.maximum(-V[:-1] / sc.dt, sc.a_min)
        x = AH - a_lb
        sp = np.maximum(x, 0) + np.log1p(np.exp(-np.abs(x)))
        np.testing.assert_allclose(A, a_lb + sp, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", [MODE_SOFTPLUS, MODE_CLAMP])
def test_stop_and_go_queues_reach_the_bounds(mode):
    """The stop-and-go lanes used by the GPU bound tests stop vehicles: speeds
    reach 0, the lower bound -v/dt of Sec. III-C (SOFTPLUS) or the clamp
    (CLAMP) is active at vehicles whose gradients those tests compare, and
    most vehicles are comparable."""
    import sys, os
    import scenarios
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from _util import kink_margins, oracle_reference
    kw = dict(speed_max=15.0, gap_range=(5.0, 15.0)) if mode == MODE_SOFTPLUS else \
        dict(speed_max=30.0, gap_range=(3.0, 12.0))
    sc = scenarios.congested(mode=mode, **kw)
    ref = oracle_reference(sc)
    mask, counts = kink_margins(sc, ref)
    assert ref["V"].min() <= (1e-3 if mode == MODE_SOFTPLUS else 0.0)
    assert counts["lower_bound" if mode == MODE_SOFTPLUS else "clamp"] > 100
    assert mask.sum() >= 0.7 * sc.n
