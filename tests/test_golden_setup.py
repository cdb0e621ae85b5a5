"""The reconstruction and forecasting code uses the constants the paper
prints for its setup (fixture tests/golden/paper_setup.txt, one citation per
entry)."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_setup.txt")


def _fixture():
    out = {}
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        body, cite = line.split("|", 1)
        key, vals = body.split("=", 1)
        assert cite.strip().startswith("Sec."), line
        out[key.strip()] = [float(v) for v in vals.split()]
    return out


@pytest.fixture(scope="module")
def G():
    return _fixture()


def test_initial_values_and_boxes(G):
    from paper_2412_16750_amd import ego
    # code order: v0, T, a, b, s0
    names = ("v_targ", "T_pref", "a_max", "a_pref", "s_min")
    assert tuple(ego.PAPER_INIT) == tuple(G["init_" + n][0] for n in names)
    assert tuple(tuple(b) for b in ego.PAPER_BOXES) == tuple(tuple(G["box_" + n]) for n in names)
    assert ego.PAPER_GAP0 == G["init_gap"][0] and ego.PAPER_DV0 == G["init_speed_diff"][0]
    for lo_hi, init in zip(ego.PAPER_BOXES, ego.PAPER_INIT):
        assert lo_hi[0] <= init <= lo_hi[1]


def test_optimiser_schedule_and_bounds(G):
    import inspect
    from paper_2412_16750_amd import ego
    sig = inspect.signature(ego.EgoFitter.__init__).parameters
    assert sig["lr0"].default == G["lr_first"][0]
    assert sig["lr1"].default == G["lr_last"][0]
    assert sig["lr_steps"].default == G["adam_steps"][0]
    assert inspect.signature(ego.EgoPlan.__init__).parameters["a_min"].default == G["a_min"][0]


def test_forecast_rollout_length(G):
    import scenarios
    sc = scenarios.forecast(n_lanes=2, lane_len=3)
    assert sc.extra["future"] == G["rollout_frames"][0]
    assert np.isclose(sc.dt, G["rollout_dt"][0])
    assert np.isclose(sc.extra["future"] * sc.dt, 8.0)


def test_reconstruction_starts_at_the_origin(G):
    """p(0) = 0 for every trajectory (the oracle's ego model), whatever the
    initial speed."""
    import oracle
    n, S = 3, 4
    prm = {k: np.full(n, v) for k, v in zip(("v0", "T", "a", "b", "s0"), (50.0, 1.0, 10.0, 2.0, 5.0))}
    pb = oracle.EgoProblem(prm, np.full((S, n), 10.0), np.zeros((S, n)), np.array([0.0, 5.0, 20.0]), S)
    P, V, _, _ = oracle.ego_forward(pb)
    assert np.all(P[0] == G["initial_position"][0])
    assert np.array_equal(V[0], pb.v_init)
