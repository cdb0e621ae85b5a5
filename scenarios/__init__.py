"""Seeded synthetic scenarios for the IDM simulator.

This module only draws random inputs and lays vehicles out on lanes. It holds
none of the simulation's arithmetic (no gap, acceleration or Euler update), so
both the FP64 CPU oracle and the HIP path can consume the same inputs.

Workload shapes follow the paper's setting (Sec. III-A: one-dimensional lanes,
each vehicle following the one directly ahead; Sec. V-A: up to 2 million
vehicles) and the five workloads the repository measures:

* ``single_lane``  : 1 open lane x 100 vehicles, 1000 steps of 0.1 s.
* ``scale``        : 2000 lanes x 1000 vehicles = 2M vehicles, 100 steps,
                     checkpoints every 32 steps.
* ``uneven``       : 10,000 independent lanes, sizes round(lognormal(5, 1.2))
                     clipped to [10, 4096], 300 steps.
* ``fit``          : 100 lanes x 1000 vehicles, 500 steps, observations every
                     10th step with N(0, 0.5 m) noise.
* ``warm``         : pairs for the learned warm start, drawn like ``fit``.

Per-vehicle draws (all uniform): v0 in [25, 35] m/s, T in [1, 2] s,
a in [1, 2] m/s^2, b in [1.5, 3] m/s^2, s0 in [1.5, 3] m; length 5 m;
bumper-to-bumper initial gaps in [20, 40] m; initial speeds in [10, 25] m/s.
The tail vehicle of every lane starts at p = 0 and leaders sit ahead of it, so
every position is non-negative. Lanes are stored head -> tail, contiguously,
with CSR offsets.

Seeds: params 1000 + c, second (target) params 2000 + c, initial state
3000 + c, noise 4000 + c, lane sizes 5000 + c, where c is the workload number
(1..5).  Random numbers are NumPy PCG64 streams (``numpy.random.default_rng``).
Parameters, speeds and lengths are drawn in float64 and rounded once to float32,
because the GPU path stores them in float32; the oracle promotes exactly those
float32 values to float64, so both sides simulate the same problem.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, Optional

import numpy as np

PARAM_NAMES = ("v0", "T", "a", "b", "s0")

# Uniform ranges of the per-vehicle IDM parameters.
PARAM_RANGES = {
    "v0": (25.0, 35.0),
    "T": (1.0, 2.0),
    "a": (1.0, 2.0),
    "b": (1.5, 3.0),
    "s0": (1.5, 3.0),
}
# Box used when fitting normalised parameters: theta = lo + u * (hi - lo).
FIT_BOXES = {
    "v0": (15.0, 45.0),
    "T": (0.5, 3.0),
    "a": (0.5, 3.0),
    "b": (0.5, 4.0),
    "s0": (0.5, 5.0),
}
# Cold start of the fit: the mean of each uniform range.
COLD_START = {k: 0.5 * (lo + hi) for k, (lo, hi) in PARAM_RANGES.items()}

MODE_SOFTPLUS = 0
MODE_CLAMP = 1


@dataclass
class Scenario:
    """One seeded problem: lanes, per-vehicle parameters and initial state."""

    name: str
    lane_offsets: np.ndarray          # int32 [L+1], vehicles head -> tail
    params: Dict[str, np.ndarray]     # float32 [N] each: v0, T, a, b, s0, length
    p0: np.ndarray                    # float64 [N] initial positions (m)
    v_init: np.ndarray                # float32 [N] initial speeds (m/s)
    n_steps: int
    dt: float = 0.1
    delta: float = 4.0
    a_min: float = -10.0
    gap_floor: float = 1e-3
    mode: int = MODE_SOFTPLUS
    ckpt_every: int = 32
    extra: Dict[str, object] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.lane_offsets[-1])

    @property
    def n_lanes(self) -> int:
        return int(len(self.lane_offsets) - 1)

    def with_(self, **kw) -> "Scenario":
        return replace(self, **kw)


def _f32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))


def draw_params(rng: np.random.Generator, n: int) -> Dict[str, np.ndarray]:
    """Per-vehicle IDM parameters (float32) plus the 5 m vehicle length."""
    out = {}
    for k in PARAM_NAMES:
        lo, hi = PARAM_RANGES[k]
        out[k] = _f32(rng.uniform(lo, hi, size=n))
    out["length"] = np.full(n, 5.0, dtype=np.float32)
    return out


def place_lanes(rng: np.random.Generator, lane_offsets: np.ndarray,
                length: np.ndarray, gap_range=(20.0, 40.0),
                speed_range=(10.0, 25.0)):
    """Initial positions (float64) and speeds (float32).

    Within a lane the tail is at 0 and vehicle i-1 (the leader of i) sits at
    p[i] + length[i-1] + gap[i], with bumper-to-bumper gaps drawn uniformly.
    """
    n = int(lane_offsets[-1])
    gaps = rng.uniform(gap_range[0], gap_range[1], size=n)
    v = _f32(rng.uniform(speed_range[0], speed_range[1], size=n))
    p = np.zeros(n, dtype=np.float64)
    lens = np.asarray(length, dtype=np.float64)
    for lane in range(len(lane_offsets) - 1):
        lo, hi = int(lane_offsets[lane]), int(lane_offsets[lane + 1])
        if hi <= lo:
            continue
        # walk from the tail (hi-1) towards the head (lo)
        seg_gap = gaps[lo + 1:hi]            # gap in front of vehicles lo+1..hi-1
        seg_len = lens[lo:hi - 1]            # length of their leaders lo..hi-2
        inc = (seg_gap + seg_len)[::-1]      # tail first
        pos = np.concatenate([[0.0], np.cumsum(inc)])[::-1]
        p[lo:hi] = pos
    return p, v


def uniform_lanes(n_lanes: int, lane_len: int) -> np.ndarray:
    return (np.arange(n_lanes + 1, dtype=np.int64) * lane_len).astype(np.int32)


def lognormal_lane_sizes(n_lanes: int, mu: float, sigma: float, lo: int, hi: int,
                         seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sizes = np.rint(rng.lognormal(mu, sigma, size=n_lanes))
    return np.clip(sizes, lo, hi).astype(np.int64)


def offsets_from_sizes(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    if off[-1] >= 2 ** 31:
        raise ValueError("too many vehicles for int32 offsets")
    return off.astype(np.int32)


def make_scenario(name: str, lane_offsets: np.ndarray, n_steps: int, c: int,
                  **kw) -> Scenario:
    n = int(lane_offsets[-1])
    params = draw_params(np.random.default_rng(1000 + c), n)
    p0, v = place_lanes(np.random.default_rng(3000 + c), lane_offsets, params["length"])
    return Scenario(name=name, lane_offsets=np.ascontiguousarray(lane_offsets, dtype=np.int32),
                    params=params, p0=p0, v_init=v, n_steps=n_steps, **kw)


def single_lane(n_vehicles: int = 100, n_steps: int = 1000, mode: int = MODE_SOFTPLUS,
                **kw) -> Scenario:
    """Workload 1: one open lane, head on free road."""
    return make_scenario("single_lane", uniform_lanes(1, n_vehicles), n_steps, 1,
                         mode=mode, **kw)


def scale(n_lanes: int = 2000, lane_len: int = 1000, n_steps: int = 100,
          ckpt_every: int = 32, **kw) -> Scenario:
    """Workload 2: 2000 x 1000 = 2M vehicles, 100 steps, checkpoints every 32."""
    return make_scenario("scale", uniform_lanes(n_lanes, lane_len), n_steps, 2,
                         ckpt_every=ckpt_every, **kw)


def uneven(n_lanes: int = 10000, n_steps: int = 300, mu: float = 5.0, sigma: float = 1.2,
           lo: int = 10, hi: int = 4096, **kw) -> Scenario:
    """Workload 3: many independent lanes of lognormal length."""
    sizes = lognormal_lane_sizes(n_lanes, mu, sigma, lo, hi, 5000 + 3)
    return make_scenario("uneven", offsets_from_sizes(sizes), n_steps, 3, **kw)


def congested(n_lanes: int = 64, lane_len: int = 12, n_steps: int = 200, dt: float = 0.1,
              c: int = 11, speed_max: float = 15.0, gap_range=(5.0, 15.0),
              mode: int = MODE_SOFTPLUS, head_speed=(0.5, 3.0), **kw) -> Scenario:
    """Stop-and-go lanes for the speed bounds of Sec. III-C: every lane head
    creeps (desired speed U[head_speed], by default U[0.5, 3] m/s, starting
    at rest) and its followers
    start at speeds U[0, speed_max] with bumper-to-bumper gaps drawn from
    gap_range, so the queues brake hard and speeds reach 0.  Parameters are the
    usual draws apart from the heads' desired speeds (seed 1000 + c); heads,
    gaps and speeds come from seed 3000 + c."""
    off = uniform_lanes(n_lanes, lane_len)
    params = draw_params(np.random.default_rng(1000 + c), int(off[-1]))
    rng = np.random.default_rng(3000 + c)
    heads = off[:-1]
    params["v0"][heads] = _f32(rng.uniform(head_speed[0], head_speed[1], len(heads)))
    p0, v = place_lanes(rng, off, params["length"], gap_range=gap_range,
                        speed_range=(0.0, speed_max))
    v = v.copy()
    v[heads] = 0.0
    return Scenario(name="congested", lane_offsets=off, params=params, p0=p0, v_init=v,
                    n_steps=n_steps, dt=dt, mode=mode, **kw)


def fit(n_lanes: int = 100, lane_len: int = 1000, n_steps: int = 500, obs_every: int = 10,
        **kw) -> Scenario:
    """Workload 4: hidden params = the usual draw; observations every 10th step."""
    sc = make_scenario("fit", uniform_lanes(n_lanes, lane_len), n_steps, 4, **kw)
    sc.extra["obs_first"] = obs_every
    sc.extra["obs_stride"] = obs_every
    return sc


def second_params(sc: Scenario, c: int) -> Dict[str, np.ndarray]:
    """An independent parameter draw for the same vehicles (target generation)."""
    p = draw_params(np.random.default_rng(2000 + c), sc.n)
    p["length"] = sc.params["length"].copy()
    return p


def cold_params(sc: Scenario) -> Dict[str, np.ndarray]:
    out = {k: np.full(sc.n, COLD_START[k], dtype=np.float32) for k in PARAM_NAMES}
    out["length"] = sc.params["length"].copy()
    return out


def noise(shape, c: int, sigma: float = 0.5) -> np.ndarray:
    """N(0, sigma) observation noise, float64."""
    return np.random.default_rng(4000 + c).normal(0.0, sigma, size=shape)


def obs_steps(n_steps: int, first: int, stride: int) -> np.ndarray:
    """Observed step indices first, first+stride, ... <= n_steps."""
    if first < 0 or stride < 1 or first > n_steps:
        raise ValueError("bad observation schedule")
    return np.arange(first, n_steps + 1, stride, dtype=np.int32)


def constant_speed_targets(sc: Scenario, steps: np.ndarray, c: int,
                           sigma: float = 0.5) -> np.ndarray:
    """Dense synthetic targets for throughput runs: p0 + v_init * t + noise.

    Returns float32 [len(steps)][N].  Only the shape and magnitude matter for a
    throughput measurement; the values are not produced by any simulator.
    """
    t = steps.astype(np.float64)[:, None] * sc.dt
    base = sc.p0[None, :] + sc.v_init.astype(np.float64)[None, :] * t
    return (base + noise(base.shape, c, sigma)).astype(np.float32)


def subset_lanes(sc: Scenario, lanes) -> Scenario:
    """A scenario made of the given lanes of ``sc`` (same values, same order)."""
    lanes = np.asarray(lanes, dtype=np.int64)
    off = sc.lane_offsets.astype(np.int64)
    idx = np.concatenate([np.arange(off[l], off[l + 1]) for l in lanes]) if len(lanes) else \
        np.zeros(0, dtype=np.int64)
    sizes = off[lanes + 1] - off[lanes]
    return Scenario(name=sc.name + "_sub", lane_offsets=offsets_from_sizes(sizes),
                    params={k: np.ascontiguousarray(v[idx]) for k, v in sc.params.items()},
                    p0=np.ascontiguousarray(sc.p0[idx]), v_init=np.ascontiguousarray(sc.v_init[idx]),
                    n_steps=sc.n_steps, dt=sc.dt, delta=sc.delta, a_min=sc.a_min,
                    gap_floor=sc.gap_floor, mode=sc.mode, ckpt_every=sc.ckpt_every,
                    extra=dict(sc.extra, vehicle_index=idx))


# ---------------------------------------------------------------- warm-start MLP

MLP_IN, MLP_IN_PAD, MLP_HIDDEN, MLP_OUT, MLP_OUT_PAD = 150, 160, 256, 5, 16


def mlp_init_params(seed: int) -> np.ndarray:
    """Seeded Kaiming-uniform draw (bound sqrt(6 / fan_in)) of the MLP's FP32
    parameter vector in the layout W1 [160 x 256], b1 [256], W2 [256 x 256],
    b2 [256], W3 [256 x 16], b3 [16]; padding rows/columns and biases are 0."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((MLP_IN_PAD, MLP_HIDDEN))
    W1[:MLP_IN] = rng.uniform(-1, 1, (MLP_IN, MLP_HIDDEN)) * np.sqrt(6.0 / MLP_IN)
    W2 = rng.uniform(-1, 1, (MLP_HIDDEN, MLP_HIDDEN)) * np.sqrt(6.0 / MLP_HIDDEN)
    W3 = np.zeros((MLP_HIDDEN, MLP_OUT_PAD))
    W3[:, :MLP_OUT] = rng.uniform(-1, 1, (MLP_HIDDEN, MLP_OUT)) * np.sqrt(6.0 / MLP_HIDDEN)
    parts = [W1, np.zeros(MLP_HIDDEN), W2, np.zeros(MLP_HIDDEN), W3, np.zeros(MLP_OUT_PAD)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def normalized_params(params: Dict[str, np.ndarray]) -> np.ndarray:
    """[N, 5] FP32 targets u = (theta - lo) / (hi - lo) in the fit boxes."""
    cols = [(np.asarray(params[k], np.float64) - FIT_BOXES[k][0]) / (FIT_BOXES[k][1] - FIT_BOXES[k][0])
            for k in PARAM_NAMES]
    return np.ascontiguousarray(np.stack(cols, axis=1).astype(np.float32))


def warm_training(n_lanes: int = 1000, lane_len: int = 1000, n_steps: int = 500,
                  obs_every: int = 10, **kw) -> Scenario:
    """Workload 5: training pairs for the warm start, drawn like workload 4 from
    independent seeds (1000 lanes x 1000 vehicles = 1M pairs by default)."""
    sc = make_scenario("warm", uniform_lanes(n_lanes, lane_len), n_steps, 5, **kw)
    sc.extra["obs_first"] = obs_every
    sc.extra["obs_stride"] = obs_every
    return sc


# ---------------------------------------------------------------------------
# Sparse observed trajectories for the ego-only reconstruction (Sec. IV-A /
# V-B): stand-ins for the paper's trajectory sets (NGSIM at 10 Hz for filtering,
# a non-public set of 21,750 trajectories sampled at >= 1 s and up to 20 min
# long for reconstruction), which are not available here.  A trajectory is a
# smooth random speed profile (a mean plus three sinusoids of 30-300 s period
# whose slopes stay within 0.5 m/s^2 each, floored at 0), integrated on a
# 0.1 s grid and sampled at irregular times, with N(0, sigma) position noise;
# times and positions are taken relative to the first sample (p(0) = 0).  No
# traffic model is involved.

@dataclass
class EgoData:
    """CSR by trajectory: t [M] (s, FP64), pos [M] (m, FP64), offsets [N+1]."""
    offsets: np.ndarray
    t: np.ndarray
    pos: np.ndarray
    duration: np.ndarray  # [N] time of the last sample (s)
    dt: float             # simulation step of the reconstruction
    n_steps: int          # steps that cover the longest trajectory

    @property
    def n(self) -> int:
        return len(self.offsets) - 1


def ego_trajectories(n_traj: int, c: int, dt: float = 1.0, min_s: float = 120.0,
                     max_s: float = 1200.0, min_gap: float = 1.0, mean_extra_gap: float = 4.0,
                     sigma: float = 0.5, dense: bool = False) -> EgoData:
    """n_traj synthetic observed trajectories (seeds 6000 + c).  Sparse
    sampling: intervals min_gap + Exp(mean_extra_gap) s; dense (filtering):
    every dt."""
    rng = np.random.default_rng(6000 + c)
    dur = rng.uniform(min_s, max_s, n_traj)
    ts, ps, counts = [], [], []
    for i in range(n_traj):
        if dense:
            t = np.arange(0.0, dur[i] + 1e-9, dt)
        else:
            gaps = min_gap + rng.exponential(mean_extra_gap, int(dur[i] / min_gap) + 2)
            t = np.concatenate([[0.0], np.cumsum(gaps)])
            t = t[t <= dur[i]]
        grid = np.arange(0.0, t[-1] + 0.1 + 1e-9, 0.1)
        vbar = rng.uniform(8.0, 25.0)
        per = rng.uniform(30.0, 300.0, 3)
        amp = rng.uniform(0.0, 0.5, 3) * per / (2 * np.pi)
        ph = rng.uniform(0.0, 2 * np.pi, 3)
        v = vbar + np.sum(amp[:, None] * np.sin(2 * np.pi * grid[None, :] / per[:, None] + ph[:, None]),
                          axis=0)
        v = np.maximum(v, 0.0)
        x = np.concatenate([[0.0], np.cumsum(0.5 * (v[1:] + v[:-1]) * 0.1)])
        p = np.interp(t, grid, x) + rng.normal(0.0, sigma, len(t))
        ts.append(t - t[0])
        ps.append(p - p[0])
        counts.append(len(t))
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    t_all = np.concatenate(ts)
    dur_obs = np.array([t[-1] for t in ts])
    return EgoData(off, t_all, np.concatenate(ps), dur_obs, float(dt),
                   int(np.ceil(dur_obs.max() / dt)) + 1)


def reconstruction(n_traj: int = 21750, c: int = 6) -> EgoData:
    """The reconstruction workload: 21,750 trajectories, >= 1 s sampling, up to
    20 minutes, simulated with dt = 1 s."""
    return ego_trajectories(n_traj, c, dt=1.0)


def filtering(n_traj: int = 6101, c: int = 7) -> EgoData:
    """The filtering workload: 6,101 trajectories observed every 0.1 s (NGSIM
    rate), 30 s to 3 min long, simulated with dt = 0.1 s."""
    return ego_trajectories(n_traj, c, dt=0.1, min_s=30.0, max_s=180.0, sigma=0.3, dense=True)


def ego_free_variables(n_traj: int, n_steps: int, c: int):
    """Random parameters [5, N] (config ranges), gap G [S, N] in [8, 40] m and
    speed difference D [S, N] ~ N(0, 1.5) for parity tests (seeds 7000 + c)."""
    rng = np.random.default_rng(7000 + c)
    prm = draw_params(rng, n_traj)
    P = np.stack([prm[k] for k in PARAM_NAMES]).astype(np.float32)
    G = rng.uniform(8.0, 40.0, (n_steps, n_traj)).astype(np.float32)
    D = rng.normal(0.0, 1.5, (n_steps, n_traj)).astype(np.float32)
    v = rng.uniform(8.0, 25.0, n_traj).astype(np.float32)
    return P, G, D, v


def forecast(n_lanes: int = 10000, lane_len: int = 8, history: int = 10, future: int = 80,
             **kw) -> Scenario:
    """Forecasting workload (stand-in for the paper's WOMD rollouts, Sec. V-C):
    short lanes of a few vehicles with hidden parameters = the usual draw,
    observed over a 1 s history (10 steps of 0.1 s) and rolled out 8 s (80
    steps) further; n_steps = history + future."""
    sc = make_scenario("forecast", uniform_lanes(n_lanes, lane_len), history + future, 8, **kw)
    sc.extra["history"] = history
    sc.extra["future"] = future
    return sc
