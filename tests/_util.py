"""Shared helpers of the test-suite: build seeded problems, run the oracle and
the HIP path on the same inputs, and compare them."""
from __future__ import annotations

import numpy as np

import scenarios

PARAM_NAMES = ("v0", "T", "a", "b", "s0")


def ragged_scenario(sizes, n_steps, mode=scenarios.MODE_SOFTPLUS, seed_c=7, ckpt_every=16):
    off = scenarios.offsets_from_sizes(sizes)
    return scenarios.make_scenario("ragged", off, n_steps, seed_c, mode=mode, ckpt_every=ckpt_every)


def oracle_targets(sc, steps, c=1):
    """Targets from an independent parameter draw, simulated by the ORACLE,
    plus N(0, 0.5 m) noise, rounded to FP32 (what both sides consume)."""
    import oracle
    pb2 = oracle.Problem.from_scenario(sc, params=scenarios.second_params(sc, c))
    P2, _, _, _ = oracle.forward(pb2)
    tgt = P2[steps] + scenarios.noise((len(steps), sc.n), c)
    return tgt.astype(np.float32)


def oracle_reference(sc, steps=None, target=None, dense=None):
    """FP64 oracle forward, MSE loss and adjoint on the scenario's FP32 inputs."""
    import oracle
    pb = oracle.Problem.from_scenario(sc)
    P, V, _, hits = oracle.forward(pb)
    gP = np.zeros_like(P)
    loss = 0.0
    if target is not None:
        loss, gm = oracle.mse(P, steps, target.astype(np.float64))
        gP += gm
    if dense is not None:
        gP += dense.astype(np.float64).reshape(gP.shape)
    g, gp0, gv0 = oracle.adjoint(pb, P, V, gP)
    if dense is not None:
        # a dense upstream acts on the displacements d = P - p0 at fixed p0:
        # L(d) = L(P - p0), so dL/dp0 loses the direct term sum_k dL/dd_k
        gp0 = gp0 - dense.astype(np.float64).reshape(gP.shape).sum(axis=0)
    return dict(P=P, V=V, loss=loss, g=g, gp0=gp0, gv0=gv0, floor_hits=hits)


def pos_close(p_gpu, p_ref, rtol=1e-4, floor=1.0):
    """|p_gpu - p_ref| <= rtol * max(|p_ref|, floor), elementwise."""
    err = np.abs(p_gpu - p_ref)
    lim = rtol * np.maximum(np.abs(p_ref), floor)
    return bool(np.all(err <= lim)), float(err.max()), float((err / lim).max())


def disp_close(d_gpu, p_ref, p0, rtol=1e-4, floor=1.0):
    """The displacement d = p - p0 on its own scale:
    |d_gpu - (p_ref - p0)| <= rtol * max(|p_ref - p0|, floor), elementwise
    (the kernels advance displacements, so this does not loosen with the
    distance of the lane from the origin as an absolute-position check does)."""
    d_ref = np.asarray(p_ref, dtype=np.float64) - np.asarray(p0, dtype=np.float64)[None, :]
    return pos_close(np.asarray(d_gpu, dtype=np.float64), d_ref, rtol, floor)


def grad_close(g_gpu, g_ref, rtol=1e-3, rel_floor=1e-2, where=None):
    """|g_gpu - g_ref| <= rtol * max(|g_ref|, rel_floor * max|g_ref|), per row.
    Returns (ok, worst error / limit); `where` (a list) receives the worst
    element as (row, index, g_gpu, g_ref, limit)."""
    g_gpu = np.atleast_2d(g_gpu)
    g_ref = np.atleast_2d(g_ref)
    worst = 0.0
    ok = True
    for row, (a, b) in enumerate(zip(g_gpu, g_ref)):
        scale = np.max(np.abs(b)) if b.size else 0.0
        lim = rtol * np.maximum(np.abs(b), rel_floor * scale)
        lim = np.where(lim > 0, lim, 1e-30)
        r = np.abs(a - b) / lim
        if r.size and float(r.max()) > worst:
            worst = float(r.max())
            if where is not None:
                i = int(r.argmax())
                where[:] = [(row, i, float(a[i]), float(b[i]), float(lim[i]))]
        ok = ok and bool(np.all(np.abs(a - b) <= lim))
    return ok, worst


def kink_margins(sc, ref, lb_tol=1e-2, clamp_rtol=1e-4, gap_min=0.05):
    """Which vehicles' gradients a FP32 path can match in the bound regime of
    Sec. III-C.  An evaluation is "near a kink" when the FP32 state could put
    it on the other side of a branch: -v/dt within lb_tol m/s^2 of a_min while
    the bound carries weight (1 - w > 1e-4, SOFTPLUS), v + dt * ahat within
    clamp_rtol of its terms (CLAMP), or a gap below gap_min (the gap floor and
    the stiff region above it).  A kink at vehicle i changes the adjoint of i
    and of every vehicle ahead of it in the lane (the adjoint runs from
    follower to leader), so the comparable vehicles of a lane are those behind
    its last near-kink vehicle.  Returns (mask [N], counts) where counts has
    the numbers of active bound evaluations ("lower_bound": a_lb = -v/dt with
    1 - w > 1e-3, "clamp": v + dt * ahat <= 0) at comparable vehicles, and of
    excluded vehicles."""
    import oracle
    pb = oracle.Problem.from_scenario(sc)
    AH, GAP = oracle.branch_terms(pb, ref["P"], ref["V"])
    Vk = ref["V"][:-1]
    dt, a_min = sc.dt, sc.a_min
    if sc.mode == scenarios.MODE_SOFTPLUS:
        on_v = Vk / dt < -a_min
        a_lb = np.where(on_v, -Vk / dt, a_min)
        with np.errstate(over="ignore"):
            w = 1.0 / (1.0 + np.exp(-(AH - a_lb)))
        near = (np.abs(Vk / dt + a_min) < lb_tol) & ((1.0 - w) > 1e-4)
        lower = on_v & ((1.0 - w) > 1e-3)
        clamp = np.zeros_like(on_v)
    else:
        pre = Vk + dt * AH
        near = np.abs(pre) < clamp_rtol * (np.abs(Vk) + dt * np.abs(AH)) + 1e-4
        lower = np.zeros_like(near)
        clamp = pre <= 0.0
    near = near | (GAP < gap_min)
    near_v = np.any(near, axis=0) if near.size else np.zeros(sc.n, bool)
    mask = np.ones(sc.n, bool)
    off = sc.lane_offsets
    for l in range(sc.n_lanes):
        lo, hi = int(off[l]), int(off[l + 1])
        idx = np.nonzero(near_v[lo:hi])[0]
        if idx.size:
            mask[lo:lo + idx[-1] + 1] = False
    counts = dict(lower_bound=int(lower[:, mask].sum()), clamp=int(clamp[:, mask].sum()),
                  excluded=int((~mask).sum()), floor_hits=int(ref["floor_hits"]))
    return mask, counts


def fp32_state_conditioning(sc, steps=None, target=None, dense=None, ref=None, mask=None):
    """How well an FP32 state determines the oracle's gradients here: the
    oracle is stepped one step at a time with the displacement d = p - p0 and
    the speed rounded to FP32 after every step (the resolution at which the
    HIP path carries its state), and its adjoint along that trajectory is
    compared with the FP64 one at grad_close's limits.  Returns the worst
    error / limit per gradient row (v0, T, a, b, s0, p0, v0-initial) over the
    vehicles in `mask`.  Everything here is the oracle's own arithmetic."""
    import oracle
    pb1 = oracle.Problem.from_scenario(sc, n_steps=1)
    S, n = sc.n_steps, sc.n
    P = np.empty((S + 1, n))
    V = np.empty((S + 1, n))
    P[0], V[0] = sc.p0, sc.v_init
    for k in range(S):
        pb1.p0 = np.ascontiguousarray(P[k])
        pb1.v_init = np.ascontiguousarray(V[k])
        Pk, Vk, _, _ = oracle.forward(pb1)
        P[k + 1] = sc.p0 + (Pk[1] - sc.p0).astype(np.float32).astype(np.float64)
        V[k + 1] = Vk[1].astype(np.float32).astype(np.float64)
    gP = np.zeros_like(P)
    if target is not None:
        gP += oracle.mse(P, steps, target.astype(np.float64))[1]
    if dense is not None:
        gP += dense.astype(np.float64).reshape(gP.shape)
    g, gp0, gv0 = oracle.adjoint(oracle.Problem.from_scenario(sc), P, V, gP)
    if dense is not None:
        gp0 = gp0 - dense.astype(np.float64).reshape(gP.shape).sum(axis=0)
    m = np.ones(n, bool) if mask is None else mask
    rows = list(g) + [gp0, gv0]
    refs = list(ref["g"]) + [ref["gp0"], ref["gv0"]]
    return [grad_close(a[m], b[m])[1] for a, b in zip(rows, refs)]
