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
