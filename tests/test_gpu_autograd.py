"""The torch.autograd.Function around the hand-written adjoint, checked against
the FP64 oracle's adjoint and against central finite differences of the
oracle's forward simulation."""
import numpy as np
import pytest

import oracle
from _util import grad_close, oracle_reference, ragged_scenario
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _setup(sizes=(6, 4), S=150, seed=3):
    import torch
    from paper_2412_16750_amd import sim
    sc = ragged_scenario(list(sizes), S, ckpt_every=16)
    plan = sim.Plan.for_scenario(sc)
    x = device_inputs(sc)
    rng = np.random.default_rng(seed)
    W = rng.normal(0, 1.0, size=(S + 1, sc.n)).astype(np.float32)
    return sc, plan, x, W, torch.from_numpy(W).cuda()


def test_autograd_gradients_match_oracle_adjoint():
    import torch
    from paper_2412_16750_amd.autograd import simulate
    sc, plan, x, W, Wt = _setup()
    params = x["prm"].clone().requires_grad_(True)
    p0 = x["p0"].clone().requires_grad_(True)
    v = x["v"].clone().requires_grad_(True)
    d = simulate(plan, params, p0, v, x["length"])
    loss = (d.double() * Wt.double()).sum()
    loss.backward()
    ref = oracle_reference(sc, dense=W)
    okg, wg = grad_close(params.grad.double().cpu().numpy(), ref["g"])
    ok0, w0 = grad_close(p0.grad.cpu().numpy(), ref["gp0"])
    ok1, w1 = grad_close(v.grad.double().cpu().numpy(), ref["gv0"])
    log("autograd vs oracle adjoint: worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1
    # positions p0 + d: autograd adds the direct term; compare with the oracle's
    # total derivative for L = sum W * P
    p0b = x["p0"].clone().requires_grad_(True)
    d2 = simulate(plan, x["prm"], p0b, x["v"], x["length"])
    P = p0b[None, :] + d2.double()
    (P * Wt.double()).sum().backward()
    import scenarios  # noqa: F401
    pb = oracle.Problem.from_scenario(sc)
    Pr, Vr, _, _ = oracle.forward(pb)
    _, gp0_total, _ = oracle.adjoint(pb, Pr, Vr, W.astype(np.float64))
    ok, w = grad_close(p0b.grad.cpu().numpy(), gp0_total)
    log("autograd positions vs oracle total dL/dp0: worst/limit %.3f" % w)
    assert ok


def test_autograd_gradients_match_central_differences():
    """Central differences (FP64 oracle forward, h = 1e-6 max(1, |x|)) of
    L = sum W * d for every parameter of every vehicle and both initial states."""
    from paper_2412_16750_amd.autograd import simulate
    sc, plan, x, W, Wt = _setup(sizes=(5, 3), S=120, seed=4)
    params = x["prm"].clone().requires_grad_(True)
    p0 = x["p0"].clone().requires_grad_(True)
    v = x["v"].clone().requires_grad_(True)
    d = simulate(plan, params, p0, v, x["length"])
    (d.double() * Wt.double()).sum().backward()
    g_gpu = params.grad.double().cpu().numpy()
    pb = oracle.Problem.from_scenario(sc)

    def L():
        P, _, _, _ = oracle.forward(pb)
        return float(np.sum(W.astype(np.float64) * (P - pb.p0[None, :])))

    fd = np.zeros((5, sc.n))
    for j, name in enumerate(oracle.PARAM_NAMES):
        for i in range(sc.n):
            b = pb.params[name][i]
            h = 1e-6 * max(1.0, abs(b))
            pb.params[name][i] = b + h
            lp = L()
            pb.params[name][i] = b - h
            lm = L()
            pb.params[name][i] = b
            fd[j, i] = (lp - lm) / (2 * h)
    fd0 = np.zeros(sc.n)
    fdv = np.zeros(sc.n)
    for arr, out in ((pb.p0, fd0), (pb.v_init, fdv)):
        for i in range(sc.n):
            b = arr[i]
            h = 1e-6 * max(1.0, abs(b))
            arr[i] = b + h
            lp = L()
            arr[i] = b - h
            lm = L()
            arr[i] = b
            out[i] = (lp - lm) / (2 * h)
    okg, wg = grad_close(g_gpu, fd)
    ok0, w0 = grad_close(p0.grad.cpu().numpy(), fd0)
    ok1, w1 = grad_close(v.grad.double().cpu().numpy(), fdv)
    log("autograd vs central differences: worst/limit %.3f %.3f %.3f" % (wg, w0, w1))
    assert okg and ok0 and ok1


def test_autograd_two_forwards_before_backward():
    """Each forward owns its checkpoints, so interleaved graphs stay correct."""
    from paper_2412_16750_amd.autograd import simulate
    sc, plan, x, W, Wt = _setup(seed=5)
    p1 = x["prm"].clone().requires_grad_(True)
    p2 = (x["prm"] * 1.01).requires_grad_(True)
    d1 = simulate(plan, p1, x["p0"], x["v"], x["length"])
    d2 = simulate(plan, p2, x["p0"], x["v"], x["length"])
    ((d1 + d2) * Wt).sum().backward()
    ref1 = oracle_reference(sc, dense=W)
    ok, w = grad_close(p1.grad.double().cpu().numpy(), ref1["g"])
    assert ok, w
