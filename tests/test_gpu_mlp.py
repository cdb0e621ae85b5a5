"""The warm-start MLP kernels (BF16 MFMA, FP32 accumulation) against the FP64
oracle with BF16 rounding mirrored, the feature / lane-loss / lane-select
kernels, and a small end-to-end warm start."""
import numpy as np
import pytest

import oracle
import scenarios
from oracle import mlp as omlp
from _util import grad_close
from gpu_run import device_inputs, log

pytestmark = pytest.mark.gpu


def _net(seed=3, bias_scale=0.1):
    rng = np.random.default_rng(seed)
    theta = scenarios.mlp_init_params(seed).astype(np.float64)
    p = omlp.unpack(theta)
    p["b1"] = rng.normal(0, bias_scale, p["b1"].shape)
    p["b2"] = rng.normal(0, bias_scale, p["b2"].shape)
    p["b3"][:5] = rng.normal(0, bias_scale, 5)
    return omlp.pack(p).astype(np.float32)


def _batch(B, seed=0):
    import torch
    rng = np.random.default_rng(seed)
    X = np.zeros((B, omlp.IN_PAD), np.float32)
    X[:, :omlp.IN] = rng.normal(0, 1, (B, omlp.IN))
    U = rng.uniform(0, 1, (B, omlp.OUT)).astype(np.float32)
    Xt = torch.from_numpy(X).to(torch.bfloat16).cuda()
    return X, U, Xt, torch.from_numpy(U).cuda()


# 20000 rows: more than 64 slabs of 256 rows, so the slabs lengthen to 320
@pytest.mark.parametrize("B", [4096, 777, 64, 1, 20000])
def test_mlp_forward_and_gradients_match_oracle(B):
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    theta = _net()
    X, U, Xt, Ut = _batch(B)
    net = MLP(theta)
    Y = net.forward(Xt)
    G = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.gradients(Xt, Ut, G, loss)
    torch.cuda.synchronize()
    Yr, _ = omlp.forward(theta.astype(np.float64), X, mirror=True)
    Lr, Gr = omlp.loss_and_grad(theta.astype(np.float64), X, U, mirror=True)
    Yg = Y.double().cpu().numpy()
    err = np.abs(Yg[:, :5] - Yr[:, :5]).max()
    log("mlp B=%d: max |Y - Y_oracle| = %.3e (|Y| max %.3f), loss %.6e vs %.6e"
        % (B, err, np.abs(Yr[:, :5]).max(), loss.item(), Lr))
    assert err <= 1e-2 * max(1.0, np.abs(Yr[:, :5]).max())
    assert abs(loss.item() - Lr) <= 1e-2 * Lr
    g = G.double().cpu().numpy()
    sizes = np.cumsum([0] + [int(np.prod(s)) for _, s in omlp.SHAPES])
    for b, (name, _) in enumerate(omlp.SHAPES):
        a, r = g[sizes[b]:sizes[b + 1]], Gr[sizes[b]:sizes[b + 1]]
        nr = np.linalg.norm(r)
        rel = np.linalg.norm(a - r) / max(nr, 1e-30)
        # element by element: |g - r| <= 2e-2 max(|r|, 2e-2 max|r|) per block (a
        # mis-indexed slab row or a few wrong weights fail here, not in a norm)
        where = []
        ok_e, worst = grad_close(a, r, rtol=2e-2, rel_floor=2e-2, where=where)
        log("mlp B=%d: grad %s norm %.3e rel err %.3e, element worst/limit %.3f %s"
            % (B, name, nr, rel, worst, where))
        if nr > 0:
            assert rel <= 2e-2, name
            assert ok_e, (name, worst, where)
        else:
            assert np.all(a == 0.0), name


def test_mlp_forward_any_alignment_and_large_batch():
    """The forward stages X rows with 16-byte loads when X is 16-byte aligned
    and element loads otherwise: both give the same bits.  At 100,000 rows
    (1563 row tiles, ragged last tile) sampled rows match the oracle."""
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    theta = _net(seed=11)
    net = MLP(theta)
    B = 100_000
    X, _, Xt, _ = _batch(B, seed=9)
    Y = net.forward(Xt)
    buf = torch.zeros(B * omlp.IN_PAD + 1, dtype=torch.bfloat16, device="cuda")
    Xo = buf[1:].view(B, omlp.IN_PAD)
    Xo.copy_(Xt)
    assert Xo.data_ptr() % 16 != 0
    Yo = net.forward(Xo)
    torch.cuda.synchronize()
    assert torch.equal(Y, Yo)
    rows = np.r_[0, 1, 63, 64, 65, np.random.default_rng(2).integers(0, B, 200), B - 1]
    Yr, _ = omlp.forward(theta.astype(np.float64), X[rows], mirror=True)
    Yg = Y[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    err = np.abs(Yg[:, :5] - Yr[:, :5]).max()
    log("mlp B=%d: sampled rows max |Y - Y_oracle| = %.3e" % (B, err))
    assert err <= 1e-2 * max(1.0, np.abs(Yr[:, :5]).max())


def test_mlp_forward_small_and_large_launches_agree():
    """Batches of at most 256 row tiles take the launch that keeps every
    weight chunk of a layer in flight; larger ones the 3-waves-per-SIMD
    launch.  Same products in the same order: the same bits."""
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    net = MLP(_net(seed=8))
    _, _, Xt, _ = _batch(20000, seed=8)
    Y_large = net.forward(Xt)                   # 313 tiles
    Y_small = net.forward(Xt[:4096].contiguous())  # 64 tiles
    Y_edge = net.forward(Xt[:16384].contiguous())  # 256 tiles
    torch.cuda.synchronize()
    assert torch.equal(Y_large[:4096], Y_small)
    assert torch.equal(Y_large[:16384], Y_edge)


@pytest.mark.parametrize("B", [3000, 4096, 20000])
def test_train_step_is_adam_on_the_gradients(B):
    """The training step sums the weight gradients' split-K slabs inside its
    Adam kernel; the gradients entry point sums them in a kernel of its own.
    After one step the first moment is exactly (1 - beta1) g, the second
    (1 - beta2) g^2, for the g that idm_mlp_gradients returns (B = 3000 ends
    in a partial slab)."""
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    theta = _net(seed=4)
    _, _, Xt, Ut = _batch(B, seed=4)
    a, b = MLP(theta, lr=1e-3), MLP(theta, lr=1e-3)
    G = torch.empty(theta.size, dtype=torch.float32, device="cuda")
    a.gradients(Xt, Ut, G)
    b.train_step(Xt, Ut)
    torch.cuda.synchronize()
    one = torch.tensor(1.0, dtype=torch.float32)
    c1 = (one - torch.tensor(0.9, dtype=torch.float32)).item()
    c2 = (one - torch.tensor(0.999, dtype=torch.float32)).item()
    assert torch.count_nonzero(G) > 0.9 * G.numel()
    assert torch.equal(b.m, G * c1)
    assert torch.equal(b.v, (G * c2) * G)
    log("mlp B=%d: train step moments match the gradients entry point" % B)


def test_mlp_training_reduces_loss():
    """Adam steps on a learnable target (u = sigmoid of a fixed projection of X)."""
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    rng = np.random.default_rng(5)
    B = 4096
    X = np.zeros((B, omlp.IN_PAD), np.float32)
    X[:, :omlp.IN] = rng.normal(0, 1, (B, omlp.IN))
    A = rng.normal(0, 0.15, (omlp.IN_PAD, 5))
    U = (1 / (1 + np.exp(-(X @ A)))).astype(np.float32)
    Xt = torch.from_numpy(X).to(torch.bfloat16).cuda()
    Ut = torch.from_numpy(U).cuda()
    net = MLP(scenarios.mlp_init_params(7), lr=1e-3)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    for _ in range(200):
        net.train_step(Xt, Ut, loss)
        losses.append(loss.item())
    log("mlp training: loss %.4e -> %.4e" % (losses[0], losses[-1]))
    assert losses[-1] < 0.2 * losses[0]
    # the BF16 copies track the FP32 masters
    w16 = net.w16.float().cpu().numpy()
    p = net.params.cpu().numpy()
    n1 = omlp.IN_PAD * omlp.HID
    w1 = torch.from_numpy(p[:n1]).to(torch.bfloat16).float().numpy()
    np.testing.assert_array_equal(w16[:n1], w1)
    # and the transposed copy of W1 that follows the three plain copies
    t1 = n1 + omlp.HID * omlp.HID + omlp.HID * omlp.OUT_PAD
    np.testing.assert_array_equal(w16[t1:t1 + n1].reshape(omlp.HID, omlp.IN_PAD),
                                  w1.reshape(omlp.IN_PAD, omlp.HID).T)


def test_bf16_copies_round_like_torch_at_special_values():
    """The BF16 weight copies (hardware conversion) equal torch's float32 ->
    bfloat16 rounding: halfway cases to even, values next to them, subnormals,
    signed zeros, the largest finite value, infinities; NaN stays NaN."""
    import torch
    from paper_2412_16750_amd.warmstart import MLP
    n1 = omlp.IN_PAD * omlp.HID
    theta = _net(seed=2)
    one = np.float32(1.0)
    ulp = np.float32(2.0 ** -7)
    special = np.array([
        one + ulp / 2,                      # tie, rounds down to even (1.0)
        one + 3 * ulp / 2,                  # tie, rounds up to even
        np.nextafter(one + ulp / 2, np.float32(2)),   # just above the tie
        np.nextafter(one + ulp / 2, np.float32(0)),   # just below the tie
        -(one + 3 * ulp / 2),
        np.float32(1e-40), np.float32(-3e-39), np.float32(1.5e-45),  # subnormals
        np.float32(0.0), np.float32(-0.0),
        np.finfo(np.float32).max,           # rounds up to infinity
        np.float32(np.inf), np.float32(-np.inf),
        np.float32(3.3895314e38),           # the largest finite BF16 value
        np.float32(np.nan),
    ], dtype=np.float32)
    theta[:special.size] = special
    net = MLP(theta)
    torch.cuda.synchronize()
    got = net.w16[:n1].cpu()
    want = torch.from_numpy(theta[:n1].copy()).to(torch.bfloat16)
    nan = torch.isnan(want.float())
    assert torch.equal(torch.isnan(got.float()), nan)
    gb, wb = got.view(torch.int16)[~nan], want.view(torch.int16)[~nan]
    bad = (gb != wb).nonzero().flatten()[:5].tolist()
    assert not bad, [(float(theta[:n1][~nan.numpy()][j]), int(gb[j]), int(wb[j])) for j in bad]


def test_features_lane_loss_and_selection():
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd import warmstart as ws
    sizes = [40, 1, 25, 0, 70]
    sc = scenarios.make_scenario("feat", scenarios.offsets_from_sizes(sizes), 100, 9, ckpt_every=16)
    plan = sim.Plan.for_scenario(sc)
    x = device_inputs(sc)
    traj = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], traj, None, None)
    noise = torch.from_numpy(scenarios.noise((10, sc.n), 9).astype(np.float32)).cuda()
    tgt = ws.observe(plan, traj, x["p0"], noise, 10, 10, 10)
    d = traj.double().cpu().numpy()
    exp_tgt = (sc.p0[None, :] + d[10::10] + noise.double().cpu().numpy()).astype(np.float32)
    np.testing.assert_array_equal(tgt.cpu().numpy(), exp_tgt)
    obs = sim.Obs(tgt, 10, 10)
    X = ws.features(plan, obs, x["p0"], x["length"])
    F = oracle.mlp.features(tgt.cpu().numpy(), 10, 10, sc.dt, sc.p0, sc.params["length"],
                            sc.lane_offsets)
    ref = omlp.bf16(F.astype(np.float32))
    got = X.float().double().cpu().numpy()
    bad = np.abs(got - ref) > np.abs(ref) * 2 ** -7  # at most one BF16 ulp apart
    log("features: %d of %d values differ by more than one BF16 ulp" % (bad.sum(), bad.size))
    assert not bad.any()
    assert np.mean(got == ref) > 0.99
    # rows written through 2-byte stores when X is not 4-byte aligned: same bits
    buf = torch.zeros(sc.n * omlp.IN_PAD + 1, dtype=torch.bfloat16, device="cuda")
    Xo = ws.features(plan, obs, x["p0"], x["length"], X=buf[1:].view(sc.n, omlp.IN_PAD))
    assert Xo.data_ptr() % 4 != 0
    assert torch.equal(Xo, X)
    # per-lane observed squared error
    ll = ws.lane_loss(plan, traj, x["p0"], obs).cpu().numpy()
    P = sc.p0[None, :] + d
    r = P[10::10] - tgt.double().cpu().numpy()
    per_vehicle = (r * r).sum(axis=0)
    off = sc.lane_offsets
    expect = np.array([per_vehicle[off[l]:off[l + 1]].sum() for l in range(len(sizes))])
    np.testing.assert_allclose(ll, expect, rtol=1e-12, atol=1e-12)
    # per-lane choice
    la = torch.tensor([1.0, 5.0, 2.0, 0.0, 9.0], dtype=torch.float64, device="cuda")
    lb = torch.tensor([2.0, 4.0, 2.0, 1.0, 1.0], dtype=torch.float64, device="cuda")
    pa = torch.full((5, sc.n), 1.0, device="cuda")
    pb = torch.full((5, sc.n), 2.0, device="cuda")
    out, chose = ws.select_by_lane(plan, la, lb, pa, pb)
    lane_of = np.repeat(np.arange(len(sizes)), sizes)
    want_a = (la.cpu().numpy() <= lb.cpu().numpy())[lane_of]
    assert np.array_equal(chose.cpu().numpy().astype(bool), want_a)
    assert np.array_equal(out.cpu().numpy(), np.where(want_a[None, :], 1.0, 2.0).repeat(1, 0) * np.ones((5, 1)))


def test_warm_start_end_to_end_small():
    """Train on 200k simulated pairs, then warm vs cold fit on a held-out
    4-lane problem: the warm start begins closer to the hidden trajectory and
    reaches 0.5 m RMSE in fewer iterations."""
    import torch
    from paper_2412_16750_amd import sim
    from paper_2412_16750_amd import warmstart as ws
    from paper_2412_16750_amd.fit import Fitter
    train_sc = scenarios.warm_training(n_lanes=200, lane_len=1000)
    data = ws.make_pairs(train_sc)
    net = ws.MLP(scenarios.mlp_init_params(11), lr=1e-3)
    rep = ws.train(net, data, batch=4096, epochs=4, log=log)
    assert rep["history"][-1]["train_mse"] < 0.5 * rep["history"][0]["train_mse"]
    sc = scenarios.fit(n_lanes=4, lane_len=1000)
    plan = sim.Plan.for_scenario(sc)
    x = device_inputs(sc)
    hidden = torch.empty(sc.n_steps + 1, sc.n, dtype=torch.float32, device="cuda")
    sim.idm_sim_forward(plan, x["prm"], x["length"], x["p0"], x["v"], hidden, None, None)
    noise = torch.from_numpy(scenarios.noise((50, sc.n), 4).astype(np.float32)).cuda()
    tgt = ws.observe(plan, hidden, x["p0"], noise, 10, 10, 50)
    obs = sim.Obs(tgt, 10, 10)
    cold = sim.params_tensor(scenarios.cold_params(sc))
    res = {}
    for mode in ("cold", "warm"):
        f = Fitter(plan, x["length"], x["p0"], x["v"], obs, lr0=1e-2)
        if mode == "cold":
            f.init(cold)
        else:
            info = ws.warm_init(f, net, plan, obs, x["p0"], x["v"], x["length"], cold)
            log("warm start: %s" % info)
        res[mode] = ws.fit_until(f, plan, x["length"], x["p0"], x["v"], hidden, 0.5, chunk=10,
                                 cap=600)
        log("%s: start RMSE %.3f m, %d iterations, final %.3f m"
            % (mode, res[mode]["curve"][0][1], res[mode]["iterations"], res[mode]["rmse"]))
    assert res["warm"]["curve"][0][1] < res["cold"]["curve"][0][1]
    assert res["warm"]["reached"] and res["warm"]["iterations"] < res["cold"]["iterations"]


def _random_pairs(n, seed):
    import torch
    from paper_2412_16750_amd import warmstart as ws
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = torch.zeros(n, 160)
    X[:, :150] = torch.randn(n, 150, generator=g)
    U = torch.rand(n, 5, generator=g)
    return ws.Dataset(X.to(torch.bfloat16).cuda(), U.cuda())


def test_scheduled_training_step_graph_replays_match_eager_steps():
    """Scheduled training steps captured in a HIP graph (one step, and an
    epoch of three steps) and replayed: after every replay (with unrelated
    eager work and synchronisations between the replays) the weights, BF16
    copies, Adam moments, step counter and loss history equal those of the
    same number of eager calls, bit for bit, across changes of the row
    permutation (new epochs)."""
    import torch
    from paper_2412_16750_amd import warmstart as ws
    data = _random_pairs(3 * 512 + 100, 41)
    for per_graph in (1, 3):
        _graph_vs_eager(ws, data, per_graph)


def _graph_vs_eager(ws, data, per_graph):
    import torch
    nets = [ws.MLP(scenarios.mlp_init_params(12), lr=2e-3) for _ in range(2)]
    trs = [ws.ScheduledTrainer(n, data, 512, total_steps=9, lr_final=1e-4) for n in nets]
    eager, graph = trs
    graph.capture(per_graph)
    gen = torch.Generator(device="cpu").manual_seed(5)
    for step in range(0, 9, per_graph):
        if step % 3 == 0:
            perm = torch.randperm(data.X.shape[0], generator=gen)
            for t in trs:
                t.set_permutation(perm)
        for _ in range(per_graph):
            eager.step()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").square().sum()  # unrelated eager work
        torch.cuda.synchronize()
        del junk
        a, b = nets
        for x, y in ((a.params, b.params), (a.w16, b.w16), (a.m, b.m), (a.v, b.v)):
            assert torch.equal(x, y), step
        assert eager.steps_done() == graph.steps_done() == step + per_graph
        assert torch.equal(eager.loss_hist, graph.loss_hist)
    log("scheduled MLP steps, %d per graph: losses %s" % (per_graph, eager.loss_hist.cpu().numpy()))


def test_scheduled_training_step_is_the_train_step_with_the_cosine_rate():
    """The scheduled step on the permuted rows equals idm_mlp_train_step on
    the same rows (index_select) with the learning rate of the cosine computed
    on the host: same weights to FP32 rounding of the rate, same losses."""
    import math
    import torch
    from paper_2412_16750_amd import warmstart as ws
    data = _random_pairs(2 * 512, 42)
    a = ws.MLP(scenarios.mlp_init_params(13), lr=3e-3)
    b = ws.MLP(scenarios.mlp_init_params(13), lr=3e-3)
    total, lr0, lr1 = 4, 3e-3, 2e-4
    tr = ws.ScheduledTrainer(a, data, 512, total_steps=total, lr_final=lr1)
    perm = torch.randperm(data.X.shape[0], generator=torch.Generator().manual_seed(3))
    tr.set_permutation(perm)
    pd = perm.cuda()
    losses = []
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for t in range(1, total + 1):
        tr.step()
        rows = pd[((t - 1) % 2) * 512:((t - 1) % 2 + 1) * 512]
        b._st.lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * (t - 1) / total))
        b.train_step(data.X.index_select(0, rows).contiguous(),
                     data.U.index_select(0, rows).contiguous(), loss)
        losses.append(float(loss.item()))
    torch.cuda.synchronize()
    pa, pb = a.params.double().cpu().numpy(), b.params.double().cpu().numpy()
    rel = float(np.max(np.abs(pa - pb)) / np.max(np.abs(pb)))
    log("scheduled vs train_step: max param diff / max |param| %.2e, losses %s vs %s"
        % (rel, tr.loss_hist.cpu().numpy()[:total], losses))
    assert rel <= 1e-6
    # the history holds one epoch (2 batches): steps 3 and 4 after four steps
    assert np.allclose(tr.loss_hist.cpu().numpy(), losses[2:4], rtol=1e-6, atol=0.0)
