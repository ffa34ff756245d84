"""The learned warm-start pipeline on the GPU: network gradients chained
through the layers against the FP64 oracle, and a small end-to-end run."""
import numpy as np
import pytest

from oracle import nn

pytestmark = pytest.mark.gpu


def _h(t):
    return t.detach().double().cpu().numpy()


def test_network_gradients_match_oracle_chain(gpu_lib):
    """Forward/backward of the 4-layer net: each layer's weight gradient equals
    the oracle's, given the same bfloat16 activations and incoming gradient."""
    import torch

    from paper_1602_05700_amd import warmstart as ws

    net = ws.Net.create("cuda", seed=3)
    for i in range(ws.N_LAYERS):  # non-trivial biases and last-layer weights
        net.b[i] += 0.05 * torch.arange(16, device="cuda", dtype=torch.float32) / 16
        net.w16[i] = net.w[i].to(torch.bfloat16)
    rng = np.random.default_rng(0)
    planar = torch.from_numpy(rng.standard_normal((2, 2, 4, 6, 16)).astype(np.float32)).cuda()
    x = ws.pack(planar)
    acts = net.forward(x)
    g = torch.from_numpy(nn.bf16_round(rng.standard_normal((2, 4, 6, 16, 16)).astype(np.float32))).cuda()
    g = g.to(torch.bfloat16)
    grads, _ = net.backward(acts, g)
    # replay the backward in the oracle, layer by layer, with the GPU's activations
    gin = _h(g)
    for i in range(ws.N_LAYERS - 1, -1, -1):
        a = _h(acts[i])
        w = _h(net.w16[i])
        dw_ref = nn.conv3d_grad_weight(a, gin)
        assert np.max(np.abs(_h(grads[i][0]) - dw_ref)) <= 2e-5 * np.max(np.abs(dw_ref)) + 1e-12
        assert np.allclose(_h(grads[i][1]), nn.conv3d_grad_bias(gin), rtol=2e-5, atol=1e-9)
        if i > 0:
            gin = nn.bf16_round(nn.tanh_grad(a, nn.conv3d_grad_input(gin, w)).astype(np.float32))
    # the forward itself
    ref = _h(acts[0])
    for i in range(ws.N_LAYERS):
        z = nn.conv3d(ref, _h(net.w16[i]), _h(net.b[i]))
        ref = z if i == ws.N_LAYERS - 1 else nn.bf16_round(np.tanh(z).astype(np.float32))
        got = _h(acts[i + 1])
        assert np.max(np.abs(got - ref)) <= 2 ** -7 * np.max(np.abs(ref)) + 1e-6


def test_small_end_to_end(gpu_lib):
    """n = 32: coarse cue, targets, a few Adam steps (loss decreases) and a
    finite fine-grid prediction accepted by set_state."""
    import torch

    import workloads
    from paper_1602_05700_amd import hgs, warmstart as ws

    n = 32
    feats = ws.Features(n, "cuda", coarse_steps=60)
    rho = torch.stack([workloads.blob_density_torch(n, workloads.warmstart_blobs(s), "cuda", torch.float32)
                       for s in range(5)])
    planar, phi2, scale = feats.inputs(rho)
    assert planar.shape == (5, 3, 16, 16, 16) and torch.isfinite(planar).all()
    phis, res = ws.converged_phi(list(rho), n, "cuda", steps=600)
    assert max(res) < 1e-8
    ex2 = torch.empty_like(phi2)
    hgs.nn_restrict2(torch.stack([p.float() for p in phis]), ex2)
    corr = (ex2 - phi2) / scale.view(-1, 1, 1, 1)
    net = ws.Net.create("cuda", seed=1)
    net.out_scale = float(1.0 / corr.std().item())
    tgt = torch.zeros((5, 2, 16, 16, 16), dtype=torch.float32, device="cuda")
    tgt[:, 0] = corr * net.out_scale
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    parts = torch.empty(hgs.NN_MSE_PARTIALS, dtype=torch.float64, device="cuda")
    losses = []
    wsb = None
    for it in range(60):
        x = ws.pack(planar)
        acts = net.forward(x)
        grad = torch.empty_like(x)
        hgs.nn_mse(acts[-1], tgt, grad, loss, parts)
        grads, wsb = net.backward(acts, grad, wsb)
        net.adam_step(grads, 3e-3)
        losses.append(loss.item())
    assert losses[-1] < 0.5 * losses[0]
    phi, pd = ws.predict_fine(net, planar[:1].contiguous(), phi2[:1].contiguous(), scale[:1], n)
    assert phi.shape == (1, n, n, n) and torch.isfinite(phi).all() and torch.isfinite(pd).all()
    steps, r0, rb, _ = ws.steps_to_tolerance(rho[0], n, 1e-4, start=(phi[0], pd[0]))
    assert rb < 1e-4 and steps < 4000


def test_committed_weights_cut_steps_threefold(gpu_lib):
    """The trained network shipped with the package, on held-out 128^3
    densities: substeps of the damped FP32 solver to R_b < 1e-4 from its warm
    start (through start_solver, the coarse cue counted in fine-substep
    equivalents) against the zero start.  The median gain must reach 3x with
    no fallback to the zero start."""
    import os

    import torch

    import workloads
    from paper_1602_05700_amd import warmstart as ws

    assert os.path.exists(ws.WEIGHTS)
    n = 128
    net = ws.Net.load(ws.WEIGHTS, "cuda")
    feats = ws.Features(n, "cuda", coarse_steps=net.coarse_steps)
    seeds = list(range(20000, 20006))
    rho = torch.stack([workloads.blob_density_torch(n, workloads.warmstart_blobs(s), "cuda", torch.float32)
                       for s in seeds])
    planar, phi2, scale = feats.inputs(rho)
    phi, pd = ws.predict_fine(net, planar, phi2, scale, n)
    ratios = []
    for i in range(len(seeds)):
        zero = ws.steps_to_tolerance(rho[i], n, 1e-4)
        warm = ws.steps_to_tolerance(rho[i], n, 1e-4, start=(phi[i], pd[i]))
        assert warm[3] and warm[1] < zero[1] and warm[2] < 1e-4
        ratios.append(zero[0] / (warm[0] + feats.coarse_cost_fine_steps))
    assert np.median(ratios) >= 3.0, ratios


def test_start_solver_falls_back_to_zero(gpu_lib):
    """start_solver keeps a start whose residual R_b is below the zero start's
    (1) and otherwise resets the solver to zero: a start far off the solution
    (R_b > 1) is refused, the state is then zero, and the direct Poisson
    solution of the same density (R_b ~ 0) is kept."""
    import torch

    import workloads
    from paper_1602_05700_amd import hgs, warmstart as ws

    n = 32
    dx = 2.0 / n
    rho = workloads.blob_density_torch(n, workloads.warmstart_blobs(3), "cuda", torch.float32)
    s = hgs.Solver(n, storage="f32", lmax=4, eta=ws.eta_critical(n, dx))
    bad = torch.full((n, n, n), 50.0, dtype=torch.float32, device="cuda")
    assert ws.start_solver(s, rho, bad, None, 0.4 * dx).item() == 0
    phi, pd = s.potential()
    assert torch.count_nonzero(phi) == 0 and torch.count_nonzero(pd) == 0
    assert s.residual(rho)[0] == pytest.approx(1.0, abs=1e-12)  # the zero start, with rho's ghosts
    nan = bad.clone()
    nan[3, 4, 5] = float("nan")
    assert ws.start_solver(s, rho, nan, None, 0.4 * dx).item() == 0
    assert torch.count_nonzero(s.potential(with_phidot=False)[0]) == 0
    ref = hgs.Solver(n, storage="f32", lmax=4)
    ref.poisson_direct(rho)
    good = ref.potential(with_phidot=False)[0]
    assert ws.start_solver(s, rho, good, torch.zeros_like(good), 0.4 * dx).item() == 1
    assert torch.equal(s.potential(with_phidot=False)[0], good)
    assert s.residual(rho)[0] < 1e-5
    r = hgs.Solver(n, storage="f32", bc="robin")
    with pytest.raises(hgs.HGSError):
        r.keep_start_if_better(rho)


def test_captured_predictor_matches_eager_prediction(gpu_lib):
    """The graph-captured prediction equals the eager one bit for bit, replay
    after replay, with other densities and eager library work in between."""
    import torch

    import workloads
    from paper_1602_05700_amd import hgs, warmstart as ws

    n = 64
    net = ws.Net.load(ws.WEIGHTS, "cuda")
    pred = ws.Predictor(net, n, B=1, device="cuda")
    feats = ws.Features(n, "cuda", coarse_steps=net.coarse_steps)
    other = hgs.Solver(32, storage="f32", lmax=4, eta=1.0)
    r_other = workloads.blob_density_torch(32, workloads.warmstart_blobs(99), "cuda", torch.float32)
    for seed in (20000, 20001, 20000, 20002):
        rho = workloads.blob_density_torch(n, workloads.warmstart_blobs(seed), "cuda", torch.float32)[None]
        planar, phi2, scale = feats.inputs(rho)
        want = ws.predict_fine(net, planar, phi2, scale, n)
        got = pred(rho)
        torch.cuda.synchronize()
        assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1]), seed
        other.step(r_other, 1.0, 0.4 * 2 / 32, 8)  # eager work between replays
        torch.cuda.synchronize()
