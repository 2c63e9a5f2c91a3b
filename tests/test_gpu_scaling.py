"""GPU parity of the learned-scaling pieces against the FP64 oracle:
features and targets (FP64 device arithmetic stored in FP32 -> 1e-6
relative); the BF16 network forward and gradients against the FP64 oracle
whose matrix-product operands are rounded to BF16 exactly where the device
rounds them, so only FP32 accumulation order (and an occasional one-ulp BF16
flip after tanhf) differs (1e-3 relative per parameter block; the unrounded FP64 gradient is reported and within 0.1:
BF16 operands in back-propagation lose up to a few percent to cancellation);
training (the loss falls, bitwise reproducibly) and the gain of S P^-1 S
over P."""
import numpy as np
import pytest

import synth
from helpers import rel, to_dev, to_host
from oracle import assembly, fd, mlp as omlp, pcg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


def _torch():
    import torch
    return torch


def bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("prob", [synth.uniform_problem(3, [5, 6, 4], 3, geometry=synth.warped_geometry(3),
                                                        coefficient=synth.sincos_coefficient(0.5, 1, 2, 0.3, 0.1)),
                                  synth.uniform_problem(2, [9, 7], 2, geometry={"kind": "ring"})])
def test_features_and_targets_match_oracle(api, prob):
    torch = _torch()
    with api.igafd_setup(prob) as ctx:
        f = torch.empty(ctx.N * 8, dtype=torch.float32, device="cuda")
        t = torch.empty(ctx.N, dtype=torch.float32, device="cuda")
        api.igafd_features(ctx, f)
        api.igafd_scaling_targets(ctx, t)
        fo = omlp.features(prob)
        np.testing.assert_allclose(to_host(f).reshape(-1, 8), fo, rtol=2e-6, atol=2e-7)
        np.testing.assert_allclose(to_host(t), omlp.targets(prob), rtol=1e-5, atol=1e-6)


def _random_batch(n, seed):
    rng = np.random.default_rng(seed)
    feat = rng.standard_normal((n, 8)).astype(np.float32)
    feat[:, 7] = rng.integers(2, 6, n)
    target = (0.3 * np.tanh(feat[:, 0]) + 0.1 * feat[:, 6]).astype(np.float32)
    return feat, target


def test_forward_and_gradient_match_fp64(api):
    torch = _torch()
    m = api.igafd_mlp_create(seed=5)
    n = 1000  # several 16-sample groups per wave and a ragged tail
    feat, target = _random_batch(n, 1)
    fd_ = torch.from_numpy(feat.reshape(-1)).cuda()
    td = torch.from_numpy(target).cuda()
    api.igafd_mlp_fit_normalization(m, fd_, n)
    params = api.igafd_mlp_get_params(m)
    npar = api.igafd_mlp_num_params()
    theta = params[:npar].astype(np.float64)
    mean, inv_std = params[npar:npar + 8].astype(np.float64), params[npar + 8:].astype(np.float64)
    np.testing.assert_allclose(mean, feat.mean(0), rtol=1e-5, atol=1e-6)
    # the device normalises in FP32 and feeds BF16-rounded operands to every
    # matrix product; the oracle gets the same normalised inputs and rounding
    fn = ((feat - params[npar:npar + 8]) * params[npar + 8:]).astype(np.float32).astype(np.float64)
    zero, one = np.zeros(8), np.ones(8)
    t_ref, _ = omlp.forward(theta, zero, one, fn, rnd=bf16_round)
    tout = torch.empty(n, dtype=torch.float32, device="cuda")
    api.igafd_mlp_forward(m, fd_, n, t=tout)
    # FP32 accumulation order, tanhf vs tanh: an occasional one-ulp BF16 flip
    assert np.max(np.abs(to_host(tout) - t_ref)) <= 1e-3 * max(1.0, np.abs(t_ref).max())
    L_ref, g_ref = omlp.loss_and_grad(theta, zero, one, fn, target, rnd=bf16_round)
    _, g_exact = omlp.loss_and_grad(theta, zero, one, fn, target)
    L, g = api.igafd_mlp_gradient(m, fd_, td, n)
    assert abs(L - L_ref) <= 1e-3 * L_ref
    k = 0
    for name, shape in omlp.SIZES:
        size = int(np.prod(shape))
        a = g[k:k + size].astype(np.float64)
        assert rel(a, g_ref[k:k + size]) < 1e-3, (name, rel(a, g_ref[k:k + size]))
        assert rel(a, g_exact[k:k + size]) < 1e-1, (name, rel(a, g_exact[k:k + size]))
        k += size
    m.close()


def test_training_reduces_loss_and_is_deterministic(api):
    torch = _torch()
    n = 4096
    feat, target = _random_batch(n, 2)
    fd_ = torch.from_numpy(feat.reshape(-1)).cuda()
    td = torch.from_numpy(target).cuda()
    losses = []
    finals = []
    for _ in range(2):
        m = api.igafd_mlp_create(seed=3)
        api.igafd_mlp_fit_normalization(m, fd_, n)
        L0, _ = api.igafd_mlp_gradient(m, fd_, td, n)
        for it in range(150):
            api.igafd_mlp_train_step(m, fd_, td, n, 3e-3)
        L1, _ = api.igafd_mlp_gradient(m, fd_, td, n)
        losses.append((L0, L1))
        finals.append(api.igafd_mlp_get_params(m))
        m.close()
    assert losses[0][1] < 0.1 * losses[0][0]
    assert np.array_equal(finals[0], finals[1])


def test_learned_scaling_gains_over_plain(api):
    # train on small seeded warped cubes, evaluate on an unseen one: fewer
    # iterations than plain P; the exact diagonal ratio is reported beside it
    torch = _torch()
    from paper_1602_01636_amd import scaling
    probs = [synth.training_problem(s) for s in range(60)]
    feat, targ, total = scaling.build_dataset(probs)
    m = api.igafd_mlp_create(seed=0)
    hist = scaling.train(m, feat, targ, total, epochs=30, batch=4096)
    assert hist[-1] < hist[0]
    prob = synth.warped_cube(E=24, p=4, seed=10000)
    with api.igafd_setup(prob) as ctx:
        b = torch.zeros(ctx.N, dtype=torch.float64, device="cuda")
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u = torch.zeros_like(b)
        plain = api.igafd_solve(ctx, b, u)
        u_plain = u.clone()
        scaling.predict_scaling(m, ctx)
        learned = api.igafd_solve(ctx, b, u, use_scaling=True)
        assert learned["true_relres"] <= 1e-8 and not learned["fallback"]
        assert rel(to_host(u), to_host(u_plain)) < 1e-6
        api.igafd_set_scaling_diag_ratio(ctx)
        exact = api.igafd_solve(ctx, b, u, use_scaling=True)
        print(f"iterations: plain {plain['iters']} learned {learned['iters']} exact-ratio {exact['iters']}")
        assert learned["iters"] < plain["iters"]
    m.close()


def test_scaled_solve_matches_oracle(api):
    prob = synth.uniform_problem(3, [6, 5, 7], 3, geometry=synth.warped_geometry(4),
                                 coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.0, 0.0))
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    S = np.exp(omlp.targets(prob, A))
    u_or, info_or = pcg.solve(prob, A, F, b, scaling=S)
    with api.igafd_setup(prob) as ctx:
        api.igafd_set_scaling_diag_ratio(ctx)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, use_scaling=True)
        assert abs(info["iters"] - info_or["iters"]) <= 1
        assert rel(to_host(u), u_or) <= 1e-7
