"""Training and use of the learned diagonal scaling S P^-1 S.

Orchestration only: every arithmetic step (assembly, features, targets,
forward/backward passes, Adam, the solves) runs in libigafd.so through the C
ABI.  Training pairs come from the solver's own assembly on seeded warped
cubes with random coefficients (inputs: per-dof statistics of
|det J| J^-1 J^-T and kappa, plus p; target: 1/2 log(P_ii / A_ii)).
"""
from __future__ import annotations

import numpy as np

import synth

from . import binding as B


def _dofs(problem):
    p = problem["degree"]
    return int(np.prod([len(k) - p - 3 for k in problem["knots"]]))


def build_dataset(problems, shuffle_seed=0, log=None):
    """Features (M x 8 float32) and targets (M float32) on the device, rows of
    all problems concatenated and then shuffled once."""
    import torch
    sizes = [_dofs(pr) for pr in problems]
    total = sum(sizes)
    feat = torch.empty(total * 8, dtype=torch.float32, device="cuda")
    targ = torch.empty(total, dtype=torch.float32, device="cuda")
    off = 0
    for k, (pr, n) in enumerate(zip(problems, sizes)):
        with B.igafd_setup(pr, features=True) as ctx:  # features summed by the assembly itself
            B.igafd_features(ctx, feat[off * 8:(off + n) * 8])
            B.igafd_scaling_targets(ctx, targ[off:off + n])
        off += n
        if log and (k + 1) % 250 == 0:
            log(f"dataset: {k + 1} of {len(problems)} problems")
    g = torch.Generator(device="cuda").manual_seed(shuffle_seed)
    perm = torch.randperm(total, device="cuda", generator=g)
    feat = feat.view(total, 8)[perm].contiguous().view(-1)
    targ = targ[perm].contiguous()
    return feat, targ, total


def train(mlp, feat, targ, total, epochs=20, batch=8192, lr=3e-3, lr_final=3e-4, log=None):
    """Adam over contiguous minibatches of the shuffled set; cosine-free
    geometric learning-rate decay from lr to lr_final.  Returns the loss history."""
    B.igafd_mlp_fit_normalization(mlp, feat, total)
    steps = epochs * ((total + batch - 1) // batch)
    gamma = (lr_final / lr) ** (1.0 / max(1, steps - 1))
    hist = []
    k = 0
    for ep in range(epochs):
        for s in range(0, total, batch):
            n = min(batch, total - s)
            last = s + batch >= total
            loss = B.igafd_mlp_train_step(mlp, feat[s * 8:(s + n) * 8], targ[s:s + n], n, lr * gamma ** k,
                                          want_loss=last)
            k += 1
        hist.append(loss)
        if log:
            log(f"epoch {ep}: last-batch loss {loss:.3e}")
    return hist


def predict_scaling(mlp, ctx):
    """S = exp(MLP(features)) for the problem of ctx, set on ctx; returns S.
    With a context set up with features=True the features are a copy of
    what the assembly summed."""
    import torch
    feat = torch.empty(ctx.N * 8, dtype=torch.float32, device="cuda")
    B.igafd_features(ctx, feat)
    S = torch.empty(ctx.N, dtype=torch.float64, device="cuda")
    B.igafd_mlp_forward(mlp, feat, ctx.N, S=S)
    B.igafd_set_scaling(ctx, S)
    return S


def train_default(n_train=2000, seed=0, epochs=20, log=None):
    """The standard training run: seeds 0..n_train-1 of synth.training_problem."""
    import time
    t0 = time.perf_counter()
    probs = [synth.training_problem(s) for s in range(n_train)]
    feat, targ, total = build_dataset(probs, shuffle_seed=seed, log=log)
    t1 = time.perf_counter()
    mlp = B.igafd_mlp_create(seed)
    hist = train(mlp, feat, targ, total, epochs=epochs, log=log)
    if log:
        log(f"dataset {t1 - t0:.1f} s ({total} dofs), training {time.perf_counter() - t1:.1f} s")
    return mlp, hist, total


def save(mlp, path):
    np.save(path, B.igafd_mlp_get_params(mlp), allow_pickle=False)


def load(path, seed=0):
    mlp = B.igafd_mlp_create(seed)
    B.igafd_mlp_set_params(mlp, np.load(path, allow_pickle=False))
    return mlp
