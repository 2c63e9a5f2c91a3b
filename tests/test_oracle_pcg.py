"""Pins of the oracle's PCG: P = A converges in one iteration (Sec. 3, Sec. 7.1),
the Prop. 1 spectral inclusion, agreement with a direct sparse solve, and the
flexible variant with an exact preconditioner."""
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse.linalg as spla

import synth
from oracle import assembly, fd, geometry, pcg


@pytest.mark.parametrize("dim,E,p", [(2, 8, 3), (3, 4, 2)])
def test_identity_one_iteration(dim, E, p):
    prob = synth.uniform_problem(dim, E, p)
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u, info = pcg.solve(prob, A, F, b)
    assert info["iters"] == 1
    assert info["true_relres"] < 1e-12


def test_prop1_spectral_inclusion_ring():
    # thick ring: Q = diag(w, 1/w, w), w in [pi/2, pi] -> lambda(P^-1 A) in [1/pi, pi]
    prob = synth.make_problem(3, 2, [synth.jittered_knots(3, 2, s) for s in (1, 2, 3)], geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob).toarray()
    P = fd.kron_P(fd.setup(prob))
    lam = scipy.linalg.eigh(A, P, eigvals_only=True)
    assert lam.min() >= 1 / np.pi - 1e-12 and lam.max() <= np.pi + 1e-12


def test_prop1_spectral_inclusion_warped_kappa():
    prob = synth.uniform_problem(3, 3, 2, geometry=synth.warped_geometry(3),
                                 coefficient=synth.sincos_coefficient(0.5, 1, 2, 0.1, 0.2))
    A = assembly.assemble_matrix(prob).toarray()
    P = fd.kron_P(fd.setup(prob))
    lam = scipy.linalg.eigh(A, P, eigvals_only=True)
    xi, _ = assembly.quadrature_points(prob)
    Q, _, _ = geometry.q_matrix(prob, xi)
    ev = np.linalg.eigvalsh(Q)
    assert lam.min() >= ev[:, 0].min() * (1 - 1e-12)
    assert lam.max() <= ev[:, -1].max() * (1 + 1e-12)


@pytest.mark.parametrize("flexible", [False, True])
def test_pcg_matches_direct_solve(flexible):
    prob = synth.uniform_problem(3, 5, 3, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u, info = pcg.solve(prob, A, F, b, rtol=1e-10, flexible=flexible)
    ref = spla.spsolve(A.tocsc(), b)
    assert info["true_relres"] <= 1e-10
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-8
    assert 5 <= info["iters"] <= 40


def test_flexible_equals_standard_with_exact_preconditioner():
    prob = synth.uniform_problem(2, 12, 2, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u1, i1 = pcg.solve(prob, A, F, b, flexible=False)
    u2, i2 = pcg.solve(prob, A, F, b, flexible=True)
    assert i1["iters"] == i2["iters"]
    np.testing.assert_allclose(i1["history"], i2["history"], rtol=1e-6)
    assert np.linalg.norm(u1 - u2) / np.linalg.norm(u1) < 1e-9


def test_lanczos_ritz_values_inside_prop1_interval():
    # the CG coefficients give the Lanczos tridiagonal of P^-1 A; its Ritz
    # values must lie in [1/pi, pi] on the thick ring (Prop. 1)
    prob = synth.uniform_problem(3, 6, 2, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    alphas, betas = [], []
    x = np.zeros_like(b)
    r = b.copy()
    z = fd.fd_apply(F, r)
    rho = r @ z
    p = z.copy()
    for _ in range(15):
        q = A @ p
        a = rho / (p @ q)
        r = r - a * q
        z = fd.fd_apply(F, r)
        rn = r @ z
        bta = rn / rho
        alphas.append(a)
        betas.append(bta)
        rho = rn
        p = z + bta * p
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j else 0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    ritz = np.linalg.eigvalsh(T)
    assert ritz.min() >= 1 / np.pi - 1e-8 and ritz.max() <= np.pi + 1e-8


def test_pcg_zero_rhs_and_maxit():
    prob = synth.uniform_problem(2, 6, 2, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    u, info = pcg.solve(prob, A, F, np.zeros(A.shape[0]))
    assert info["iters"] == 0 and np.all(u == 0)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u, info = pcg.solve(prob, A, F, b, maxit=2)
    assert info["iters"] == 2 and not info["converged"]


def test_mlp_gradient_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(7)
    theta = rng.standard_normal(mlp.NPARAM) * 0.3
    feat = rng.standard_normal((40, mlp.NIN))
    target = rng.standard_normal(40) * 0.2
    mean, inv_std = np.zeros(8), np.ones(8)
    L, g = mlp.loss_and_grad(theta, mean, inv_std, feat, target)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 512, 4700]])  # b3, W1, b1, w3 entries
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        Lp, _ = mlp.loss_and_grad(theta + e, mean, inv_std, feat, target)
        Lm, _ = mlp.loss_and_grad(theta - e, mean, inv_std, feat, target)
        assert abs((Lp - Lm) / (2 * h) - g[k]) <= 1e-7 + 1e-5 * abs(g[k])


def test_features_identity_and_ring():
    from scipy.interpolate import BSpline
    from oracle import mlp
    prob = synth.uniform_problem(3, [3, 4, 2], 2)
    f = mlp.features(prob)
    np.testing.assert_allclose(f, np.tile([1, 1, 1, 0, 0, 0, 1, 2], (f.shape[0], 1)), atol=1e-14)
    # thick ring: G = diag(w, 1/w, w) with w = pi (1 + xi1) / 2 depends on xi1 only,
    # so each average is a 1D B-spline-weighted average in direction 1
    p = 2
    kn = [synth.jittered_knots(4, p, 1), synth.uniform_knots(3, p), synth.uniform_knots(2, p)]
    prob = synth.make_problem(3, p, kn, geometry={"kind": "ring"})
    f = mlp.features(prob)
    k1 = kn[0]
    xs, ws = [], []
    for i in range(len(k1) - 1):
        if k1[i] < k1[i + 1]:
            t, w = np.polynomial.legendre.leggauss(p + 1)
            xs.append(k1[i] + (k1[i + 1] - k1[i]) * (t + 1) / 2)
            ws.append(w * (k1[i + 1] - k1[i]) / 2)
    x, w = np.concatenate(xs), np.concatenate(ws)
    m = len(k1) - p - 1
    B = np.stack([np.nan_to_num(BSpline(k1, np.eye(m)[i], p, extrapolate=False)(x)) for i in range(m)], 1)[:, 1:-1]
    wr = np.pi * (1 + x) / 2
    avg_w = (B * (w * wr)[:, None]).sum(0) / (B * w[:, None]).sum(0)
    avg_iw = (B * (w / wr)[:, None]).sum(0) / (B * w[:, None]).sum(0)
    n = [len(k) - p - 3 for k in kn]
    F = f.reshape(n[2], n[1], n[0], 8)
    np.testing.assert_allclose(F[..., 0], np.broadcast_to(avg_w, F[..., 0].shape), rtol=1e-13)
    np.testing.assert_allclose(F[..., 1], np.broadcast_to(avg_iw, F[..., 1].shape), rtol=1e-13)
    np.testing.assert_allclose(F[..., 3:6], 0.0, atol=1e-14)


def test_scaling_targets_identity_zero_and_exact_ratio_helps():
    from oracle import mlp
    prob = synth.uniform_problem(2, 6, 2)
    np.testing.assert_allclose(mlp.targets(prob), 0.0, atol=1e-13)
    # on a warped domain with kappa the exact diagonal ratio S P^-1 S does not
    # need more iterations than P
    prob = synth.uniform_problem(3, 6, 2, geometry=synth.warped_geometry(3),
                                 coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.0, 0.0))
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    S = np.exp(mlp.targets(prob, A))
    _, i0 = pcg.solve(prob, A, F, b)
    _, i1 = pcg.solve(prob, A, F, b, scaling=S)
    assert i1["iters"] <= i0["iters"]


def test_q_spectral_bounds_ring_closed_form():
    # thick ring: Q = diag(w, 1/w, w), w = pi (1 + xi1) / 2, so the extremes
    # over the Gauss points follow from the direction-1 Gauss abscissae alone
    E, p = 5, 2
    prob = synth.uniform_problem(3, [E, 3, 4], p, geometry={"kind": "ring"})
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    xi1 = ((np.arange(E)[:, None] + 0.5 * (g[None, :] + 1.0)) / E).ravel()
    w = np.pi * (1.0 + xi1) / 2.0
    lo, hi = assembly.q_spectral_bounds(prob)
    assert abs(lo - np.minimum(w, 1 / w).min()) < 1e-13
    assert abs(hi - np.maximum(w, 1 / w).max()) < 1e-13
    # identity map, kappa = 1: Q = I
    lo, hi = assembly.q_spectral_bounds(synth.uniform_problem(3, 3, 2))
    assert abs(lo - 1) < 1e-14 and abs(hi - 1) < 1e-14


def test_q_spectral_bounds_contain_generalised_eigenvalues():
    # Prop. 1 for the discrete matrices: the eigenvalues of the pencil (A, P)
    # lie in [qmin, qmax] (warped map with a coefficient, so Q is full)
    import scipy.linalg
    prob = synth.uniform_problem(3, [3, 4, 3], 2, geometry=synth.warped_geometry(9),
                                 coefficient=synth.sincos_coefficient(0.4, 1, 2, 0.2, 0.7))
    A = assembly.assemble_matrix(prob).toarray()
    P = fd.kron_P(fd.setup(prob))
    ev = scipy.linalg.eigh(A, P, eigvals_only=True)
    lo, hi = assembly.q_spectral_bounds(prob)
    assert lo > 0 and ev.min() >= lo * (1 - 1e-12) and ev.max() <= hi * (1 + 1e-12)
    # and the bound is not loose by orders of magnitude
    assert ev.max() / ev.min() > 0.2 * hi / lo


def test_q_local_ratio_closed_forms():
    """qloc = max over the Gauss points of lambda_max(Q) / lambda_min(Q)."""
    # ring: Q = diag(w, 1/w, w), pointwise ratio w^2, largest at the largest
    # direction-1 abscissa, where it equals qmax / qmin
    E, p = 5, 2
    prob = synth.uniform_problem(3, [E, 3, 4], p, geometry={"kind": "ring"})
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    w = np.pi * (1.0 + ((np.arange(E)[:, None] + 0.5 * (g[None, :] + 1.0)) / E).ravel()) / 2.0
    lo, hi, loc = assembly.q_spectral_bounds(prob, local=True)
    assert abs(loc - (w.max() ** 2)) < 1e-12 and abs(loc - hi / lo) < 1e-12
    # identity map with a coefficient: Q = kappa I, isotropic at every point
    prob = synth.uniform_problem(3, 4, 2, coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.0, 0.0))
    lo, hi, loc = assembly.q_spectral_bounds(prob, local=True)
    assert abs(loc - 1.0) < 1e-12 and hi / lo > 2.0
    # 2D warped map: the ratio of a 2x2 SPD matrix from its trace and determinant
    prob = synth.uniform_problem(2, [6, 5], 3, geometry=synth.warped_geometry(4, dim=2),
                                 coefficient=synth.sincos_coefficient(0.3, 2, 1, 0.5, 0.1))
    xi, _ = assembly.quadrature_points(prob)
    from oracle import geometry
    Q, _, _ = geometry.q_matrix(prob, xi)
    t = Q[:, 0, 0] + Q[:, 1, 1]
    det = Q[:, 0, 0] * Q[:, 1, 1] - Q[:, 0, 1] ** 2
    disc = np.sqrt(t * t - 4 * det)
    ratio = (t + disc) / (t - disc)
    lo, hi, loc = assembly.q_spectral_bounds(prob, local=True)
    assert abs(loc - ratio.max()) < 1e-10 * ratio.max()
    assert 1.0 < loc <= hi / lo


def test_scaling_gate_rule_on_the_oracle():
    """The rule behind the library's scaling gate, checked on the oracle: where
    Q is anisotropic but of constant size (ring: (qmax/qmin) / qloc = 1) the
    diagonal scaling S P^-1 S costs iterations; where its size varies
    (constant map, kappa varying 3x: ratio 3) it saves many."""
    from oracle import mlp as omlp
    for prob, gate in ((synth.thick_ring(E=12, p=3), False),
                       (synth.uniform_problem(3, 12, 3, coefficient=synth.sincos_coefficient(0.5, 1, 1, 0, 0)), True)):
        lo, hi, loc = assembly.q_spectral_bounds(prob, local=True)
        assert ((hi / lo) / loc >= 2.0) == gate
        A = assembly.assemble_matrix(prob)
        F = fd.setup(prob)
        b = assembly.assemble_load(prob, synth.RHS_SINPROD)
        S = np.exp(omlp.targets(prob, A))
        _, i0 = pcg.solve(prob, A, F, b)
        _, i1 = pcg.solve(prob, A, F, b, scaling=S)
        if gate:
            assert i1["iters"] <= 0.7 * i0["iters"]
        else:
            assert i1["iters"] >= i0["iters"]
