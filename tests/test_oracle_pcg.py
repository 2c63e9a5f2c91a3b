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
