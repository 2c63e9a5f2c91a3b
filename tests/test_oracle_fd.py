"""Pins of the oracle's preconditioner: the Kronecker identities (Sec. 2.2), the
explicit Kronecker sum P (Sec. 3 eq. prec) and the FD apply (Alg. 1, Alg. 3)."""
import numpy as np
import pytest

import synth
from oracle import fd


def test_kronprod_identity_vs_mode_products(rng):
    # (A (x) B) vec(X) = vec(B X A^T), vec stacking columns (Sec. 2.2 eq. kronprod)
    A = rng.standard_normal((3, 3))
    B = rng.standard_normal((4, 4))
    X = rng.standard_normal((4, 3))
    lhs = np.kron(A, B) @ X.reshape(-1, order="F")
    np.testing.assert_allclose(lhs, (B @ X @ A.T).reshape(-1, order="F"), atol=1e-13)
    # in the (n2, n1) C-order layout, direction 1 is the fast axis: kron(W2, W1)
    # acting on the flat vector equals mode-1 then mode-2 products
    W1 = rng.standard_normal((5, 5))
    W2 = rng.standard_normal((3, 3))
    T = rng.standard_normal((3, 5))
    out = fd.mode_product(fd.mode_product(T, W1, 0), W2, 1)
    np.testing.assert_allclose(out.reshape(-1), np.kron(W2, W1) @ T.reshape(-1), atol=1e-13)


def _problem(dim, p, seed):
    Es = [3, 4, 5][:dim]
    kn = [synth.jittered_knots(E, p, seed=seed + i) for i, E in enumerate(Es)]
    return synth.make_problem(dim, p, kn)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_fd_apply_equals_dense_solve(dim, p, rng):
    prob = _problem(dim, p, seed=10 * dim + p)
    F = fd.setup(prob)
    P = fd.kron_P(F)
    r = rng.standard_normal(P.shape[0])
    s = fd.fd_apply(F, r)
    ref = np.linalg.solve(P, r)
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-12
    np.testing.assert_allclose(P @ s, r, atol=1e-10 * np.abs(r).max() * np.abs(P).max())


def test_fd_shape_sensitivity(rng):
    # n1 != n2 != n3: a transposed direction ordering must not pass
    prob = _problem(3, 2, seed=5)
    F = fd.setup(prob)
    P = fd.kron_P(F)
    r = rng.standard_normal(P.shape[0])
    wrong = [F[2], F[1], F[0]]
    shape = tuple(len(f["lam"]) for f in F[::-1])
    s_ok = fd.fd_apply(F, r)
    assert np.linalg.norm(P @ s_ok - r) < 1e-9 * np.linalg.norm(r)
    assert shape[0] != shape[2]
    s_bad = fd.fd_apply(wrong, r)
    assert np.linalg.norm(P @ s_bad - r) > 1e-2 * np.linalg.norm(r)


def test_kron_P_ordering_matches_definition(rng):
    # P_ij = int grad B_i . grad B_j with B_i = B1(i1) B2(i2): the K factor sits
    # on the fast (direction 1) axis in the first term
    prob = _problem(2, 2, seed=1)
    F = fd.setup(prob)
    n1, n2 = len(F[0]["lam"]), len(F[1]["lam"])
    P = fd.kron_P(F)
    i1, i2, j1, j2 = 1, 2, 2, 1
    i = i1 + n1 * i2
    j = j1 + n1 * j2
    ref = F[0]["K"][i1, j1] * F[1]["M"][i2, j2] + F[0]["M"][i1, j1] * F[1]["K"][i2, j2]
    assert P[i, j] == pytest.approx(ref, rel=1e-14)
    np.testing.assert_allclose(fd.diag_P(F), np.diag(P), rtol=1e-14)


def test_fd_scaling_is_symmetric_positive(rng):
    prob = _problem(2, 2, seed=3)
    F = fd.setup(prob)
    P = fd.kron_P(F)
    S = rng.uniform(0.5, 2.0, P.shape[0])
    r = rng.standard_normal(P.shape[0])
    ref = S * np.linalg.solve(P, S * r)
    np.testing.assert_allclose(fd.fd_apply(F, r, scaling=S), ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 1), (3, 3)])
def test_apply_P_matches_kron_and_assembly(dim, p, rng):
    # banded Kronecker-sum product == the explicit Kronecker matrix, and on the
    # unit square / cube with kappa = 1 (P = A, Sec. 3) == the assembled A
    prob = _problem(dim, p, seed=40 + dim + p)
    F = fd.setup(prob)
    x = rng.standard_normal(int(np.prod([len(f["lam"]) for f in F])))
    y = fd.apply_P(F, x)
    np.testing.assert_allclose(y, fd.kron_P(F) @ x, rtol=0, atol=1e-12 * np.abs(y).max())
    from oracle import assembly
    A = assembly.assemble_matrix(prob)
    np.testing.assert_allclose(y, A @ x, rtol=0, atol=1e-11 * np.abs(y).max())
    # FD is its inverse
    r = rng.standard_normal(x.size)
    np.testing.assert_allclose(fd.apply_P(F, fd.fd_apply(F, r)), r, rtol=0, atol=1e-9 * np.abs(r).max())
