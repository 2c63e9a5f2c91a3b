"""Pins of the oracle's univariate layer against library routines, closed forms
and the paper's Table cond (Sec. 2.1, Sec. 3, Sec. 4.1-4.2)."""
import json
import os

import numpy as np
import pytest
from scipy.interpolate import BSpline
from scipy.linalg import eigh

import synth
from oracle import fd, splines

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def scipy_basis(knots, p, x, nu=0):
    """All B-splines (and derivatives) via scipy, independent of the oracle."""
    m = len(knots) - p - 1
    out = np.zeros((len(x), m))
    for i in range(m):
        c = np.zeros(m)
        c[i] = 1.0
        s = BSpline(knots, c, p, extrapolate=False)
        if nu:
            s = s.derivative(nu)
        out[:, i] = np.nan_to_num(s(x))
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_basis_matches_scipy(p):
    kn = synth.jittered_knots(7, p, seed=p)
    x = np.linspace(0.0, 1.0, 301)[:-1] + 1e-4
    np.testing.assert_allclose(splines.basis(kn, p, x), scipy_basis(kn, p, x), atol=1e-13)
    np.testing.assert_allclose(splines.basis_derivative(kn, p, x), scipy_basis(kn, p, x, 1), atol=1e-11)


def test_basis_repeated_interior_knot():
    p = 3
    kn = np.array([0, 0, 0, 0, 0.25, 0.5, 0.5, 0.75, 1, 1, 1, 1], float)
    splines.check_knots(kn, p)
    x = np.linspace(0.01, 0.99, 97)
    np.testing.assert_allclose(splines.basis(kn, p, x), scipy_basis(kn, p, x), atol=1e-13)
    np.testing.assert_allclose(splines.basis_derivative(kn, p, x), scipy_basis(kn, p, x, 1), atol=1e-11)


def test_partition_of_unity_and_endpoint():
    for p in (1, 2, 4):
        kn = synth.jittered_knots(6, p, seed=3)
        x = np.linspace(0, 1, 57)
        B = splines.basis(kn, p, x)
        np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
        # the last span closed on the right: B_m(1) = 1 (C6 reading)
        assert B[-1, -1] == pytest.approx(1.0)


def test_p1_hat_functions():
    E = 5
    kn = synth.uniform_knots(E, 1)
    x = np.linspace(0, 1, 41)
    B = splines.basis(kn, 1, x)
    for i in range(E + 1):
        np.testing.assert_allclose(B[:, i], np.maximum(0.0, 1.0 - np.abs(x * E - i)), atol=1e-14)


def test_invalid_knots_rejected():
    with pytest.raises(ValueError):
        splines.check_knots([0, 0, 0.5, 1, 1], 2)
    with pytest.raises(ValueError):
        splines.check_knots([0, 0, 0, 0.5, 0.5, 0.5, 1, 1, 1], 2)
    with pytest.raises(ValueError):
        splines.check_knots([0, 0, 0.6, 0.5, 1, 1], 1)


@pytest.mark.parametrize("q", [1, 2, 3, 6])
def test_gauss_rule_exact_on_monomials(q):
    for k in range(2 * q):
        x, w = splines.gauss_rule(q, 0.2, 0.7)
        exact = (0.7 ** (k + 1) - 0.2 ** (k + 1)) / (k + 1)
        assert np.dot(w, x ** k) == pytest.approx(exact, rel=1e-13, abs=1e-15)
    x, w = splines.gauss_rule(q, 0.0, 1.0)
    k = 2 * q
    assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) > 1e-8  # not exact beyond 2q-1


def test_p1_mass_stiffness_closed_form():
    E = 9
    h = 1.0 / E
    M, K = splines.univariate_matrices(synth.uniform_knots(E, 1), 1)
    n = E - 1
    T = lambda a, b: np.diag(np.full(n, a)) + np.diag(np.full(n - 1, b), 1) + np.diag(np.full(n - 1, b), -1)
    np.testing.assert_allclose(M, h / 6 * T(4, 1), atol=1e-15)
    np.testing.assert_allclose(K, 1 / h * T(2, -1), atol=1e-12)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_full_space_identities(p):
    kn = synth.jittered_knots(8, p, seed=10 + p)
    M, K = splines.univariate_matrices(kn, p, interior=False)
    one = np.ones(M.shape[0])
    assert one @ M @ one == pytest.approx(1.0, rel=1e-13)
    np.testing.assert_allclose(M @ one, (kn[p + 1:] - kn[:-p - 1]) / (p + 1), atol=1e-14)
    np.testing.assert_allclose(K @ one, 0.0, atol=1e-10)
    greville = np.array([kn[i + 1:i + p + 1].mean() for i in range(M.shape[0])])
    assert greville @ K @ greville == pytest.approx(1.0, rel=1e-12)   # int (x')^2 = 1
    assert greville @ M @ greville == pytest.approx(1.0 / 3.0, rel=1e-12)  # int x^2


@pytest.mark.parametrize("p", [2, 3, 5])
def test_matrices_match_scipy_basis_and_are_exact(p):
    kn = synth.jittered_knots(6, p, seed=p)
    M, K = splines.univariate_matrices(kn, p)
    # independent evaluation: scipy basis at a much finer Gauss rule (exactness of q = p+1)
    xs, ws = [], []
    for (_, a, b) in splines.elements(kn):
        t, w = np.polynomial.legendre.leggauss(p + 6)
        xs.append(a + (b - a) * (t + 1) / 2)
        ws.append(w * (b - a) / 2)
    x, w = np.concatenate(xs), np.concatenate(ws)
    B = scipy_basis(kn, p, x)[:, 1:-1]
    dB = scipy_basis(kn, p, x, 1)[:, 1:-1]
    np.testing.assert_allclose(M, B.T @ (w[:, None] * B), atol=1e-15)
    np.testing.assert_allclose(K, dB.T @ (w[:, None] * dB), rtol=1e-11, atol=1e-10)
    assert np.count_nonzero(np.abs(np.triu(M, p + 1)) > 0) == 0  # bandwidth p
    assert np.all(np.linalg.eigvalsh(M) > 0) and np.all(np.linalg.eigvalsh(K) > 0)


def test_p1_generalized_eigenvalues_closed_form():
    E = 16
    h = 1.0 / E
    M, K = splines.univariate_matrices(synth.uniform_knots(E, 1), 1)
    U, lam = fd.generalized_eig(K, M)
    k = np.arange(1, E)
    c = np.cos(k * np.pi * h)
    np.testing.assert_allclose(np.sort(lam), np.sort(6 * (1 - c) / (h * h * (2 + c))), rtol=1e-12)
    # eigenvectors proportional to sin(k pi j h)
    j = np.arange(1, E)
    for col in range(E - 1):
        v = np.sin((col + 1) * np.pi * j * h)
        u = U[:, col]
        cosang = abs(u @ v) / np.linalg.norm(u) / np.linalg.norm(v)
        assert cosang == pytest.approx(1.0, abs=1e-10)


@pytest.mark.parametrize("p", [1, 3, 4])
def test_generalized_eig_properties(p):
    kn = synth.jittered_knots(11, p, seed=7)
    M, K = splines.univariate_matrices(kn, p)
    U, lam = fd.generalized_eig(K, M)
    np.testing.assert_allclose(U.T @ M @ U, np.eye(len(lam)), atol=1e-11)
    np.testing.assert_allclose(U.T @ K @ U, np.diag(lam), atol=1e-9 * lam.max())
    np.testing.assert_allclose(lam, eigh(K, M, eigvals_only=True), rtol=1e-10)


def test_table_cond_from_paper():
    g = json.load(open(os.path.join(GOLDEN, "table_cond.json")))
    for p, printed, check in zip(g["degrees"], g["printed"], g["assert"]):
        M, K = splines.univariate_matrices(synth.uniform_knots(g["elements"], p), p)
        _, lam = fd.generalized_eig(K, M)
        kappa = lam.max() / lam.min()
        one_digit = float(f"{kappa:.0e}")
        if check:
            assert one_digit == printed, (p, kappa, printed)
