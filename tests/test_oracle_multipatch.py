"""Pins of the multi-patch oracle (Sec. 6, Sec. 7 multi-patch experiment):
the C^0 gluing against an independent single-patch assembly, continuity and
boundary values of the glued functions, the closed form of the subdomain
matrices, spectral bounds of the Schwarz operators, and the iteration counts
of Table L."""
import json
import pathlib

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import assembly, fd, multipatch as mp, splines

GOLDEN = pathlib.Path(__file__).parent / "golden" / "table_L_iterations.json"


def lshape(E, p, jitter_seed=None):
    kn = synth.uniform_knots(E, p) if jitter_seed is None else synth.jittered_knots(E, p, jitter_seed)
    return mp.LShape(kn, p)


@pytest.mark.parametrize("E,p", [(4, 1), (5, 2), (6, 3), (3, 5)])
def test_dof_count_closed_form(E, p):
    # three patch interiors of (m-2)^2 functions plus two interface lines of m-2
    L = lshape(E, p)
    m = E + p
    assert L.m == m
    assert L.N == 3 * (m - 2) ** 2 + 2 * (m - 2)


@pytest.mark.parametrize("E,p,seed", [(4, 2, None), (5, 3, 7), (6, 1, None), (3, 4, 11)])
def test_glued_matrix_equals_single_patch_assembly(E, p, seed):
    """The conforming C^0 space on the L equals the functions of the square
    [0,1]^2 with a p-fold knot at 1/2 in both directions that vanish on the
    removed quarter; the element-loop assembly of that single patch,
    restricted to the L's functions, must reproduce the glued Kronecker
    sums (an independent construction)."""
    L = lshape(E, p, seed)
    A = L.matrix()
    km = mp.merged_knots(L.knots, p)
    As = assembly.assemble_matrix(synth.make_problem(2, p, [km, km]))
    pos, n = L.square_index()
    assert As.shape[0] == n * n
    assert len(np.unique(pos)) == L.N and pos.min() >= 0
    D = (As[pos][:, pos] - A).toarray()
    assert np.abs(D).max() <= 1e-13 * abs(A).max()
    # the square's functions left out are exactly those touching the removed quarter
    i1, i2 = pos % n, pos // n
    c = L.m - 2
    assert not np.any((i1 >= c) & (i2 >= c))
    assert L.N + (n - c) ** 2 == n * n


def test_matrix_rows_match_matrix():
    L = lshape(5, 3, 4)
    A = L.matrix().toarray()
    rows = np.array([0, 3, L.N // 3, L.N // 2, L.N - 1])
    assert np.abs(L.matrix_rows(rows).toarray() - A[rows]).max() <= 1e-15 * np.abs(A).max() * 10


def _patch_values(L, k, x, y, u):
    """Value at parameter points (x[i], y[i]) of patch k of the global function u."""
    Bx = splines.basis(L.knots, L.p, x)
    By = splines.basis(L.knots, L.p, y)
    g = L.gid[k]
    coef = np.where(g >= 0, u[np.maximum(g, 0)], 0.0)   # [b, a]
    return np.einsum("ib,ba,ia->i", By, coef, Bx)


@pytest.mark.parametrize("E,p", [(5, 2), (4, 3), (6, 1)])
def test_glued_functions_continuous_and_zero_on_boundary(E, p):
    L = lshape(E, p, 3)
    u = synth.random_vector(L.N, 21)
    t = np.linspace(0.0, 1.0, 37)
    z, o = np.zeros_like(t), np.ones_like(t)
    # G12: top edge of Omega_2 (y = 1) = bottom edge of Omega_1 (y = 0), same x
    a = _patch_values(L, 2, t, o, u)
    b = _patch_values(L, 1, t, z, u)
    assert np.abs(a - b).max() <= 1e-13 * (1 + np.abs(a).max())
    assert np.abs(a).max() > 1e-3
    # G23: right edge of Omega_2 = left edge of Omega_3, same y
    a = _patch_values(L, 2, o, t, u)
    b = _patch_values(L, 3, z, t, u)
    assert np.abs(a - b).max() <= 1e-13 * (1 + np.abs(a).max())
    assert np.abs(a).max() > 1e-3
    # boundary of Omega, edge by edge (parameter coordinates of each patch)
    for k, xs, ys in [(1, z, t), (1, o, t), (1, t, o), (2, z, t), (2, t, z), (3, t, z), (3, o, t), (3, t, o)]:
        assert np.abs(_patch_values(L, k, xs, ys, u)).max() <= 1e-14


def _stretched(F, i):
    # Theta_1 = [0,1/2] x [0,1] (J = diag(1/2, 1)), Theta_2 = [0,1] x [0,1/2];
    # Q = |det J| J^-1 J^-T = diag(2, 1/2) resp. diag(1/2, 2)
    Mx, Kx, My, Ky = F[0]["M"], F[0]["K"], F[1]["M"], F[1]["K"]
    q1, q2 = (2.0, 0.5) if i == 0 else (0.5, 2.0)
    return q1 * np.kron(My, Kx) + q2 * np.kron(Ky, Mx)


@pytest.mark.parametrize("E,p,seed", [(4, 2, None), (5, 3, 5), (6, 1, None)])
def test_subdomain_matrix_is_stretched_single_patch(E, p, seed):
    """Sec. 6: A_i = R_i A R_i^T is the stiffness matrix of Theta_i as one
    patch; for the 2:1 rectangle that is Q-weighted Kronecker sums."""
    L = lshape(E, p, seed)
    S = mp.Schwarz(L)
    A = S.A.toarray()
    for i, R in enumerate(S.R):
        Ai = A[np.ix_(R, R)]
        C = _stretched(S.factors[i], i)
        assert np.abs(Ai - C).max() <= 1e-13 * np.abs(C).max()
        # the local preconditioner is eq. prec of Theta_i's parameter domain
        P = fd.kron_P(S.factors[i])
        ev = sla.eigh(Ai, P, eigvals_only=True)
        assert ev.min() >= 0.5 - 1e-10 and ev.max() <= 2.0 + 1e-10


def _operator(apply, N):
    return np.column_stack([apply(e) for e in np.eye(N)])


@pytest.mark.parametrize("E,p", [(4, 2), (5, 1)])
def test_schwarz_spectra(E, p):
    """P_EAS^-1 A = P_1 + P_2 (A-orthogonal projections on the two local
    spaces): eigenvalues in (0, 2], and 2 is attained on the functions
    supported in Omega_2.  With eig(P_i^-1 A_i) in [1/2, 2], P_IAS^-1 A has
    its eigenvalues in [lmin_EAS / 2, 4]; P_IAS^-1 is symmetric."""
    L = lshape(E, p)
    S = mp.Schwarz(L)
    A = S.A.toarray()
    Te = _operator(S.eas, L.N)
    Ti = _operator(S.ias, L.N)
    assert np.abs(Ti - Ti.T).max() <= 1e-12 * np.abs(Ti).max()
    ee = np.sort(sla.eigh(A, np.linalg.inv(Te), eigvals_only=True))
    assert ee.min() > 0 and abs(ee.max() - 2.0) <= 1e-10
    # multiplicity of 2 = interior functions of Omega_2
    assert np.sum(ee > 2.0 - 1e-8) == (L.m - 2) ** 2
    ei = np.sort(sla.eigh(A, np.linalg.inv(Ti), eigvals_only=True))
    assert ei.min() >= ee.min() / 2 - 1e-10 and ei.max() <= 4.0 + 1e-10


def test_ias_apply_equals_explicit_kronecker_inverse():
    L = lshape(5, 2)
    S = mp.Schwarz(L)
    r = synth.random_vector(L.N, 8)
    z = np.zeros(L.N)
    for R, F in zip(S.R, S.factors):
        z[R] += np.linalg.solve(fd.kron_P(F), r[R])
    assert np.abs(S.ias(r) - z).max() <= 1e-12 * np.abs(z).max()


def test_load_of_constant_is_integral_of_basis():
    # f = 1: b_g = int B_g = (1/4) sum over the patches holding g of the
    # products of 1D integrals int B_a = (t_{a+p+1} - t_a) / (p+1)
    L = lshape(6, 3, 2)
    b = L.load({"kind": "one"})
    t, p = L.knots, L.p
    w = (t[p + 1:] - t[: -p - 1]) / (p + 1)
    ref = np.zeros(L.N)
    for k in (1, 2, 3):
        g = L.gid[k]
        keep = g >= 0
        np.add.at(ref, g[keep], 0.25 * np.outer(w, w)[keep])
    assert np.abs(b - ref).max() <= 1e-15 * np.abs(ref).max() * 10


def test_table_L_iterations():
    """CG + P_IAS iteration counts: independent of h and p (the paper's
    finding) and within the stated tolerance of Table L at h^-1 = 128."""
    g = json.loads(GOLDEN.read_text())
    tol = g["tolerance_ias"]
    counts = {}
    for E in (32, 128):
        for j, p in enumerate(g["degrees"]):
            L = lshape(E, p)
            S = mp.Schwarz(L)
            b = L.load(synth.RHS_PAPER_POLY)
            x, info = S.solve(b, "ias")
            assert info["true_relres"] <= 1e-8
            counts[E, p] = info["iters"]
            if E == 128:
                assert abs(info["iters"] - g["ias"][0][j]) <= tol, (p, info["iters"])
    it = np.array(list(counts.values()))
    assert it.max() - it.min() <= 2, counts
