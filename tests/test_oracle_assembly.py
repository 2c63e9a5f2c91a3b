"""Pins of the oracle's discretisation: geometry maps, Q (Sec. 2.1 eq. Q), the
stiffness matrix A (eq. A), the load vector, and Galerkin exactness."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

import synth
from oracle import assembly, fd, geometry, pcg, splines


def scipy_basis(knots, p, x, nu=0):
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


def weighted_1d(knots, p, weight):
    """int w B_i B_j and int w B_i' B_j' on the interior functions, by scipy
    basis evaluation and numpy's Gauss nodes with q = p+1 points per element
    (the rule the discretisation uses), independent of the oracle's code."""
    xs, ws = [], []
    kn = np.asarray(knots)
    for i in range(len(kn) - 1):
        if kn[i] < kn[i + 1]:
            t, w = np.polynomial.legendre.leggauss(p + 1)
            xs.append(kn[i] + (kn[i + 1] - kn[i]) * (t + 1) / 2)
            ws.append(w * (kn[i + 1] - kn[i]) / 2)
    x, w = np.concatenate(xs), np.concatenate(ws)
    w = w * weight(x)
    B = scipy_basis(kn, p, x)[:, 1:-1]
    dB = scipy_basis(kn, p, x, 1)[:, 1:-1]
    return B.T @ (w[:, None] * B), dB.T @ (w[:, None] * dB)


def test_warped_jacobian_and_fixed_boundary(rng):
    g = synth.warped_geometry(seed=3)
    xi = rng.random((50, 3))
    x, J = geometry.map_and_jacobian(g, xi)
    eps = 1e-6
    for j in range(3):
        d = np.zeros(3)
        d[j] = eps
        xp, _ = geometry.map_and_jacobian(g, xi + d)
        xm, _ = geometry.map_and_jacobian(g, xi - d)
        np.testing.assert_allclose((xp - xm) / (2 * eps), J[:, :, j], atol=1e-8)
    face = rng.random((20, 3))
    face[:, 1] = 1.0
    xf, _ = geometry.map_and_jacobian(g, face)
    np.testing.assert_allclose(xf, face, atol=1e-15)
    assert np.max(np.linalg.norm(x - xi, axis=1)) <= 0.1 + 1e-12


def test_ring_jacobian_and_Q_closed_form(rng):
    xi = rng.random((40, 3))
    g = {"kind": "ring"}
    x, J = geometry.map_and_jacobian(g, xi)
    eps = 1e-6
    for j in range(3):
        d = np.zeros(3)
        d[j] = eps
        np.testing.assert_allclose((geometry.map_and_jacobian(g, xi + d)[0] -
                                    geometry.map_and_jacobian(g, xi - d)[0]) / (2 * eps), J[:, :, j], atol=1e-8)
    prob = synth.thick_ring(E=2, p=1)
    Q, det, _ = geometry.q_matrix(prob, xi)
    w = np.pi * (1 + xi[:, 0]) / 2
    np.testing.assert_allclose(det, w, rtol=1e-14)
    ref = np.zeros((40, 3, 3))
    ref[:, 0, 0], ref[:, 1, 1], ref[:, 2, 2] = w, 1 / w, w
    np.testing.assert_allclose(Q, ref, atol=1e-14)


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 3), (3, 2)])
def test_identity_map_A_equals_P(dim, p):
    Es = [3, 4, 5][:dim]
    prob = synth.make_problem(dim, p, [synth.jittered_knots(E, p, seed=E) for E in Es])
    A = assembly.assemble_matrix(prob).toarray()
    P = fd.kron_P(fd.setup(prob))
    np.testing.assert_allclose(A, P, atol=1e-13 * np.abs(P).max())
    nnz_row = np.count_nonzero(np.abs(A) > 0, axis=1)
    assert nnz_row.max() <= (2 * p + 1) ** dim
    assert nnz_row.min() >= (p + 1) ** dim or min(Es) + p - 2 < p + 1


def test_thick_ring_separable_closed_form():
    p = 2
    kn = [synth.jittered_knots(3, p, 1), synth.jittered_knots(4, p, 2), synth.jittered_knots(2, p, 3)]
    prob = synth.make_problem(3, p, kn, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob).toarray()
    w = lambda s: np.pi * (1 + s) / 2
    M1w, K1w = weighted_1d(kn[0], p, w)
    M1i, _ = weighted_1d(kn[0], p, lambda s: 1 / w(s))
    M2, K2 = weighted_1d(kn[1], p, np.ones_like)
    M3, K3 = weighted_1d(kn[2], p, np.ones_like)
    ref = np.kron(M3, np.kron(M2, K1w)) + np.kron(M3, np.kron(K2, M1i)) + np.kron(K3, np.kron(M2, M1w))
    np.testing.assert_allclose(A, ref, atol=1e-13 * np.abs(ref).max())


def test_quarter_annulus_separable_closed_form():
    p = 3
    kn = [synth.jittered_knots(5, p, 4), synth.jittered_knots(4, p, 5)]
    prob = synth.make_problem(2, p, kn, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob).toarray()
    w = lambda s: np.pi * (1 + s) / 2
    _, K1w = weighted_1d(kn[0], p, w)
    M1i, _ = weighted_1d(kn[0], p, lambda s: 1 / w(s))
    M2, K2 = weighted_1d(kn[1], p, np.ones_like)
    ref = np.kron(M2, K1w) + np.kron(K2, M1i)
    np.testing.assert_allclose(A, ref, atol=1e-13 * np.abs(ref).max())


def test_coefficient_scales_A():
    # kappa = 1 + amp sin(2 pi x) cos(2 pi y) with amp = 0 leaves A unchanged; a
    # constant-coefficient identity-map A is P
    prob = synth.uniform_problem(2, 4, 2, coefficient=synth.sincos_coefficient(0.0))
    A = assembly.assemble_matrix(prob).toarray()
    np.testing.assert_allclose(A, fd.kron_P(fd.setup(prob)), atol=1e-14)
    prob2 = synth.uniform_problem(2, 4, 2, coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.3, 0.2))
    A2 = assembly.assemble_matrix(prob2).toarray()
    assert np.abs(A2 - A).max() > 1e-3
    np.testing.assert_allclose(A2, A2.T, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(A2) > 0)


def test_separable_coefficient_closed_form():
    # identity map, kappa = 1 + a sin(2 pi f1 x + phi1) cos(2 pi f2 y + phi2) is
    # separable, so A = P + a (K1[s] (x) M2[c] + M1[s] (x) K2[c]) in 2D
    p = 2
    coef = synth.sincos_coefficient(0.4, 1, 2, 0.3, 0.7)
    kn = [synth.jittered_knots(5, p, 11), synth.jittered_knots(4, p, 12)]
    prob = synth.make_problem(2, p, kn, coefficient=coef)
    A = assembly.assemble_matrix(prob).toarray()
    sx = lambda x: np.sin(2 * np.pi * 1 * x + 0.3)
    cy = lambda y: np.cos(2 * np.pi * 2 * y + 0.7)
    M1, K1 = weighted_1d(kn[0], p, np.ones_like)
    M2, K2 = weighted_1d(kn[1], p, np.ones_like)
    M1s, K1s = weighted_1d(kn[0], p, sx)
    M2c, K2c = weighted_1d(kn[1], p, cy)
    ref = np.kron(M2, K1) + np.kron(K2, M1) + 0.4 * (np.kron(M2c, K1s) + np.kron(K2c, M1s))
    np.testing.assert_allclose(A, ref, atol=1e-13 * np.abs(ref).max())


def test_load_vector_of_one_is_basis_integral():
    p = 3
    kn = [synth.jittered_knots(4, p, 8), synth.jittered_knots(3, p, 9)]
    prob = synth.make_problem(2, p, kn)
    b = assembly.assemble_load(prob, {"kind": "one"})
    ints = [((k[p + 1:] - k[:-p - 1]) / (p + 1))[1:-1] for k in kn]   # int B_i = (xi_{i+p+1}-xi_i)/(p+1)
    np.testing.assert_allclose(b, np.kron(ints[1], ints[0]), rtol=1e-13)


def test_sampled_rows_match_full_assembly():
    prob = synth.warped_cube(E=4, p=2, seed=3)
    A = assembly.assemble_matrix(prob)
    rows = [0, 7, 31, 62, 63]
    As = assembly.assemble_matrix(prob, rows=rows)
    np.testing.assert_allclose(As[rows].toarray(), A[rows].toarray(), atol=1e-15, rtol=1e-13)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    bs = assembly.assemble_load(prob, synth.RHS_SINPROD, dofs_subset=rows)
    np.testing.assert_allclose(bs[rows], b[rows], rtol=1e-13)


def _evaluate(prob, u, pts):
    p = prob["degree"]
    vals = [scipy_basis(k, p, pts[:, l])[:, 1:-1] for l, k in enumerate(prob["knots"])]
    U = u.reshape([v.shape[1] for v in vals[::-1]])
    if prob["dim"] == 2:
        return np.einsum("ji,pi,pj->p", U, vals[0], vals[1])
    return np.einsum("kji,pi,pj,pk->p", U, vals[0], vals[1], vals[2])


@pytest.mark.parametrize("dim,p,E", [(2, 2, 5), (2, 3, 4), (3, 2, 3)])
def test_galerkin_exactness_bubble(dim, p, E, rng):
    # u = prod x(1-x) lies in V_h for p >= 2 on the unit square/cube, so the
    # Galerkin solution reproduces it exactly
    prob = synth.uniform_problem(dim, E, p)
    A = assembly.assemble_matrix(prob)
    b = assembly.assemble_load(prob, synth.RHS_BUBBLE)
    u = np.linalg.solve(A.toarray(), b)
    pts = rng.random((30, dim))
    exact = np.prod(pts * (1 - pts), axis=1)
    np.testing.assert_allclose(_evaluate(prob, u, pts), exact, atol=1e-12)


def test_galerkin_exactness_paper_rhs_2d(rng):
    # the paper's 2D right-hand side f = 2(x^2-x) + 2(y^2-y) (Sec. 7.1) has the
    # solution u = -x(1-x)y(1-y)
    prob = synth.uniform_problem(2, 6, 2)
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_PAPER_POLY)
    u, info = pcg.solve(prob, A, F, b, rtol=1e-13)
    assert info["iters"] == 1
    pts = rng.random((25, 2))
    np.testing.assert_allclose(_evaluate(prob, u, pts), -np.prod(pts * (1 - pts), axis=1), atol=1e-12)


def test_nonpositive_jacobian_rejected():
    g = {"kind": "warped", "amp": 2.0, "c": np.array([[1.0, 1.0, 1.0]]), "m": np.array([[1, 1, 1]])}
    prob = synth.uniform_problem(3, 2, 1, geometry=g)
    with pytest.raises(ValueError):
        assembly.assemble_matrix(prob)


def test_sinprod_rhs_converges_to_its_solution(rng):
    # f = d pi^2 prod sin(pi x_i) has u = prod sin(pi x_i); the p = 3 discrete
    # solution on 8 elements is within the interpolation error of u
    pts = rng.random((40, 2))
    errs = []
    for E in (8, 16):
        prob = synth.uniform_problem(2, E, 3)
        A = assembly.assemble_matrix(prob)
        b = assembly.assemble_load(prob, synth.RHS_SINPROD)
        u = np.linalg.solve(A.toarray(), b)
        errs.append(np.abs(_evaluate(prob, u, pts) - np.prod(np.sin(np.pi * pts), axis=1)).max())
    assert errs[0] < 1e-4
    assert errs[0] / errs[1] > 10  # order p+1 = 4 convergence


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 2), (3, 3)])
def test_ring_operator_equals_element_assembly(dim, p, rng):
    """The matrix-free Kronecker form of the ring's A (used at the full
    workload size) against the element loop, with a different knot vector
    in every direction; the absolute form bounds |A| entrywise."""
    Es = [4, 3, 5][:dim]
    kn = [synth.jittered_knots(E, p, 20 + E) for E in Es]
    prob = synth.make_problem(dim, p, kn, geometry={"kind": "ring"})
    A = assembly.assemble_matrix(prob)
    op = assembly.ring_operator(prob)
    aop = assembly.ring_operator(prob, absolute=True)
    x = rng.standard_normal(A.shape[0])
    np.testing.assert_allclose(op(x), A @ x, atol=1e-14 * (abs(A) @ np.abs(x)).max())
    # entrywise: column j of each operator
    eye = np.eye(A.shape[0])
    Ad = A.toarray()
    cols = np.stack([op(eye[j]) for j in range(A.shape[0])], axis=1)
    np.testing.assert_allclose(cols, Ad, atol=1e-14 * np.abs(Ad).max())
    acols = np.stack([aop(eye[j]) for j in range(A.shape[0])], axis=1)
    assert np.all(acols >= np.abs(Ad) - 1e-14 * np.abs(Ad).max())
    with pytest.raises(ValueError):
        assembly.ring_operator(synth.uniform_problem(dim, Es, p))


@pytest.mark.parametrize("dim,geom", [(2, {"kind": "ring"}), (3, {"kind": "ring"}), (3, "warped"), (3, None)])
def test_tensor_load_vector_equals_element_loop(dim, geom):
    """The sum-factorised load vector (used at the full workload size)
    against the element loop, in one process and over a pool of processes."""
    p = 3
    g = synth.warped_geometry(3, dim=dim) if geom == "warped" else geom
    kn = [synth.jittered_knots(E, p, 30 + E) for E in [5, 4, 6][:dim]]
    prob = synth.make_problem(dim, p, kn, geometry=g)
    for f in (synth.RHS_SINPROD, synth.RHS_PAPER_POLY, {"kind": "sinprod", "amp": 2.5, "k": [2, 1, 3][:dim]}):
        ref = assembly.assemble_load(prob, f)
        b = assembly.assemble_load_tensor(prob, f, slab=2)
        np.testing.assert_allclose(b, ref, atol=1e-15 * np.abs(ref).max() * 10)
    b2 = assembly.assemble_load_tensor(prob, synth.RHS_SINPROD, slab=3, workers=2, pool_above=0)
    np.testing.assert_allclose(b2, assembly.assemble_load(prob, synth.RHS_SINPROD),
                               atol=1e-14 * np.abs(b2).max())


def test_sinprod_parameters_closed_form():
    """f = a sin(k1 pi x) sin(k2 pi y) on the unit square is separable, so its
    load vector is a times the Kronecker product of two 1D integrals
    int sin(k pi s) B_i(s) ds (scipy basis, 12-point Gauss rule per element)."""
    p = 2
    kn = [synth.jittered_knots(6, p, 41), synth.jittered_knots(5, p, 42)]
    prob = synth.make_problem(2, p, kn, quad=10)
    f = {"kind": "sinprod", "amp": 1.7, "k": [3, 2]}
    b = assembly.assemble_load(prob, f)

    def one_d(knots, k):
        xs, ws = [], []
        kk = np.asarray(knots)
        for i in range(len(kk) - 1):
            if kk[i] < kk[i + 1]:
                t, w = np.polynomial.legendre.leggauss(12)
                xs.append(kk[i] + (kk[i + 1] - kk[i]) * (t + 1) / 2)
                ws.append(w * (kk[i + 1] - kk[i]) / 2)
        x, w = np.concatenate(xs), np.concatenate(ws)
        return scipy_basis(kk, p, x)[:, 1:-1].T @ (w * np.sin(k * np.pi * x))

    ref = 1.7 * np.kron(one_d(kn[1], 2), one_d(kn[0], 3))
    # 10 and 12 Gauss points per element: both rules are accurate to roundoff
    np.testing.assert_allclose(b, ref, atol=1e-13 * np.abs(ref).max())
    # the frequencies matter: k = (2, 3) is a different vector
    other = assembly.assemble_load(prob, {"kind": "sinprod", "amp": 1.7, "k": [2, 3]})
    assert np.abs(other - ref).max() > 1e-2 * np.abs(ref).max()
    b_def = assembly.assemble_load(prob, {"kind": "sinprod", "amp": 2 * np.pi ** 2, "k": [1, 1]})
    np.testing.assert_allclose(b_def, assembly.assemble_load(prob, synth.RHS_SINPROD), rtol=1e-15, atol=0)
