"""Univariate B-splines, Gauss quadrature and the 1D mass/stiffness matrices.

Paper Sec. 2.1 (eq. knot-vector, eq. cox-deboor-1/2, eq. Vh) and Sec. 3 (the
univariate matrices M_d, K_d entering eq. prec).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def check_knots(knots, p):
    """Open knot vector of Sec. 2.1: first/last p+1 knots equal (0 and 1),
    nondecreasing, interior multiplicity at most p."""
    k = np.asarray(knots, dtype=np.float64)
    if p < 1 or k.ndim != 1 or len(k) < 2 * p + 2:
        raise ValueError("knot vector too short for degree p")
    if np.any(np.diff(k) < 0):
        raise ValueError("knots must be nondecreasing")
    if not (np.all(k[: p + 1] == 0.0) and np.all(k[-p - 1:] == 1.0)):
        raise ValueError("knot vector must be open on [0, 1]")
    if k[p + 1] == 0.0 or k[-p - 2] == 1.0:
        raise ValueError("end knots repeated more than p+1 times")
    vals, counts = np.unique(k[p + 1: -p - 1], return_counts=True)
    if np.any(counts > p):
        raise ValueError("interior knot multiplicity exceeds p")
    return k


def n_basis(knots, p):
    """m = number of B-splines of degree p on the knot vector (length m+p+1)."""
    return len(knots) - p - 1


def basis(knots, p, x):
    """Values of all B-splines B_{i,p}, i = 1..m, at the points x: shape (len(x), m).

    Cox-de Boor: degree-0 indicators of the half-open spans [xi_i, xi_{i+1})
    (eq. cox-deboor-1) raised by the two-term recursion eq. cox-deboor-2 with
    the convention 0/0 = 0.  The half-open spans make every function vanish at
    x = 1; as the usual convention, the last nonempty span is taken closed at
    its right end so that point values at x = 1 are those of the limit.
    """
    return _basis_deg(np.asarray(knots, float), p, np.atleast_1d(np.asarray(x, float)))


def _basis_deg(k, p, x):
    nspan = len(k) - 1
    B = np.zeros((len(x), nspan))
    last = max(i for i in range(nspan) if k[i] < k[i + 1])
    for i in range(nspan):
        if k[i] < k[i + 1]:
            inside = (k[i] <= x) & (x < k[i + 1])
            if i == last:
                inside |= x == k[i + 1]
            B[:, i] = inside
    for deg in range(1, p + 1):
        Bn = np.zeros((len(x), nspan - deg))
        for i in range(nspan - deg):
            d1 = k[i + deg] - k[i]
            d2 = k[i + deg + 1] - k[i + 1]
            term = np.zeros(len(x))
            if d1 > 0:
                term += (x - k[i]) / d1 * B[:, i]
            if d2 > 0:
                term += (k[i + deg + 1] - x) / d2 * B[:, i + 1]
            Bn[:, i] = term
        B = Bn
    return B


def basis_derivative(knots, p, x):
    """First derivatives of all B_{i,p} at x: shape (len(x), m).

    The paper does not write the derivative out; this is the textbook formula
    B'_{i,p} = p/(xi_{i+p}-xi_i) B_{i,p-1} - p/(xi_{i+p+1}-xi_{i+1}) B_{i+1,p-1}
    (0/0 = 0), which differentiates eq. cox-deboor-2.
    """
    k = np.asarray(knots, float)
    x = np.atleast_1d(np.asarray(x, float))
    Bl = _basis_deg(k, p - 1, x)  # m+1 functions of degree p-1
    m = len(k) - p - 1
    dB = np.zeros((len(x), m))
    for i in range(m):
        d1 = k[i + p] - k[i]
        d2 = k[i + p + 1] - k[i + 1]
        if d1 > 0:
            dB[:, i] += p / d1 * Bl[:, i]
        if d2 > 0:
            dB[:, i] -= p / d2 * Bl[:, i + 1]
    return dB


def elements(knots):
    """Nonempty knot spans [xi_k, xi_{k+1}] (the mesh elements): list of (k, a, b)."""
    k = np.asarray(knots, float)
    return [(i, k[i], k[i + 1]) for i in range(len(k) - 1) if k[i] < k[i + 1]]


def gauss_rule(q, a, b):
    """q-point Gauss-Legendre rule on [a, b] (library nodes/weights on [-1, 1])."""
    t, w = np.polynomial.legendre.leggauss(q)
    return a + (b - a) * (t + 1.0) / 2.0, w * (b - a) / 2.0


def quadrature(knots, q):
    """Composite rule: q Gauss points on every element.  Returns (x, w, elem)
    where elem[j] is the index into elements(knots) of the point x[j]."""
    xs, ws, es = [], [], []
    for e, (_, a, b) in enumerate(elements(knots)):
        x, w = gauss_rule(q, a, b)
        xs.append(x)
        ws.append(w)
        es.append(np.full(q, e))
    return np.concatenate(xs), np.concatenate(ws), np.concatenate(es)


def univariate_matrices(knots, p, q=None, weight=None, interior=True):
    """1D mass and stiffness matrices on the Dirichlet space (Sec. 3):

        M_ij = int_0^1 B_i B_j,  K_ij = int_0^1 B_i' B_j',  i, j = 2..m-1,

    evaluated by the composite q-point Gauss rule (q = p+1 is exact).  An
    optional weight function w(x) gives int w B_i B_j and int w B_i' B_j'.
    Returns (M, K) of order n = m-2 (order m with interior=False).
    """
    q = p + 1 if q is None else q
    x, w, _ = quadrature(knots, q)
    if weight is not None:
        w = w * weight(x)
    sl = slice(1, -1) if interior else slice(None)
    B = basis(knots, p, x)[:, sl]
    dB = basis_derivative(knots, p, x)[:, sl]
    M = B.T @ (w[:, None] * B)
    K = dB.T @ (w[:, None] * dB)
    return M, K
