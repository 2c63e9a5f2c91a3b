"""Galerkin stiffness matrix A and load vector b by an element loop.

Paper Sec. 2.1 eq. A: A_ij = int_[0,1]^d grad(B_i)^T Q grad(B_j) dxi over the
Dirichlet space V_h of eq. Vh (B-splines 2..m-1 in every direction), with the
scalar index i = 1 + sum_l n^(l-1) (i_l - 2): direction 1 varies fastest, so a
vector is stored as an array of shape (n3, n2, n1) (2D: (n2, n1)).

The integral is the sum over mesh elements (tensor products of nonempty knot
spans) of the q^d-point tensor Gauss rule, q = problem["quad"] (p+1 by
default).  On each element the (p+1)^d nonzero B-splines give a local matrix

    A^e_ab = sum_t w_t grad(B_a)(t)^T Q(t) grad(B_b)(t),

which is added into the global rows/columns of the interior functions.  The
load vector uses the same rule: b_i = sum_t w_t |det J(t)| f(F(t)) B_i(t).
Test infrastructure only.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import geometry, splines


def dofs_per_direction(problem):
    p = problem["degree"]
    return [splines.n_basis(k, p) - 2 for k in problem["knots"]]


def _direction_tables(knots, p, q):
    """Per element of one direction: Gauss points, weights, values and
    derivatives of the p+1 B-splines nonzero there and their dof indices
    (B-spline index minus one; -1 and n mark the two removed functions)."""
    tabs = []
    for (k, a, b) in splines.elements(knots):
        x, w = splines.gauss_rule(q, a, b)
        V = splines.basis(knots, p, x)[:, k - p:k + 1]
        dV = splines.basis_derivative(knots, p, x)[:, k - p:k + 1]
        dof = np.arange(k - p, k + 1) - 1
        tabs.append((x, w, V, dV, dof))
    return tabs


class _Mesh:
    def __init__(self, problem):
        self.problem = problem
        self.d = problem["dim"]
        self.p = problem["degree"]
        self.q = problem["quad"]
        for k in problem["knots"]:
            splines.check_knots(k, self.p)
        self.n = dofs_per_direction(problem)
        self.N = int(np.prod(self.n))
        self.tabs = [_direction_tables(k, self.p, self.q) for k in problem["knots"]]
        self.nel = [len(t) for t in self.tabs]

    def all_elements(self):
        return list(itertools.product(*[range(ne) for ne in self.nel]))

    def elements_touching(self, rows):
        """Elements in the support of the given (flat) dof indices."""
        out = set()
        for r in rows:
            idx = np.unravel_index(int(r), self.n[::-1])[::-1]  # (i1, i2, ...)
            per_dir = []
            for l in range(self.d):
                per_dir.append([e for e, t in enumerate(self.tabs[l]) if idx[l] in t[4]])
            out.update(itertools.product(*per_dir))
        return sorted(out)

    def element_data(self, els):
        """Tensor quadrature data for a chunk of elements.

        Returns xi (C, T, d), w (C, T), vals (C, T, L), grads (C, d, T, L),
        dof (C, L) with T = q^d points and L = (p+1)^d local functions,
        direction d the slowest and direction 1 the fastest index."""
        d = self.d
        els = np.asarray(els)
        C = len(els)
        X, W, V, dV, D = [], [], [], [], []
        for l in range(d):
            t = [self.tabs[l][e] for e in els[:, l]]
            X.append(np.stack([a[0] for a in t]))
            W.append(np.stack([a[1] for a in t]))
            V.append(np.stack([a[2] for a in t]))
            dV.append(np.stack([a[3] for a in t]))
            D.append(np.stack([a[4] for a in t]))
        q, L1 = self.q, self.p + 1

        def outer(mats):
            # mats[l]: (C, q, L1) for direction l; tensor with dir d-1 slowest
            if d == 2:
                r = np.einsum("eia,ejb->eijab", mats[1], mats[0])
            else:
                r = np.einsum("eia,ejb,ekc->eijkabc", mats[2], mats[1], mats[0])
            return r.reshape(C, q ** d, L1 ** d)

        vals = outer(V)
        grads = np.stack([outer([dV[l] if l == j else V[l] for l in range(d)]) for j in range(d)], axis=1)

        def outer_pts(vecs, reduce):
            if d == 2:
                return reduce(vecs[1][:, :, None], vecs[0][:, None, :]).reshape(C, -1)
            return reduce(reduce(vecs[2][:, :, None, None], vecs[1][:, None, :, None]),
                          vecs[0][:, None, None, :]).reshape(C, -1)

        w = outer_pts(W, np.multiply)
        xi = np.zeros((C, q ** d, d))
        for l in range(d):
            parts = [X[j] if j == l else np.zeros_like(X[j]) for j in range(d)]
            xi[:, :, l] = outer_pts(parts, np.add)
        # flat dof index of each local function, -1 where it is not in V_h
        dofs = np.zeros((C,) + (L1,) * d, dtype=np.int64)
        valid = np.ones((C,) + (L1,) * d, dtype=bool)
        stride = 1
        for l in range(d):
            shape = [C] + [1] * d
            shape[d - l] = L1
            dl = D[l].reshape(shape)
            dofs = dofs + dl * stride
            valid &= (dl >= 0) & (dl < self.n[l])
            stride *= self.n[l]
        dofs = np.where(valid, dofs, -1).reshape(C, -1)
        return xi, w, vals, grads, dofs


def _chunks(els, size):
    for s in range(0, len(els), size):
        yield els[s:s + size]


def assemble_matrix(problem, rows=None, chunk=None):
    """Stiffness matrix A (scipy CSR, N x N).  With `rows`, only the elements
    touching those rows are visited and only those rows are kept."""
    mesh = _Mesh(problem)
    d, L = mesh.d, (mesh.p + 1) ** mesh.d
    els = mesh.all_elements() if rows is None else mesh.elements_touching(rows)
    keep = None if rows is None else np.zeros(mesh.N, dtype=bool)
    if keep is not None:
        keep[np.asarray(rows, dtype=np.int64)] = True
    chunk = chunk or max(1, int(2e7 // (L * L + L * mesh.q ** d * (d + 2))))
    R, Cc, Vv = [], [], []
    for part in _chunks(els, chunk):
        xi, w, vals, grads, dofs = mesh.element_data(part)
        C, T = w.shape
        Q, det, _ = geometry.q_matrix(problem, xi.reshape(-1, d))
        if np.any(det <= 0):
            raise ValueError("det J <= 0 at a quadrature point")
        Q = Q.reshape(C, T, d, d)
        # A^e_ab = sum_t w_t sum_ij grad_i B_a(t) Q_ij(t) grad_j B_b(t), written as
        # two batched matrix products (library matmul) over the same sum
        G = np.swapaxes(grads, 1, 2)                     # (C, T, d, L): grad_i B_a(t)
        QG = np.matmul(Q, G) * w[:, :, None, None]       # (C, T, d, L): w_t sum_j Q_ij grad_j B_b
        Ae = np.matmul(np.swapaxes(G.reshape(C, T * d, -1), 1, 2), QG.reshape(C, T * d, -1))
        r = np.broadcast_to(dofs[:, :, None], Ae.shape)
        c = np.broadcast_to(dofs[:, None, :], Ae.shape)
        ok = (r >= 0) & (c >= 0)
        if keep is not None:
            ok &= keep[np.where(r >= 0, r, 0)]
        R.append(r[ok])
        Cc.append(c[ok])
        Vv.append(Ae[ok])
    A = sp.coo_matrix((np.concatenate(Vv), (np.concatenate(R), np.concatenate(Cc))),
                      shape=(mesh.N, mesh.N)).tocsr()
    A.sum_duplicates()
    return A


def assemble_load(problem, f, dofs_subset=None):
    """Load vector b_i = int_Omega f B_i dx = sum_t w_t |det J| f(F(t)) B_i(t)
    (the same Gauss rule as A).  Returns a flat array of length N (with a
    subset, only those entries are filled)."""
    mesh = _Mesh(problem)
    d = mesh.d
    els = mesh.all_elements() if dofs_subset is None else mesh.elements_touching(dofs_subset)
    b = np.zeros(mesh.N)
    L = (mesh.p + 1) ** d
    for part in _chunks(els, max(1, int(2e7 // (L * mesh.q ** d * (d + 2))))):
        xi, w, vals, grads, dofs = mesh.element_data(part)
        C, T = w.shape
        x, J = geometry.map_and_jacobian(problem["geometry"], xi.reshape(-1, d))
        g = (np.abs(np.linalg.det(J)) * geometry.rhs(f, x)).reshape(C, T) * w
        be = np.einsum("et,eta->ea", g, vals)
        ok = dofs >= 0
        np.add.at(b, dofs[ok], be[ok])
    if dofs_subset is not None:
        mask = np.zeros(mesh.N, dtype=bool)
        mask[np.asarray(dofs_subset, dtype=np.int64)] = True
        b[~mask] = 0.0
    return b


def quadrature_points(problem):
    """All Gauss points of the mesh with their weights: (xi (P, d), w (P,))."""
    mesh = _Mesh(problem)
    xs, ws = [], []
    for part in _chunks(mesh.all_elements(), 4096):
        xi, w, _, _, _ = mesh.element_data(part)
        xs.append(xi.reshape(-1, mesh.d))
        ws.append(w.reshape(-1))
    return np.concatenate(xs), np.concatenate(ws)


def q_spectral_bounds(problem):
    """Sec. 3 Prop. 1: (qmin, qmax) = the smallest and largest eigenvalue of
    Q = |det J| J^-1 (kappa I) J^-T over the Gauss points of the mesh.  With A
    and P assembled by the same rule, every eigenvalue of P^-1 A lies in
    [qmin, qmax]."""
    xi, _ = quadrature_points(problem)
    lo, hi = np.inf, -np.inf
    for k in range(0, len(xi), 1 << 18):
        Q, _, _ = geometry.q_matrix(problem, xi[k:k + (1 << 18)])
        ev = np.linalg.eigvalsh(Q)
        lo, hi = min(lo, ev[:, 0].min()), max(hi, ev[:, -1].max())
    return float(lo), float(hi)
