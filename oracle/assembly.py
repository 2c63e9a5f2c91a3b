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


def q_spectral_bounds(problem, local=False):
    """Sec. 3 Prop. 1: (qmin, qmax) = the smallest and largest eigenvalue of
    Q = |det J| J^-1 (kappa I) J^-T over the Gauss points of the mesh.  With A
    and P assembled by the same rule, every eigenvalue of P^-1 A lies in
    [qmin, qmax].  local=True also returns qloc, the largest pointwise ratio
    lambda_max(Q(x)) / lambda_min(Q(x)) over the same points."""
    xi, _ = quadrature_points(problem)
    lo, hi, loc = np.inf, -np.inf, 0.0
    for k in range(0, len(xi), 1 << 18):
        Q, _, _ = geometry.q_matrix(problem, xi[k:k + (1 << 18)])
        ev = np.linalg.eigvalsh(Q)
        lo, hi = min(lo, ev[:, 0].min()), max(hi, ev[:, -1].max())
        loc = max(loc, float(np.max(ev[:, -1] / ev[:, 0])))
    return (float(lo), float(hi), loc) if local else (float(lo), float(hi))


def _along(T, B, direction):
    """Mode product of the (n_d, .., n_1) array T with the matrix B along
    `direction` (0-based; direction 1 is the last axis): Sec. 2.2 eq. kronprod
    one factor at a time."""
    ax = T.ndim - 1 - direction
    T0 = np.moveaxis(T, ax, 0)
    Y = (B @ T0.reshape(T0.shape[0], -1)).reshape((B.shape[0],) + T0.shape[1:])
    return np.moveaxis(Y, 0, ax)


def ring_operator(problem, absolute=False):
    """A of the thick quarter ring (3D) or quarter annulus (2D), K = I, as a
    matrix-free product x -> A x (flat or shaped (n_d, .., n_1)).

    With J_ij = dF_i/dxi_j, the ring map F = ((1+xi1) cos(pi xi2/2),
    (1+xi1) sin(pi xi2/2) [, xi3]) has det J = w(xi1) = pi (1 + xi1)/2 and
    J^T J = diag(1, w^2 [, 1]), so eq. Q gives Q = |det J| (J^T J)^-1 =
    diag(w, 1/w [, w]): diagonal, each entry a function of xi1 alone.  The
    tensor Gauss rule of eq. A then factorises into Kronecker products of
    weighted univariate matrices (direction 1 fastest):

        3D  A = M3 (x) M2 (x) K1[w] + M3 (x) K2 (x) M1[1/w] + K3 (x) M2 (x) M1[w]
        2D  A = M2 (x) K1[w] + K2 (x) M1[1/w]

    with M[v]_ij = int v B_i B_j and K[v]_ij = int v B_i' B_j' by the same
    q-point rule.  Each term is applied as mode products with the banded
    univariate matrices (sparse), so 10^6-10^7 unknowns take a fraction of a
    second per product.  absolute=True applies the same terms with every
    univariate entry replaced by its magnitude: an entrywise upper bound of
    |A|, for row scales sum_j |a_ij| |x_j| of rounding tolerances.  Pinned
    against assemble_matrix (the element loop)."""
    import scipy.sparse as sps

    if problem["geometry"]["kind"] != "ring" or problem["coefficient"]["kind"] != "one":
        raise ValueError("ring_operator needs the ring map and kappa = 1")
    p, q, d = problem["degree"], problem["quad"], problem["dim"]
    kn = problem["knots"]
    w = lambda s: 0.5 * np.pi * (1.0 + s)
    M1w, K1w = splines.univariate_matrices(kn[0], p, q, weight=w)
    M1i, _ = splines.univariate_matrices(kn[0], p, q, weight=lambda s: 1.0 / w(s))
    M2, K2 = splines.univariate_matrices(kn[1], p, q)
    sp_ = (lambda m: sps.csr_matrix(np.abs(m))) if absolute else sps.csr_matrix
    if d == 2:
        terms = [(sp_(K1w), sp_(M2)), (sp_(M1i), sp_(K2))]
    else:
        M3, K3 = splines.univariate_matrices(kn[2], p, q)
        terms = [(sp_(K1w), sp_(M2), sp_(M3)), (sp_(M1i), sp_(K2), sp_(M3)), (sp_(M1w), sp_(M2), sp_(K3))]
    shape = tuple(t.shape[0] for t in terms[0][::-1])

    def apply(x):
        flat = np.ndim(x) == 1
        X = np.asarray(x, float).reshape(shape)
        out = np.zeros(shape)
        for term in terms:
            T = X
            for direction, B in enumerate(term):
                T = _along(T, B, direction)
            out += T
        return out.reshape(-1) if flat else out

    return apply


def _load_tables(problem):
    """Per direction: composite Gauss points and the weighted basis matrix
    W_l B_l (points x interior functions)."""
    p, q = problem["degree"], problem["quad"]
    xs, Bs = [], []
    for kn in problem["knots"]:
        x, w, _ = splines.quadrature(kn, q)
        xs.append(x)
        Bs.append(splines.basis(kn, p, x)[:, 1:-1] * w[:, None])
    return xs, Bs


def _load_slabs(problem, f, first, stop, slab):
    """Contribution to b of the Gauss points whose last-direction index lies
    in [first, stop), `slab` of them at a time."""
    d = problem["dim"]
    xs, Bs = _load_tables(problem)
    b = np.zeros([B.shape[1] for B in Bs][::-1])
    for s0 in range(first, stop, slab):
        sl = slice(s0, min(s0 + slab, stop))
        grids = np.meshgrid(*([xs[d - 1][sl]] + [xs[l] for l in range(d - 2, -1, -1)]), indexing="ij")
        pts = np.stack(grids[::-1], axis=-1).reshape(-1, d)  # (direction 1 fastest)
        x, J = geometry.map_and_jacobian(problem["geometry"], pts)
        g = (np.abs(np.linalg.det(J)) * geometry.rhs(f, x)).reshape(grids[0].shape)
        T = g
        for direction in range(d - 1):
            T = _along(T, Bs[direction].T, direction)
        b += _along(T, Bs[d - 1][sl].T, d - 1)
    return b


def assemble_load_tensor(problem, f, slab=4, workers=None, pool_above=1 << 22):
    """The load vector of assemble_load, b_i = sum_t w_t |det J(t)| f(F(t)) B_i(t),
    with the sum over the tensor Gauss points taken one direction at a time
    (sum factorisation; the same sum reordered).  With B_l the matrix of
    direction l's interior B-splines at its composite Gauss points and W_l
    its weights, b = (B_d^T W_d (x) .. (x) B_1^T W_1) g for g = |det J| f(F) on
    the tensor grid of points, visited in slabs of `slab` points along the
    last direction so that 10^8 points fit in memory.  Grids above
    `pool_above` points are split over `workers` fresh host processes (numpy holds the
    interpreter lock in the small-matrix routines, so threads do not scale);
    their contributions are added in order.  Pinned against assemble_load
    (the element loop)."""
    import concurrent.futures
    import multiprocessing
    import os

    d = problem["dim"]
    xs, _ = _load_tables(problem)
    npts = int(np.prod([len(x) for x in xs]))
    nlast = len(xs[d - 1])
    workers = workers or min(16, os.cpu_count() or 1, nlast)
    if npts <= pool_above or workers <= 1:
        return _load_slabs(problem, f, 0, nlast, slab).reshape(-1)
    cuts = np.linspace(0, nlast, workers + 1).astype(int)
    ctx = multiprocessing.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as pool:
        futs = [pool.submit(_load_slabs, problem, f, int(a), int(b), slab) for a, b in zip(cuts[:-1], cuts[1:])]
        b = None
        for fu in futs:
            part = fu.result()
            b = part if b is None else b + part
    return b.reshape(-1)
