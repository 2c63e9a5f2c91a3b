"""Multi-patch L-shaped domain and the overlapping additive Schwarz
preconditioners P_EAS and P_IAS (Sec. 6 eq. Peas and eq. Pias; Sec. 7,
multi-patch experiment and Table L).  Test infrastructure only.

Readings (the paper's figure of the domain is not part of its text):
  * Omega = [0,1]^2 without (1/2,1] x (1/2,1], split into three square patches
        Omega_1 = [0,1/2] x [1/2,1]   (above the corner patch)
        Omega_2 = [0,1/2] x [0,1/2]   (the corner patch)
        Omega_3 = [1/2,1] x [0,1/2]   (right of the corner patch)
    with F_k(xi) = o_k + xi/2.  Every patch carries the tensor B-splines of
    one open knot vector in both directions, so the meshes match on the two
    interfaces G12 = Omega_1 /\\ Omega_2 and G23 = Omega_2 /\\ Omega_3
    (the conforming case of Sec. 6).  "h^-1" of Table L is read as the number
    of elements per patch and direction.
  * C^0 gluing: the patch functions that do not vanish on an interface are
    identified pairwise (same index along the interface); every global
    function that does not vanish on the boundary of Omega is removed
    (homogeneous Dirichlet condition).
  * Poisson with K = I.  F_k is a similarity, and the 2D Dirichlet energy is
    invariant under similarities, so each patch contributes the parametric
    Kronecker sum M (x) K + K (x) M of the full univariate matrices.
  * Subdomains Theta_1 = Omega_1 u Omega_2 and Theta_2 = Omega_2 u Omega_3
    (the pairs of patches sharing an interface).  R_i keeps the global
    functions supported in Theta_i that vanish on its boundary: the interior
    functions of Theta_i seen as one patch whose knot vector has a knot of
    multiplicity p at the interface.  A_i = R_i A R_i^T is then the Dirichlet
    stiffness matrix of Theta_i.
  * P_i is the preconditioner of eq. prec for Theta_i in its own parameter
    domain [0,1]^2; the 2:1 stretch of Theta_i is deliberately not put into
    P_i, as in the paper's experiment.
  * Right-hand side: the paper does not state it for this experiment; the
    tests use f = 2 sum (x_i^2 - x_i), its choice for the other experiments.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fd, pcg, splines


def merged_knots(knots, p):
    """Knot vector on [0,1] of two copies of `knots` placed on [0,1/2] and
    [1/2,1], joined by a knot of multiplicity p at 1/2 (C^0 continuity)."""
    k = splines.check_knots(knots, p)
    inner = k[p + 1: -p - 1]
    return np.concatenate([np.zeros(p + 1), 0.5 * inner, np.full(p, 0.5), 0.5 + 0.5 * inner, np.ones(p + 1)])


# patch index -> lower-left corner o_k
CORNERS = {1: (0.0, 0.5), 2: (0.0, 0.0), 3: (0.5, 0.0)}


class LShape:
    """Global dofs, stiffness, load and Schwarz subdomains of the L-shaped
    three-patch problem.  Patch function (a, b): a = index along x
    (direction 1), b = index along y, both 0..m-1 including boundary ones."""

    def __init__(self, knots, p):
        self.p = p
        self.knots = splines.check_knots(knots, p)
        self.m = m = splines.n_basis(self.knots, p)
        if m < 3:
            raise ValueError("need at least one interior function per patch and direction")
        # canonical key of every patch function: glued copies share one key
        def key(k, a, b):
            if k == 1 and b == 0:
                return (2, a, m - 1)      # bottom row of Omega_1 = top row of Omega_2
            if k == 3 and a == 0:
                return (2, m - 1, b)      # left column of Omega_3 = right column of Omega_2
            return (k, a, b)

        # patch edges that lie on the boundary of Omega
        def on_boundary(k, a, b):
            if k == 1:
                return a == 0 or a == m - 1 or b == m - 1
            if k == 2:
                return a == 0 or b == 0
            return b == 0 or a == m - 1 or b == m - 1

        dirichlet = set()
        for k in (1, 2, 3):
            for b in range(m):
                for a in range(m):
                    if on_boundary(k, a, b):
                        dirichlet.add(key(k, a, b))
        ids = {}
        self.gid = {}
        for k in (1, 2, 3):
            g = np.full((m, m), -1, dtype=np.int64)  # g[b, a]
            for b in range(m):
                for a in range(m):
                    kk = key(k, a, b)
                    if kk in dirichlet:
                        continue
                    if kk not in ids:
                        ids[kk] = len(ids)
                    g[b, a] = ids[kk]
            self.gid[k] = g
        self.N = len(ids)

    # ---- global system (Sec. 6: the multi-patch Galerkin matrix) ----
    def matrix(self):
        """A = sum_k G_k^T (M (x) K + K (x) M) G_k, CSR (N x N), where G_k maps
        the patch functions to the global ones (Dirichlet ones dropped)."""
        Mf, Kf = splines.univariate_matrices(self.knots, self.p, interior=False)
        Ap = (sp.kron(sp.csr_matrix(Mf), sp.csr_matrix(Kf)) + sp.kron(sp.csr_matrix(Kf), sp.csr_matrix(Mf))).tocoo()
        rows, cols, vals = [], [], []
        for k in (1, 2, 3):
            g = self.gid[k].reshape(-1)   # patch index b*m + a -> global id
            gr, gc = g[Ap.row], g[Ap.col]
            keep = (gr >= 0) & (gc >= 0)
            rows.append(gr[keep])
            cols.append(gc[keep])
            vals.append(Ap.data[keep])
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(self.N, self.N))
        return A.tocsr()

    def matrix_rows(self, rows):
        """Rows of A for a few global dofs (CSR, len(rows) x N) from the same
        patch sums, without forming A: for large meshes."""
        Mf, Kf = splines.univariate_matrices(self.knots, self.p, interior=False)
        p, m = self.p, self.m
        where = {int(g): [] for g in rows}
        for k in (1, 2, 3):
            bs, as_ = np.nonzero(np.isin(self.gid[k], list(where)))
            for b, a in zip(bs, as_):
                where[int(self.gid[k][b, a])].append((k, b, a))
        ri, ci, vals = [], [], []
        for j, g in enumerate(rows):
            for k, b, a in where[int(g)]:
                for bb in range(max(0, b - p), min(m, b + p + 1)):
                    for aa in range(max(0, a - p), min(m, a + p + 1)):
                        col = self.gid[k][bb, aa]
                        if col >= 0:
                            ri.append(j)
                            ci.append(col)
                            vals.append(Mf[b, bb] * Kf[a, aa] + Kf[b, bb] * Mf[a, aa])
        return sp.csr_matrix((vals, (ri, ci)), shape=(len(rows), self.N))

    def load(self, f):
        """b_g = sum_k int_{Omega_k} f B_g dx by the (p+1)-point Gauss rule per
        element; dx = dxi / 4 on every patch."""
        x, w, _ = splines.quadrature(self.knots, self.p + 1)
        B = splines.basis(self.knots, self.p, x)           # (nq, m)
        from .geometry import rhs
        out = np.zeros(self.N)
        for k in (1, 2, 3):
            ox, oy = CORNERS[k]
            X, Y = np.meshgrid(ox + 0.5 * x, oy + 0.5 * x)  # [qy, qx]
            F = rhs(f, np.stack([X.ravel(), Y.ravel()], axis=1)).reshape(X.shape)
            bk = 0.25 * (B * w[:, None]).T @ F @ (B * w[:, None])   # [b, a]
            g = self.gid[k]
            keep = g >= 0
            np.add.at(out, g[keep], bk[keep])
        return out

    # ---- Schwarz subdomains (Sec. 6) ----
    def subdomain(self, i):
        """R_i as an index array in the tensor order of Theta_i (direction 1
        fastest) and the two knot vectors of Theta_i's parameter domain."""
        m = self.m
        km = merged_knots(self.knots, self.p)
        if i == 1:   # Omega_2 (bottom) and Omega_1 (top) stacked along y
            rows = []
            for bb in range(1, 2 * m - 2):
                for a in range(1, m - 1):
                    rows.append(self.gid[2][bb, a] if bb < m else self.gid[1][bb - m + 1, a])
            kn = [self.knots, km]
        elif i == 2:  # Omega_2 (left) and Omega_3 (right) side by side along x
            rows = []
            for b in range(1, m - 1):
                for aa in range(1, 2 * m - 2):
                    rows.append(self.gid[2][b, aa] if aa < m else self.gid[3][b, aa - m + 1])
            kn = [km, self.knots]
        else:
            raise ValueError("subdomain index is 1 or 2")
        R = np.asarray(rows, dtype=np.int64)
        if np.any(R < 0):
            raise AssertionError("a subdomain function was taken as a Dirichlet one")
        return R, kn

    def square_index(self):
        """Position of every global dof in the interior tensor grid of the
        bounding square [0,1]^2 carrying the merged knot vector in both
        directions (direction 1 fastest, n = 2m-3 per direction)."""
        m = self.m
        n = 2 * m - 3
        pos = np.full(self.N, -1, dtype=np.int64)
        shift = {1: (0, m - 1), 2: (0, 0), 3: (m - 1, 0)}
        for k in (1, 2, 3):
            sa, sb = shift[k]
            g = self.gid[k]
            for b in range(m):
                for a in range(m):
                    if g[b, a] >= 0:
                        pos[g[b, a]] = (b + sb - 1) * n + (a + sa - 1)
        return pos, n


class Schwarz:
    """P_EAS^-1 = sum_i R_i^T A_i^-1 R_i (eq. Peas) and P_IAS^-1 =
    sum_i R_i^T P_i^-1 R_i with P_i applied by fast diagonalisation
    (eq. Pias with the local approximation taken as P_i)."""

    def __init__(self, L: LShape, A=None):
        self.L = L
        self._A = A
        self.R, self.factors, self.lu = [], [], []
        for i in (1, 2):
            R, kn = L.subdomain(i)
            self.R.append(R)
            self.factors.append(fd.setup({"degree": L.p, "quad": L.p + 1, "knots": kn}))
            self.lu.append(None)

    @property
    def A(self):
        if self._A is None:
            self._A = self.L.matrix()
        return self._A

    def ias(self, r):
        z = np.zeros_like(r)
        for R, F in zip(self.R, self.factors):
            z[R] += fd.fd_apply(F, r[R])
        return z

    def eas(self, r):
        z = np.zeros_like(r)
        for j, R in enumerate(self.R):
            if self.lu[j] is None:
                self.lu[j] = spla.splu(self.A[R][:, R].tocsc())
            z[R] += self.lu[j].solve(r[R])
        return z

    def solve(self, b, kind="ias", rtol=1e-8, maxit=500):
        M = self.ias if kind == "ias" else self.eas
        return pcg.pcg(lambda v: self.A @ v, M, b, rtol=rtol, maxit=maxit)
