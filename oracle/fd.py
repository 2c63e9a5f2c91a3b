"""The preconditioner P and its fast-diagonalisation (FD) apply.

Paper Sec. 3 eq. prec: P_ij = int_[0,1]^d grad(B_i)^T grad(B_j) dxi, which by
the tensor structure is a Kronecker sum of the 1D stiffness K_d and mass M_d.
With direction 1 the fastest index (eq. Vh ordering) and the standard
Kronecker product (Sec. 2.2, last factor fastest):

    d = 2:  P = M2 (x) K1 + K2 (x) M1
    d = 3:  P = M3 (x) M2 (x) K1 + M3 (x) K2 (x) M1 + K3 (x) M2 (x) M1.

FD (Sec. 4.1 Alg. 1, Sec. 5.1 Alg. 3).  The pencils (K_d, M_d) are
diagonalised as K_d U_d = M_d U_d D_d with U_d^T M_d U_d = I, computed as the
paper describes: Cholesky M = L L^T, symmetric eigendecomposition of
L^-1 K L^-T = Ut D Ut^T, U = L^-T Ut.  Then

    P^-1 = (U3 (x) U2 (x) U1) Lambda^-1 (U3 (x) U2 (x) U1)^T,
    Lambda = D3 (x) I (x) I + I (x) D2 (x) I + I (x) I (x) D1.

The 3D listing writes the forward product without, and the backward product
with, the transpose; that contradicts U^T M U = I and the 2D algorithm, so the
forward product is taken with U_d^T and the backward one with U_d (reading
checked by the explicit-Kronecker pin).  A Kronecker matrix-vector product is
a sequence of mode products (Sec. 2.2 eq. kronprod): mode d multiplies axis d
of the (n3, n2, n1) array.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import splines


def generalized_eig(K, M):
    """U, lam with K U = M U diag(lam), U^T M U = I (Sec. 4.1 computational cost)."""
    L = np.linalg.cholesky(M)
    Linv = np.linalg.inv(L)
    Kt = Linv @ K @ Linv.T
    Kt = 0.5 * (Kt + Kt.T)
    lam, Ut = np.linalg.eigh(Kt)
    U = Linv.T @ Ut
    return U, lam


def setup(problem):
    """1D matrices and eigendecompositions for every direction (dir 1 first)."""
    p, q = problem["degree"], problem["quad"]
    out = []
    for kn in problem["knots"]:
        M, K = splines.univariate_matrices(kn, p, q)
        U, lam = generalized_eig(K, M)
        out.append({"M": M, "K": K, "U": U, "lam": lam})
    return out


def _axis(d, direction):
    """Array axis of direction `direction` (0-based) in the (n_d, ..., n_1) layout."""
    return d - 1 - direction


def mode_product(X, W, direction):
    """Y = X x_direction W: Y[.., k, ..] = sum_i W[k, i] X[.., i, ..] along the
    axis of `direction` (Sec. 2.2 eq. kronprod applied one factor at a time)."""
    ax = _axis(X.ndim, direction)
    return np.moveaxis(np.tensordot(W, X, axes=([1], [ax])), 0, ax)


def eigen_sum(lams):
    """Lambda as an array of shape (n_d, .., n_1): lam_1[k1] + lam_2[k2] (+ lam_3[k3])."""
    d = len(lams)
    S = np.zeros([len(l) for l in lams[::-1]])
    for direction, lam in enumerate(lams):
        shape = [1] * d
        shape[_axis(d, direction)] = len(lam)
        S = S + lam.reshape(shape)
    return S


def fd_apply(factors, r, scaling=None):
    """s = P^-1 r by fast diagonalisation; r of shape (n_d, .., n_1) or flat.

    Steps (Alg. 1 / Alg. 3): r~ = (U_d (x) .. (x) U_1)^T r; s~ = Lambda^-1 r~;
    s = (U_d (x) .. (x) U_1) s~.  With `scaling` S (same shape as r) the
    operator is S P^-1 S.
    """
    shape = tuple(len(f["lam"]) for f in factors[::-1])
    flat = r.ndim == 1
    t = np.asarray(r, float).reshape(shape)
    if scaling is not None:
        t = t * scaling.reshape(shape)
    for direction, f in enumerate(factors):
        t = mode_product(t, f["U"].T, direction)
    t = t / eigen_sum([f["lam"] for f in factors])
    for direction, f in enumerate(factors):
        t = mode_product(t, f["U"], direction)
    if scaling is not None:
        t = t * scaling.reshape(shape)
    return t.reshape(-1) if flat else t


def kron_P(factors):
    """Explicit Kronecker-sum P (dense), direction 1 fastest."""
    Ms = [f["M"] for f in factors]
    Ks = [f["K"] for f in factors]
    d = len(factors)
    P = 0
    for j in range(d):
        term = np.ones((1, 1))
        for l in reversed(range(d)):  # slowest factor first
            term = np.kron(term, Ks[l] if l == j else Ms[l])
        P = P + term
    return P


def apply_P(factors, x):
    """P x from the Kronecker sum itself, one term per direction, each term a
    sequence of mode products with the banded 1D matrices (K_j along
    direction j, M_l along the others; Sec. 2.2 eq. kronprod).  The 1D
    matrices are used as sparse matrices so that grids of 10^8 points stay
    within host memory and time."""
    import scipy.sparse as sps

    shape = tuple(len(f["lam"]) for f in factors[::-1])
    flat = np.ndim(x) == 1
    X = np.asarray(x, float).reshape(shape)
    d = len(factors)

    def along(T, B, direction):
        ax = _axis(d, direction)
        T0 = np.moveaxis(T, ax, 0)
        Y = (B @ T0.reshape(T0.shape[0], -1)).reshape(T0.shape)
        return np.moveaxis(Y, 0, ax)

    Ms = [sps.csr_matrix(f["M"]) for f in factors]
    Ks = [sps.csr_matrix(f["K"]) for f in factors]
    out = np.zeros(shape)
    for j in range(d):
        T = X
        for l in range(d):
            T = along(T, Ks[l] if l == j else Ms[l], l)
        out += T
    return out.reshape(-1) if flat else out


def diag_P(factors):
    """Diagonal of P from the 1D diagonals (Sec. 3 Kronecker sum)."""
    d = len(factors)
    out = 0
    for j in range(d):
        term = np.ones(1)
        for l in reversed(range(d)):
            f = factors[l]
            term = np.kron(term, np.diag(f["K"] if l == j else f["M"]))
        out = out + term
    return out
