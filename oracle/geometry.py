"""Geometry maps, coefficient, the matrix Q and the right-hand sides.

Paper Sec. 2.1: A_ij = int grad(B_i)^T Q grad(B_j) over the parameter domain
with Q = det(J_F) J_F^-T K J_F^-1 (eq. Q).  The paper's J_F is the transposed
Jacobian; with J_ij = dF_i/dxi_j the same matrix reads

    Q = |det J| J^-1 K J^-T,

(chain rule: grad_x = J^-T grad_xi, dx = |det J| dxi).  Test infrastructure
only.  The maps are the analytic ones described in `synth`.
"""
from __future__ import annotations

import numpy as np


def map_and_jacobian(geom, xi):
    """F(xi) and J(xi) = dF/dxi for points xi of shape (P, d).

    Returns (x, J) with x of shape (P, d) and J of shape (P, d, d).
    """
    xi = np.asarray(xi, float)
    P, d = xi.shape
    kind = geom["kind"]
    if kind == "identity":
        return xi.copy(), np.broadcast_to(np.eye(d), (P, d, d)).copy()
    if kind == "ring":
        # ((1+xi1) cos(pi xi2 / 2), (1+xi1) sin(pi xi2 / 2) [, xi3])
        r = 1.0 + xi[:, 0]
        th = 0.5 * np.pi * xi[:, 1]
        x = np.zeros((P, d))
        J = np.zeros((P, d, d))
        x[:, 0] = r * np.cos(th)
        x[:, 1] = r * np.sin(th)
        J[:, 0, 0] = np.cos(th)
        J[:, 0, 1] = -0.5 * np.pi * r * np.sin(th)
        J[:, 1, 0] = np.sin(th)
        J[:, 1, 1] = 0.5 * np.pi * r * np.cos(th)
        if d == 3:
            x[:, 2] = xi[:, 2]
            J[:, 2, 2] = 1.0
        return x, J
    if kind == "warped":
        # xi + a sum_k c_k prod_l sin(pi m_kl xi_l)
        a = geom["amp"]
        c = np.asarray(geom["c"], float)
        m = np.asarray(geom["m"], float)
        x = xi.copy()
        J = np.broadcast_to(np.eye(d), (P, d, d)).copy()
        for k in range(c.shape[0]):
            s = np.sin(np.pi * m[k] * xi)              # (P, d)
            dc = np.pi * m[k] * np.cos(np.pi * m[k] * xi)
            prod = np.prod(s, axis=1)
            x += a * prod[:, None] * c[k][None, :]
            for j in range(d):
                others = np.prod(np.delete(s, j, axis=1), axis=1)
                J[:, :, j] += a * (dc[:, j] * others)[:, None] * c[k][None, :]
        return x, J
    raise ValueError(f"unknown geometry kind {kind!r}")


def kappa(coef, x):
    """Scalar coefficient kappa(x), K = kappa I."""
    kind = coef["kind"]
    if kind == "one":
        return np.ones(len(x))
    if kind == "sincos":
        return 1.0 + coef["amp"] * np.sin(2 * np.pi * coef["f1"] * x[:, 0] + coef["phi1"]) * \
            np.cos(2 * np.pi * coef["f2"] * x[:, 1] + coef["phi2"])
    raise ValueError(f"unknown coefficient kind {kind!r}")


def q_matrix(problem, xi):
    """Q(xi) = |det J| J^-1 (kappa I) J^-T at the points xi, plus det J.

    Returns (Q, detJ, x) with Q of shape (P, d, d).
    """
    x, J = map_and_jacobian(problem["geometry"], xi)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    kap = kappa(problem["coefficient"], x)
    Q = (np.abs(det) * kap)[:, None, None] * (Jinv @ np.swapaxes(Jinv, 1, 2))
    return Q, det, x


def rhs(f, x):
    """Right-hand side f(x) of -div(K grad u) = f (Sec. 2.1 eq. poisson).
    Optional keys: "amp" (a factor; for sinprod the whole amplitude, default
    d pi^2) and, for sinprod, "k" (one frequency per direction, default 1)."""
    kind = f["kind"]
    d = x.shape[1]
    if kind == "sinprod":        # u = prod sin(pi x_i), K = I (default amp and k)
        amp = f.get("amp", d * np.pi ** 2)
        k = np.asarray(f.get("k", np.ones(d)), float)
        return amp * np.prod(np.sin(k * np.pi * x), axis=1)
    amp = f.get("amp", 1.0)
    if kind == "paper_poly":     # Sec. 7: f = 2 sum (x_i^2 - x_i)
        return amp * 2.0 * np.sum(x * x - x, axis=1)
    if kind == "bubble":         # u = prod x_l (1 - x_l), K = I
        g = x * (1.0 - x)
        return amp * 2.0 * sum(np.prod(np.delete(g, i, axis=1), axis=1) for i in range(d))
    if kind == "one":
        return amp * np.ones(len(x))
    raise ValueError(f"unknown rhs kind {kind!r}")
