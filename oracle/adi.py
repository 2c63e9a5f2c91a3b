"""Three-variable ADI of Douglas as an inexact application of P^-1 (Sec. 5.2,
eq. ADI3D, eq. ADI3D2, Alg. '3D ADI method'; Sec. 4.2 Thm. ADIprec for its use
as a CG preconditioner P_J).  Test infrastructure only.

Readings (the paper cites Douglas for the parameters without restating them):
  * [a, b]: the smallest and the largest eigenvalue of M_d^-1 K_d over the
    three directions (the paper takes one interval for all three).
  * Parameters for a count J: omega_j = a (b/a)^((j-1)/(J-1)), j = 1..J,
    geometric between a and b (J = 1: sqrt(a b)).  J is the smallest count
    with rho_J <= eps, at most J0 = ceil(1.16 ln(b/a) ln(1/eps)) (eq.
    ADI3Diter).  rho_J is evaluated exactly: the error operator T_J is
    diagonal in the eigenvector basis of the three pencils (K_d, M_d), with
    entry prod_j g_j(l1, l2, l3),
        g_j = 1 - 2 omega_j^2 (l1 + l2 + l3) / ((omega_j + l1)(omega_j + l2)(omega_j + l3)),
    so rho_J = ||T_J|| is the largest |prod_j g_j| over the triples of actual
    eigenvalues (the bound of the paper's rho_J over [a, b]^3 restricted to
    the spectrum).
  * eps = 0.1, the tolerance of the paper's 3D experiments.
  * Greedy parameters (eq. greedy1/2), the paper's alternative: the triple
    of largest remaining error over the actual eigenvalue triples (as for
    rho_J), the minimiser of |g| there in closed form (best_parameter), and
    sqrt(a b) as the first parameter, which the paper leaves open.
"""
from __future__ import annotations

import math

import numpy as np

from . import fd


def spectrum_interval(factors):
    lo = min(float(f["lam"].min()) for f in factors)
    hi = max(float(f["lam"].max()) for f in factors)
    return lo, hi


def geometric_parameters(a, b, J):
    if J == 1:
        return np.array([math.sqrt(a * b)])
    return a * (b / a) ** (np.arange(J) / (J - 1))


def error_factor(omegas, l1, l2, l3):
    """prod_j g_j at eigenvalue triples (broadcasting arrays)."""
    s = l1 + l2 + l3
    out = np.ones(np.broadcast(l1, l2, l3).shape)
    for w in omegas:
        out = out * (1.0 - 2.0 * w * w * s / ((w + l1) * (w + l2) * (w + l3)))
    return out


def rho(omegas, lams):
    """||T_J||: the largest |prod_j g_j| over all eigenvalue triples."""
    l1, l2, l3 = lams
    return float(np.abs(error_factor(omegas, l1[None, None, :], l2[None, :, None], l3[:, None, None])).max())


def parameters(factors, eps=0.1):
    """(omegas, rho_J, J0) by the rule in the module header."""
    a, b = spectrum_interval(factors)
    J0 = max(1, math.ceil(1.16 * math.log(b / a) * math.log(1.0 / eps)))
    lams = [f["lam"] for f in factors]
    for J in range(1, J0 + 1):
        w = geometric_parameters(a, b, J)
        r = rho(w, lams)
        if r <= eps:
            return w, r, J0
    return w, r, J0


def best_parameter(l1, l2, l3):
    """eq. greedy2: the omega >= 0 that minimises |g(omega; l1, l2, l3)|,
    g = 1 - 2 omega^2 S / ((omega + l1)(omega + l2)(omega + l3)).

    g = 0 where (omega + l1)(omega + l2)(omega + l3) = 2 S omega^2, i.e. at the
    positive roots of omega^3 - S omega^2 + e2 omega + e3 (none or two, by the
    signs of the coefficients); the smaller one is taken.  Without such a root
    g > 0 everywhere and the minimum is where 2 S omega^2 / prod(omega + l_d)
    peaks: d/d omega log(...) = 2/omega - sum 1/(omega + l_d) = 0, i.e. the one
    positive root of omega^3 - e2 omega - 2 e3.  (S, e2, e3: the elementary
    symmetric functions of l1, l2, l3.)"""
    S = l1 + l2 + l3
    e2 = l1 * l2 + l1 * l3 + l2 * l3
    e3 = l1 * l2 * l3

    def positive_roots(coef):
        r = np.roots(coef)
        return sorted(float(x.real) for x in r if abs(x.imag) <= 1e-9 * abs(x) and x.real > 0)

    zeros = positive_roots([1.0, -S, e2, e3])
    if zeros:
        return zeros[0]
    return positive_roots([1.0, 0.0, -e2, -2.0 * e3])[-1]


def greedy_parameters(factors, eps=0.1):
    """(omegas, rho_J, J0) by the greedy rule of eq. greedy1/2: after k steps
    take the eigenvalue triple where |prod_{j<=k} g_j| is largest (the first
    one in (k3, k2, k1) order on ties) and the next omega by best_parameter;
    stop once the largest |prod g_j| is <= eps, or at J0 steps.  The first
    parameter is sqrt(a b), the one-parameter choice of the geometric rule."""
    a, b = spectrum_interval(factors)
    J0 = max(1, math.ceil(1.16 * math.log(b / a) * math.log(1.0 / eps)))
    l1, l2, l3 = (f["lam"] for f in factors)
    L1, L2, L3 = l1[None, None, :], l2[None, :, None], l3[:, None, None]
    w = [math.sqrt(a * b)]
    G = error_factor(w, L1, L2, L3)
    while np.abs(G).max() > eps and len(w) < J0:
        k3, k2, k1 = np.unravel_index(np.argmax(np.abs(G)), G.shape)
        w.append(best_parameter(float(l1[k1]), float(l2[k2]), float(l3[k3])))
        G = G * error_factor(w[-1:], L1, L2, L3)
    return np.array(w), float(np.abs(G).max()), J0


def _along(X, B, direction):
    """Apply the n_d x n_d matrix B along `direction` of X (shape (n3, n2, n1))."""
    return fd.mode_product(X, B, direction)


def _solve_along(X, B, direction):
    return fd.mode_product(X, np.linalg.inv(B), direction)


def apply(factors, r, omegas):
    """s_J for P s = r by the steps of Alg. '3D ADI method' (eq. ADI3D2), s_0 = 0.
    factors: fd.setup output (M, K per direction, direction 1 first)."""
    shape = tuple(len(f["lam"]) for f in factors[::-1])
    flat = np.ndim(r) == 1
    r = np.asarray(r, float).reshape(shape)
    M1, M2, M3 = (f["M"] for f in factors)
    K1, K2, K3 = (f["K"] for f in factors)
    rt = 2.0 * _solve_along(_solve_along(r, M2, 1), M3, 2)       # r~ = 2 (I x M2 x M3)^-1 r
    s = np.zeros(shape)
    v = np.zeros(shape)
    for w in omegas:
        u = _solve_along(_along(s, K2, 1), M2, 1)                # u_j = (I x M2^-1 K2 x I) s_{j-1}
        rs = rt - _along(s, K1 - w * M1, 0) - 2.0 * _along(u + v, M1, 0)
        s1 = _solve_along(rs, K1 + w * M1, 0)                    # s*_j
        rss = _along(u + w * s1, M2, 1)
        s2 = _solve_along(rss, K2 + w * M2, 1)                   # s**_j
        bj = v + w * s2
        s = _solve_along(_along(bj, M3, 2), K3 + w * M3, 2)      # s_j
        v = bj - w * s                                           # v_{j+1}
    return s.reshape(-1) if flat else s


def closed_form(factors, r, omegas):
    """s_J = U diag((1 - prod_j g_j) / (l1 + l2 + l3)) U^T r (the error
    operator is diagonal in the FD eigenbasis, Sec. 4.1 / 5.1)."""
    shape = tuple(len(f["lam"]) for f in factors[::-1])
    flat = np.ndim(r) == 1
    t = np.asarray(r, float).reshape(shape)
    for d, f in enumerate(factors):
        t = fd.mode_product(t, f["U"].T, d)
    l1, l2, l3 = (f["lam"] for f in factors)
    L1, L2, L3 = l1[None, None, :], l2[None, :, None], l3[:, None, None]
    t = t * (1.0 - error_factor(omegas, L1, L2, L3)) / (L1 + L2 + L3)
    for d, f in enumerate(factors):
        t = fd.mode_product(t, f["U"], d)
    return t.reshape(-1) if flat else t
