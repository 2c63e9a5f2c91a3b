"""Preconditioned conjugate gradients (Sec. 3: P is SPD, so CG with P applies).

The paper gives no listing, tolerance, initial guess or norm.  Reading used
throughout: x0 = 0, stop when ||r_k||_2 <= rtol ||b||_2 on the recursively
updated residual, at most maxit iterations; one iteration is one product with
A and one preconditioner application.  On exit the true residual b - A x is
evaluated; if it does not meet the tolerance the iteration restarts from it.

`flexible=True` uses the Polak-Ribiere form of beta,
beta = (r_{k+1}, z_{k+1} - z_k) / (r_k, z_k), which tolerates a preconditioner
that is only approximately fixed (mixed-precision applies).  With an exact,
fixed preconditioner (r_{k+1}, z_k) = 0 and both forms coincide.
Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def pcg(apply_A, apply_M, b, rtol=1e-8, maxit=2000, flexible=False, x0=None, max_restarts=3):
    b = np.asarray(b, float)
    x = np.zeros_like(b) if x0 is None else np.array(x0, float)
    bnorm = np.linalg.norm(b)
    hist = []
    iters = 0
    restarts = 0
    if bnorm == 0.0:
        return x, {"iters": 0, "relres": 0.0, "true_relres": 0.0, "history": [0.0], "converged": True}
    r = b - apply_A(x) if x0 is not None else b.copy()
    while True:
        hist.append(np.linalg.norm(r) / bnorm)
        converged = hist[-1] <= rtol
        if not converged:
            z = apply_M(r)
            rho = r @ z
            p = z.copy()
            while iters < maxit:
                q = apply_A(p)
                pq = p @ q
                if not pq > 0:
                    raise FloatingPointError("CG breakdown: p^T A p <= 0")
                alpha = rho / pq
                x = x + alpha * p
                r = r - alpha * q
                iters += 1
                hist.append(np.linalg.norm(r) / bnorm)
                if hist[-1] <= rtol:
                    converged = True
                    break
                z_old = z
                z = apply_M(r)
                rho_new = r @ z
                if flexible:
                    beta = (rho_new - r @ z_old) / rho
                else:
                    beta = rho_new / rho
                rho = rho_new
                p = z + beta * p
        true_res = np.linalg.norm(b - apply_A(x)) / bnorm
        if true_res <= rtol or iters >= maxit or restarts >= max_restarts:
            break
        restarts += 1
        r = b - apply_A(x)
    return x, {"iters": iters, "relres": hist[-1], "true_relres": true_res, "history": hist,
               "converged": bool(true_res <= rtol), "restarts": restarts}


def solve(problem, A, factors, b, rtol=1e-8, maxit=2000, flexible=False, scaling=None):
    """PCG for A u = b with the FD preconditioner (optionally S P^-1 S)."""
    from . import fd
    return pcg(lambda v: A @ v, lambda r: fd.fd_apply(factors, r, scaling), b, rtol, maxit, flexible)
