"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: knot vectors, the random parameters of the
geometry maps and coefficients, random right-hand sides and the workload
descriptions.  It holds none of the solver's arithmetic (no basis functions, no
quadrature, no assembly, no preconditioner).  Both the CPU oracle and the HIP
library receive the plain dictionaries built here and interpret them on their
own.

Problem dictionary (every field is plain data):

    {
      "dim": 2 | 3,
      "degree": p,
      "knots": [np.ndarray, ...]          # one open knot vector per direction
      "geometry": {"kind": "identity"}
                | {"kind": "ring"}        # 2D quarter annulus / 3D thick quarter ring
                | {"kind": "warped", "amp": a, "c": (K, d) array, "m": (K, d) int array},
      "coefficient": {"kind": "one"}
                   | {"kind": "sincos", "amp": a, "f1": f1, "f2": f2, "phi1": p1, "phi2": p2},
      "quad": q,                          # Gauss points per element per direction
    }

The maps (paper Sec. 2.1 asks only for a smooth single-patch parametrisation):

* ring:   F(xi) = ((1+xi1) cos(pi xi2/2), (1+xi1) sin(pi xi2/2) [, xi3])
* warped: F(xi) = xi + a * sum_k c_k prod_l sin(pi m_kl xi_l)  (boundary fixed)

Coefficient K(x) = kappa(x) I with kappa = 1 + amp sin(2 pi f1 x + phi1) cos(2 pi f2 y + phi2).
"""
from __future__ import annotations

import numpy as np

# --------------------------------------------------------------------------
# knot vectors (paper eq. knot-vector: open, first/last p+1 knots repeated)
# --------------------------------------------------------------------------


def uniform_knots(E: int, p: int) -> np.ndarray:
    """Open uniform knot vector with E elements, interior multiplicity 1."""
    if E < 1 or p < 1:
        raise ValueError("need E >= 1 and p >= 1")
    inner = np.arange(1, E, dtype=np.float64) / E
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


def jittered_knots(E: int, p: int, seed: int, jitter: float = 0.3) -> np.ndarray:
    """Open knot vector with E elements of random (positive) lengths."""
    rng = np.random.default_rng(seed)
    h = 1.0 + jitter * (2.0 * rng.random(E) - 1.0)
    inner = np.cumsum(h)[:-1] / h.sum()
    return np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])


# --------------------------------------------------------------------------
# random parameters of maps / coefficients
# --------------------------------------------------------------------------


def warped_geometry(seed: int, dim: int = 3, modes: int = 8, amp: float = 0.1) -> dict:
    """Smooth displacement of the unit cube with `modes` seeded sine modes.

    c_k ~ N(0, I_d), m_kl ~ U{1, 2}; a = amp / sum_k |c_k| so that |F - xi| <= amp.
    """
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((modes, dim))
    m = rng.integers(1, 3, size=(modes, dim))
    a = amp / float(np.linalg.norm(c, axis=1).sum())
    return {"kind": "warped", "amp": a, "c": c, "m": m}


def sincos_coefficient(amp=0.5, f1=1, f2=1, phi1=0.0, phi2=0.0) -> dict:
    return {"kind": "sincos", "amp": float(amp), "f1": float(f1), "f2": float(f2),
            "phi1": float(phi1), "phi2": float(phi2)}


def random_coefficient(rng: np.random.Generator) -> dict:
    return sincos_coefficient(amp=rng.uniform(0.0, 0.5), f1=rng.integers(1, 3), f2=rng.integers(1, 3),
                              phi1=rng.uniform(0.0, 2 * np.pi), phi2=rng.uniform(0.0, 2 * np.pi))


def make_problem(dim, degree, knots, geometry=None, coefficient=None, quad=None) -> dict:
    if len(knots) != dim:
        raise ValueError("one knot vector per direction")
    return {
        "dim": int(dim),
        "degree": int(degree),
        "knots": [np.asarray(k, dtype=np.float64) for k in knots],
        "geometry": geometry or {"kind": "identity"},
        "coefficient": coefficient or {"kind": "one"},
        "quad": int(quad if quad is not None else degree + 1),
    }


def uniform_problem(dim, E, p, geometry=None, coefficient=None, quad=None) -> dict:
    Es = E if isinstance(E, (list, tuple)) else [E] * dim
    return make_problem(dim, p, [uniform_knots(e, p) for e in Es], geometry, coefficient, quad)


# --------------------------------------------------------------------------
# right-hand sides and random vectors
# --------------------------------------------------------------------------

RHS_SINPROD = {"kind": "sinprod"}        # f = d pi^2 prod sin(pi x_i)  (u = prod sin(pi x_i))
RHS_PAPER_POLY = {"kind": "paper_poly"}  # f = 2 sum (x_i^2 - x_i)      (paper Sec. 7)
RHS_BUBBLE = {"kind": "bubble"}          # f = 2 sum_i prod_{l!=i} x_l(1-x_l)  (u = prod x_l(1-x_l))


def random_vector(shape, seed: int) -> np.ndarray:
    """Seeded N(0,1) vector (mirrors b = randn on the cube, paper Sec. 7.2)."""
    return np.random.default_rng(seed).standard_normal(shape)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------


def square_2d(E: int = 64, p: int = 3) -> dict:
    """2D unit square, identity map, K = I (P = A)."""
    return uniform_problem(2, E, p)


def unit_cube(E: int = 512, p: int = 3) -> dict:
    """3D unit cube, identity map, K = I: P = A, so the FD apply is the direct
    solver (the paper's Table cube, h^-1 = E, right-hand side randn)."""
    return uniform_problem(3, E, p)


def thick_ring(E: int = 128, p: int = 3) -> dict:
    """3D thick quarter ring, K = I."""
    return uniform_problem(3, E, p, geometry={"kind": "ring"})


def warped_cube(E: int = 96, p: int = 5, seed: int = 3, coefficient=None) -> dict:
    """Unit cube warped by 8 seeded sine modes of amplitude 0.1; kappa in A only."""
    coef = coefficient if coefficient is not None else sincos_coefficient(0.5, 1, 1, 0.0, 0.0)
    return uniform_problem(3, E, p, geometry=warped_geometry(seed), coefficient=coef)


def quarter_annulus_2d(E=(8, 8), p: int = 2) -> dict:
    return uniform_problem(2, list(E), p, geometry={"kind": "ring"})


def band_bytes(n, p) -> int:
    """FP64 bytes of the exact nonzeros of A: prod_d (n_d(2p+1) - p(p+1)) * 8."""
    nnz = 1
    for nd in n:
        nnz *= max(nd * (2 * p + 1) - p * (p + 1), 0)
    return 8 * nnz


def batch_problems(seed: int = 4, count: int = 64, budget_bytes: float = 200e9):
    """Batch of uneven 3D problems: m_d ~ U{32..96} per direction, p ~ U{2..5},
    map ~ {thick ring, warped cube (seed 1000+k)}.  Redrawn until the summed
    size of the A matrices stays below `budget_bytes`."""
    rng = np.random.default_rng(seed)
    while True:
        probs = []
        total = 0
        for k in range(count):
            m = rng.integers(32, 97, size=3)
            p = int(rng.integers(2, 6))
            kind = "ring" if rng.random() < 0.5 else "warped"
            Es = [int(mm) - p for mm in m]
            geom = {"kind": "ring"} if kind == "ring" else warped_geometry(1000 + k)
            probs.append(uniform_problem(3, Es, p, geometry=geom))
            total += band_bytes([e + p - 2 for e in Es], p)
        if total <= budget_bytes:
            return probs


def training_problem(seed: int) -> dict:
    """One learned-scaling training instance: warped cube with a random kappa."""
    rng = np.random.default_rng(100000 + seed)
    p = int(rng.integers(2, 6))
    E = int(rng.integers(8, 25))
    return uniform_problem(3, E, p, geometry=warped_geometry(seed), coefficient=random_coefficient(rng))


def learned_eval_problem(E: int = 112, p: int = 4) -> dict:
    return warped_cube(E=E, p=p, seed=10000)
