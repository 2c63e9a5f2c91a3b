"""Thin ctypes binding of the C ABI declared in include/igafd.h.

Argument marshalling only: every step of the solver runs in libigafd.so.
Functions keep the C names.  Vectors are torch float64 CUDA tensors,
contiguous, N = prod(n) elements laid out as [n3][n2][n1] (direction 1
fastest).  Calls are ordered on the stream passed to igafd_setup (default: the
current torch stream).  A non-OK status raises IgafdError with the library's
message; there is no fallback when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigafd.so")

IGAFD_OK, IGAFD_NOT_CONVERGED = 0, 1
IGAFD_FP64, IGAFD_FP32, IGAFD_BF16, IGAFD_BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": IGAFD_FP64, "fp32": IGAFD_FP32, "bf16": IGAFD_BF16, "bf16x3": IGAFD_BF16X3}
GEOM_KINDS = {"identity": 0, "ring": 1, "warped": 2}
COEF_KINDS = {"one": 0, "sincos": 1}
RHS_KINDS = {"sinprod": 0, "paper_poly": 1, "bubble": 2, "one": 3}
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_ALLOC", -3: "ERR_HIP",
                -4: "ERR_GEOMETRY", -5: "ERR_NOT_SPD", -6: "ERR_BREAKDOWN"}


class IgafdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class igafd_problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("degree", C.c_int), ("nknots", C.c_int * 3),
                ("knots", C.POINTER(C.c_double) * 3), ("geom_kind", C.c_int), ("n_geom_params", C.c_int),
                ("geom_params", C.POINTER(C.c_double)), ("coef_kind", C.c_int), ("n_coef_params", C.c_int),
                ("coef_params", C.POINTER(C.c_double)), ("quad_per_dir", C.c_int), ("want_features", C.c_int)]


class igafd_solve_opts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int), ("precision", C.c_int), ("flexible", C.c_int),
                ("use_scaling", C.c_int), ("check_every", C.c_int), ("use_x0", C.c_int),
                ("history", C.POINTER(C.c_double)), ("timers", C.c_int)]


class igafd_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("relres", C.c_double), ("true_relres", C.c_double),
                ("status", C.c_int), ("t_solve_ms", C.c_double), ("fallback", C.c_int), ("history_len", C.c_int),
                ("t_setup_ms", C.c_double), ("t_spmv_ms", C.c_double), ("t_fd_ms", C.c_double),
                ("t_vec_ms", C.c_double), ("scaled", C.c_int), ("kappa_bound", C.c_double)]


SCALING_MODES = {False: 0, True: 1, "auto": 2, 0: 0, 1: 1, 2: 2}


def _info_dict(info, st):
    return {"iters": info.iters, "restarts": info.restarts, "relres": info.relres,
            "true_relres": info.true_relres, "status": STATUS_NAMES.get(st, st), "t_solve_ms": info.t_solve_ms,
            "fallback": bool(info.fallback), "history_len": info.history_len, "t_setup_ms": info.t_setup_ms,
            "t_spmv_ms": info.t_spmv_ms, "t_fd_ms": info.t_fd_ms, "t_vec_ms": info.t_vec_ms,
            "scaled": bool(info.scaled), "kappa_bound": info.kappa_bound}


_lib = None

_SIGNATURES = {
    "igafd_setup": (C.c_int, [C.POINTER(igafd_problem), C.c_void_p, C.POINTER(C.c_void_p)]),
    "igafd_sizes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                              C.POINTER(C.c_longlong)]),
    "igafd_load_vector": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_void_p]),
    "igafd_apply_A": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "igafd_apply_precond": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "igafd_set_scaling": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(igafd_solve_opts),
                              C.POINTER(igafd_solve_info)]),
    "igafd_diagonals": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "igafd_get_eigen": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "igafd_univariate": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.POINTER(C.c_int)]),
    "igafd_destroy": (None, [C.c_void_p]),
    "igafd_last_error": (C.c_char_p, []),
    "igafd_features": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_features_noalloc": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_solve_batched": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.POINTER(igafd_solve_opts),
                                      C.c_void_p, C.POINTER(C.c_double)]),
    "igafd_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "igafd_get_shape": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_int)] * 6),
    "igafd_spectral_bounds": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]),
    "igafd_scaling_gate": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]),
    "igafd_setup_precond": (C.c_int, [C.POINTER(igafd_problem), C.c_void_p, C.POINTER(C.c_void_p)]),
    "igafd_lshape_setup": (C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_void_p)]),
    "igafd_set_adi": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "igafd_set_adi_greedy": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "igafd_get_adi": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double),
                                C.c_void_p, C.c_int]),
    "igafd_lshape_corner": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_longlong)]),
    "igafd_scaling_targets": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_set_scaling_diag_ratio": (C.c_int, [C.c_void_p]),
    "igafd_mlp_num_params": (C.c_int, []),
    "igafd_mlp_create": (C.c_int, [C.c_ulonglong, C.c_void_p, C.POINTER(C.c_void_p)]),
    "igafd_mlp_destroy": (None, [C.c_void_p]),
    "igafd_mlp_fit_normalization": (C.c_int, [C.c_void_p, C.c_void_p, C.c_longlong]),
    "igafd_mlp_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_mlp_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "igafd_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p]),
    "igafd_mlp_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p]),
    "igafd_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_longlong, C.c_float, C.c_void_p]),
}


def lib():
    """Load libigafd.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch ships its own HIP runtime (same soname).  Loading torch first makes
        # the library bind to that runtime instead of pulling a second copy into
        # the process, so both see the same device, streams and allocations.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def igafd_last_error() -> str:
    return lib().igafd_last_error().decode()


def _check(status):
    if status < 0:
        raise IgafdError(status, igafd_last_error())
    return status


def _dptr(t, N=None, name="vector"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if N is not None and t.numel() != N:
        raise ValueError(f"{name} has {t.numel()} elements, expected {N}")
    return C.c_void_p(t.data_ptr())


def _fptr(t, n=None, name="array", cols=1):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    if n is not None and t.numel() != n * cols:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n * cols}")
    return C.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def geometry_params(geom: dict, dim: int):
    kind = GEOM_KINDS[geom["kind"]]
    if geom["kind"] != "warped":
        return kind, []
    c = np.asarray(geom["c"], float).reshape(-1, dim)
    m = np.asarray(geom["m"], float).reshape(-1, dim)
    return kind, [float(geom["amp"]), float(len(c))] + list(c.reshape(-1)) + list(m.reshape(-1))


def coefficient_params(coef: dict):
    kind = COEF_KINDS[coef["kind"]]
    if coef["kind"] == "one":
        return kind, []
    return kind, [coef["amp"], coef["f1"], coef["f2"], coef["phi1"], coef["phi2"]]


class Context:
    """Owner of an igafd_ctx handle; `handle` is passed to the igafd_* calls."""

    def __init__(self, handle, n, N, nnz, band_bytes, dim, degree=None):
        self.handle = handle
        self.n = n
        self.N = N
        self.nnz = nnz
        self.band_bytes = band_bytes
        self.dim = dim
        self.p = degree

    @property
    def shape(self):
        return tuple(self.n[: self.dim][::-1])

    def close(self):
        if self.handle:
            lib().igafd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def igafd_setup(problem: dict, stream=None, features=False) -> Context:
    """Setup of one problem (host 1D setup + device assembly); features=True
    also assembles the learned scaling's per-dof inputs."""
    return _setup(problem, stream, "igafd_setup", features)


def igafd_setup_precond(problem: dict, stream=None) -> Context:
    """Preconditioner-only setup (no A): on the unit square / cube P = A, so
    igafd_apply_precond is the fast-diagonalisation direct solver."""
    return _setup(problem, stream, "igafd_setup_precond")


def _setup(problem: dict, stream, entry: str, features=False) -> Context:
    d = int(problem["dim"])
    pr = igafd_problem()
    pr.dim = d
    pr.degree = int(problem["degree"])
    keep = []
    for l in range(3):
        if l < d:
            k = np.ascontiguousarray(problem["knots"][l], dtype=np.float64)
            keep.append(k)
            pr.nknots[l] = len(k)
            pr.knots[l] = k.ctypes.data_as(C.POINTER(C.c_double))
        else:
            pr.nknots[l] = 0
    gk, gp = geometry_params(problem["geometry"], d)
    ck, cp = coefficient_params(problem["coefficient"])
    gpa = (C.c_double * max(1, len(gp)))(*gp)
    cpa = (C.c_double * max(1, len(cp)))(*cp)
    pr.geom_kind, pr.n_geom_params, pr.geom_params = gk, len(gp), gpa
    pr.coef_kind, pr.n_coef_params, pr.coef_params = ck, len(cp), cpa
    pr.quad_per_dir = int(problem.get("quad", 0) or 0)
    pr.want_features = int(bool(features))
    h = C.c_void_p()
    _check(getattr(lib(), entry)(C.byref(pr), stream if stream is not None else _current_stream(), C.byref(h)))
    n, N, nnz, bb = igafd_sizes(h)
    return Context(h, n, N, nnz, bb, d, pr.degree)


def igafd_lshape_setup(knots, degree: int, stream=None) -> Context:
    """L-shaped three-patch problem (C^0 interfaces) with the additive Schwarz
    preconditioner P_IAS; every patch carries `knots` in both directions.
    Vectors have the bounding square's N = n^2 entries; `ctx.hole` is the first
    index of the entries that are not unknowns, `ctx.ndofs` the unknowns."""
    k = np.ascontiguousarray(knots, dtype=np.float64)
    h = C.c_void_p()
    _check(lib().igafd_lshape_setup(int(degree), len(k), k.ctypes.data_as(C.POINTER(C.c_double)),
                                    stream if stream is not None else _current_stream(), C.byref(h)))
    n, N, nnz, bb = igafd_sizes(h)
    ctx = Context(h, n, N, nnz, bb, 2, int(degree))
    ctx.hole, ctx.ndofs = igafd_lshape_corner(ctx)
    return ctx


def igafd_set_adi(ctx, eps):
    """Switch the preconditioner to J steps of the three-variable ADI with
    ||T_J|| <= eps (eps = 0: back to FD).  Returns (J, rho)."""
    J, rho = C.c_int(), C.c_double()
    _check(lib().igafd_set_adi(_h(ctx), float(eps), C.byref(J), C.byref(rho)))
    return J.value, rho.value


def igafd_set_adi_greedy(ctx, eps):
    """As igafd_set_adi with the greedy parameters (eq. greedy1/2).  Returns (J, rho)."""
    J, rho = C.c_int(), C.c_double()
    _check(lib().igafd_set_adi_greedy(_h(ctx), float(eps), C.byref(J), C.byref(rho)))
    return J.value, rho.value


def igafd_get_adi(ctx) -> dict:
    """{"J", "J0", "rho", "omegas"} of the ADI preconditioner (J = 0: off)."""
    J, J0, rho = C.c_int(), C.c_int(), C.c_double()
    _check(lib().igafd_get_adi(_h(ctx), C.byref(J), C.byref(J0), C.byref(rho), None, 0))
    om = np.zeros(max(J.value, 1))
    _check(lib().igafd_get_adi(_h(ctx), None, None, None, om.ctypes.data_as(C.c_void_p), len(om)))
    return {"J": J.value, "J0": J0.value, "rho": rho.value, "omegas": om[: J.value].copy()}


def igafd_lshape_corner(ctx):
    """(hole, ndofs): hole = -1 and ndofs = N for a single-patch context."""
    hole, nd = C.c_int(), C.c_longlong()
    _check(lib().igafd_lshape_corner(_h(ctx), C.byref(hole), C.byref(nd)))
    return hole.value, nd.value


def _h(ctx):
    return ctx.handle if isinstance(ctx, Context) else ctx


def igafd_sizes(ctx):
    n = (C.c_int * 3)()
    N, nnz, bb = C.c_longlong(), C.c_longlong(), C.c_longlong()
    _check(lib().igafd_sizes(_h(ctx), n, C.byref(N), C.byref(nnz), C.byref(bb)))
    return list(n), N.value, nnz.value, bb.value


def rhs_params(rhs: dict, dim: int):
    """Parameter array of a right-hand side dict (empty: the library's defaults)."""
    if rhs.get("kind") == "sinprod":
        if "amp" not in rhs and "k" not in rhs:
            return []
        k = list(rhs.get("k", [1.0] * dim))  # the library checks the count
        return [float(rhs.get("amp", dim * np.pi ** 2))] + [float(v) for v in k]
    return [float(rhs["amp"])] if "amp" in rhs else []


def igafd_load_vector(ctx: Context, rhs, b):
    if isinstance(rhs, dict):
        kind, prm = RHS_KINDS[rhs["kind"]], rhs_params(rhs, ctx.dim)
    else:
        kind, prm = int(rhs), []
    arr = (C.c_double * max(1, len(prm)))(*prm)
    _check(lib().igafd_load_vector(_h(ctx), kind, arr if prm else None, len(prm), _dptr(b, ctx.N, "b")))


def igafd_apply_A(ctx: Context, x, y):
    _check(lib().igafd_apply_A(_h(ctx), _dptr(x, ctx.N, "x"), _dptr(y, ctx.N, "y")))


def igafd_apply_precond(ctx: Context, precision, r, s):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().igafd_apply_precond(_h(ctx), prec, _dptr(r, ctx.N, "r"), _dptr(s, ctx.N, "s")))


def igafd_set_scaling(ctx: Context, S):
    _check(lib().igafd_set_scaling(_h(ctx), None if S is None else _dptr(S, ctx.N, "S")))


def igafd_diagonals(ctx: Context, dA=None, dP=None):
    _check(lib().igafd_diagonals(_h(ctx), None if dA is None else _dptr(dA, ctx.N, "diagA"),
                                 None if dP is None else _dptr(dP, ctx.N, "diagP")))


def igafd_solve(ctx: Context, b, u, rtol=1e-8, maxit=2000, precision="fp64", flexible=None,
                use_scaling=False, check_every=4, x0=False, history=False, timers=False) -> dict:
    """use_scaling: False / True / "auto" (the Prop. 1 gate decides)."""
    o = _opts(rtol, maxit, precision, flexible, use_scaling, check_every, x0)
    o.timers = int(bool(timers))
    hist = None
    if history:
        hist = np.zeros(int(maxit) + 1)
        o.history = hist.ctypes.data_as(C.POINTER(C.c_double))
    info = igafd_solve_info()
    st = _check(lib().igafd_solve(_h(ctx), _dptr(b, ctx.N, "b"), _dptr(u, ctx.N, "u"), C.byref(o), C.byref(info)))
    out = _info_dict(info, st)
    if hist is not None:
        out["history"] = hist[: info.history_len].copy()
    return out


def _opts(rtol, maxit, precision, flexible, use_scaling, check_every, x0):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if flexible is None:
        flexible = prec != IGAFD_FP64
    o = igafd_solve_opts()
    o.rtol, o.maxit, o.precision, o.flexible = float(rtol), int(maxit), prec, int(bool(flexible))
    o.use_scaling, o.check_every, o.use_x0 = SCALING_MODES[use_scaling], int(check_every), int(bool(x0))
    return o


def igafd_solve_batched(ctxs, bs, us, rtol=1e-8, maxit=2000, precision="fp64", flexible=None, use_scaling=False,
                        check_every=4):
    """Solve len(ctxs) independent problems together; returns (infos, wall_ms)."""
    n = len(ctxs)
    if not (len(bs) == len(us) == n) or n == 0:
        raise ValueError("need one b and one u per context")
    H = (C.c_void_p * n)(*[_h(c) for c in ctxs])
    Bp = (C.c_void_p * n)(*[_dptr(b, c.N, "b").value for b, c in zip(bs, ctxs)])
    Up = (C.c_void_p * n)(*[_dptr(u, c.N, "u").value for u, c in zip(us, ctxs)])
    infos = (igafd_solve_info * n)()
    wall = C.c_double()
    o = _opts(rtol, maxit, precision, flexible, use_scaling, check_every, False)
    _check(lib().igafd_solve_batched(H, n, Bp, Up, C.byref(o), infos, C.byref(wall)))
    out = [_info_dict(i, i.status) for i in infos]
    return out, wall.value


def igafd_autotune(ctx: Context, fd_tiles=0, spmv_rows=0):
    """Kernel shape of one problem (0, 0: time the candidates and keep the fastest)."""
    _check(lib().igafd_autotune(_h(ctx), int(fd_tiles), int(spmv_rows)))


def igafd_spectral_bounds(ctx: Context, local=False):
    """(qmin, qmax): every eigenvalue of P^-1 A lies in [qmin, qmax] (Prop. 1);
    with local=True also qloc, the largest pointwise ratio of Q's eigenvalues."""
    lo, hi, loc = C.c_double(), C.c_double(), C.c_double()
    _check(lib().igafd_spectral_bounds(_h(ctx), C.byref(lo), C.byref(hi), C.byref(loc)))
    return (lo.value, hi.value, loc.value) if local else (lo.value, hi.value)


def igafd_scaling_gate(ctx: Context, gain=2.0):
    """(use, kappa_q, kappa_loc) of the scaled-preconditioner gate."""
    use, kq, kl = C.c_int(), C.c_double(), C.c_double()
    _check(lib().igafd_scaling_gate(_h(ctx), float(gain), C.byref(use), C.byref(kq), C.byref(kl)))
    return bool(use.value), kq.value, kl.value


def igafd_get_shape(ctx: Context) -> dict:
    """Kernel shape in use: {"spmv_rows", "tile_b2", "tile_b3", "fd_fused", "fd_tiles", "tile_threads"}."""
    v = [C.c_int() for _ in range(6)]
    _check(lib().igafd_get_shape(_h(ctx), *[C.byref(x) for x in v]))
    return dict(zip(("spmv_rows", "tile_b2", "tile_b3", "fd_fused", "fd_tiles", "tile_threads"),
                    [x.value for x in v]))


def igafd_get_eigen(ctx: Context, direction: int):
    n = ctx.n[direction]
    U = np.zeros((n, n))
    lam = np.zeros(n)
    _check(lib().igafd_get_eigen(_h(ctx), int(direction), U.ctypes.data_as(C.c_void_p),
                                 lam.ctypes.data_as(C.c_void_p)))
    return U, lam


def igafd_univariate(degree: int, knots, quad: int = 0):
    """Host-only 1D setup: (M, K, U, lam) for one knot vector."""
    k = np.ascontiguousarray(knots, dtype=np.float64)
    n = len(k) - degree - 3
    if n < 1:
        raise ValueError("no interior functions")
    M, K, U = (np.zeros((n, n)) for _ in range(3))
    lam = np.zeros(n)
    nout = C.c_int()
    _check(lib().igafd_univariate(int(degree), len(k), k.ctypes.data_as(C.POINTER(C.c_double)), int(quad),
                                  M.ctypes.data_as(C.c_void_p), K.ctypes.data_as(C.c_void_p),
                                  U.ctypes.data_as(C.c_void_p), lam.ctypes.data_as(C.c_void_p), C.byref(nout)))
    return M, K, U, lam


def igafd_destroy(ctx):
    if isinstance(ctx, Context):
        ctx.close()
    elif ctx:
        lib().igafd_destroy(ctx)


# ---------------- learned diagonal scaling ----------------

def igafd_features(ctx: Context, feat):
    """Per-dof network inputs into feat (float32, N x 8)."""
    _check(lib().igafd_features(_h(ctx), _fptr(feat, ctx.N, "feat", 8)))


def igafd_features_noalloc(ctx: Context, feat):
    """igafd_features without any device allocation (static accumulator, N <= 2^20)."""
    _check(lib().igafd_features_noalloc(_h(ctx), _fptr(feat, ctx.N, "feat", 8)))


def igafd_scaling_targets(ctx: Context, t):
    """t_i = 1/2 log(P_ii / A_ii) into t (float32, N)."""
    _check(lib().igafd_scaling_targets(_h(ctx), _fptr(t, ctx.N, "targets")))


def igafd_set_scaling_diag_ratio(ctx: Context):
    """Scaling S_i = (P_ii / A_ii)^(1/2) set on the context."""
    _check(lib().igafd_set_scaling_diag_ratio(_h(ctx)))


def igafd_mlp_num_params() -> int:
    return int(lib().igafd_mlp_num_params())


class Mlp:
    """Owner of an igafd_mlp handle."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            lib().igafd_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def igafd_mlp_create(seed=0, stream=None) -> Mlp:
    h = C.c_void_p()
    _check(lib().igafd_mlp_create(int(seed), stream if stream is not None else _current_stream(), C.byref(h)))
    return Mlp(h)


def igafd_mlp_destroy(m: Mlp):
    m.close()


def igafd_mlp_fit_normalization(m: Mlp, feat, n):
    _check(lib().igafd_mlp_fit_normalization(m.handle, _fptr(feat, n, "feat", 8), int(n)))


def igafd_mlp_get_params(m: Mlp) -> np.ndarray:
    out = np.zeros(igafd_mlp_num_params() + 16, dtype=np.float32)
    _check(lib().igafd_mlp_get_params(m.handle, out.ctypes.data_as(C.c_void_p)))
    return out


def igafd_mlp_set_params(m: Mlp, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    if a.size != igafd_mlp_num_params() + 16:
        raise ValueError("parameter array has the wrong length")
    _check(lib().igafd_mlp_set_params(m.handle, a.ctypes.data_as(C.c_void_p)))


def igafd_mlp_forward(m: Mlp, feat, n, t=None, S=None):
    tp = None if t is None else _fptr(t, n, "t")
    if S is not None:
        _dptr(S, n, "S")
    Sp = None if S is None else C.c_void_p(S.data_ptr())
    _check(lib().igafd_mlp_forward(m.handle, _fptr(feat, n, "feat", 8), int(n), tp, Sp))


def igafd_mlp_gradient(m: Mlp, feat, target, n):
    g = np.zeros(igafd_mlp_num_params(), dtype=np.float32)
    loss = np.zeros(1, dtype=np.float32)
    _check(lib().igafd_mlp_gradient(m.handle, _fptr(feat, n, "feat", 8), _fptr(target, n, "target"), int(n),
                                    g.ctypes.data_as(C.c_void_p), loss.ctypes.data_as(C.c_void_p)))
    return float(loss[0]), g


def igafd_mlp_train_step(m: Mlp, feat, target, n, lr, want_loss=False):
    loss = np.zeros(1, dtype=np.float32)
    _check(lib().igafd_mlp_train_step(m.handle, _fptr(feat, n, "feat", 8), _fptr(target, n, "target"), int(n),
                                      float(lr), loss.ctypes.data_as(C.c_void_p) if want_loss else None))
    return float(loss[0]) if want_loss else None
