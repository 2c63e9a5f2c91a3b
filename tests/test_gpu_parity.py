"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances:

* A x, b, diag A: FP64 with a different summation order; the bound is a
  small multiple of eps times sum |a_ij x_j| per row -> 1e-12 relative.
* P^-1 r in FP64: rounding of six dense mode products of length n <= 130,
  amplified by cond(U) ~ sqrt(cond(M)) -> 1e-11 relative.
* P^-1 r in FP32 (unit roundoff 6e-8) -> 1e-4; BF16 inputs (unit roundoff
  3.9e-3, FP32 accumulation) -> 5e-2 relative in the 2-norm.
* Solutions at rtol = 1e-8: |u_gpu - u_oracle| / |u_oracle| <= 1e-7 with
  iteration counts within one (the stated target of this path).
"""
import numpy as np
import pytest

import synth
from helpers import rel, small_problems, to_dev, to_host
from oracle import assembly, fd, pcg

pytestmark = pytest.mark.gpu

PROBLEMS = small_problems()
IDS = [p[0] for p in PROBLEMS]


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


_cache = {}


def oracle_of(name, prob):
    if name not in _cache:
        A = assembly.assemble_matrix(prob)
        F = fd.setup(prob)
        _cache[name] = (A, F)
    return _cache[name]


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_apply_A_matches_oracle(api, name, prob, rng):
    A, F = oracle_of(name, prob)
    with api.igafd_setup(prob) as ctx:
        assert ctx.N == A.shape[0]
        x = rng.standard_normal(ctx.N)
        y = to_dev(np.zeros(ctx.N))
        api.igafd_apply_A(ctx, to_dev(x), y)
        yg = to_host(y)
        ref = A @ x
        scale = abs(A) @ np.abs(x)
        assert np.max(np.abs(yg - ref) / scale) < 1e-12
        dA = to_dev(np.zeros(ctx.N))
        dP = to_dev(np.zeros(ctx.N))
        api.igafd_diagonals(ctx, dA, dP)
        np.testing.assert_allclose(to_host(dA), A.diagonal(), rtol=1e-12)
        np.testing.assert_allclose(to_host(dP), fd.diag_P(F), rtol=1e-12)


TILE_CASES = [
    # (problem, tile shape "b2xb3[xthreads]" or "0" for the row-parallel kernel)
    ("3d_warped_kappa_p3", "4x1"), ("3d_warped_kappa_p3", "2x2"), ("3d_warped_kappa_p3", "4x4"),
    ("3d_warped_kappa_p3", "0"), ("3d_ring_p2", "8x1"), ("3d_ring_p2", "2x6"), ("3d_identity_p1", "4x3"),
    ("3d_warped_p5", "2x2"), ("3d_warped_p5", "0"), ("long_n1_p3", "4x4"), ("long_n1_p3", "0"),
    # 512 threads per block (one block per CU, larger tiles)
    ("3d_warped_kappa_p3", "4x4x512"), ("3d_ring_p2", "2x6x512"), ("3d_warped_p5", "2x2x512"),
    ("long_n1_p3", "4x4x512"),
    # the combine's unrolled forms: at most 2x2 (identity 4x3), 2x3, 3x3 (ring 8x1) and 2x6
    # (p = 5, 2x5) covering tiles per row; the loop for the others
    ("3d_warped_p5", "2x5x512"),
]


def _tile_problem(name):
    if name == "long_n1_p3":  # n1 = 129: 9 row chunks per lane, LDS tile above 64 KB
        return synth.uniform_problem(3, [128, 6, 7], 3, geometry=synth.warped_geometry(8))
    return dict(PROBLEMS)[name]


@pytest.mark.parametrize("name,tile", TILE_CASES, ids=[f"{n}-{t}" for n, t in TILE_CASES])
def test_apply_A_kernel_shapes(api, name, tile, rng, monkeypatch):
    # every A-product kernel and tile shape against the oracle's assembled A
    prob = _tile_problem(name)
    A, _ = oracle_of(name, prob)
    monkeypatch.setenv("IGAFD_SPMV_TILE", tile)
    with api.igafd_setup(prob) as ctx:
        x = rng.standard_normal(ctx.N)
        y = to_dev(np.zeros(ctx.N))
        if "x" in tile:
            shape = api.igafd_get_shape(ctx)
            want = [int(v) for v in tile.split("x")] + [256]
            assert (shape["tile_b2"], shape["tile_b3"], shape["tile_threads"]) == tuple(want[:3])
        api.igafd_apply_A(ctx, to_dev(x), y)
        scale = abs(A) @ np.abs(x)
        assert np.max(np.abs(to_host(y) - A @ x) / scale) < 1e-12


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_spectral_bounds_match_oracle(api, name, prob):
    # Prop. 1 bounds: extreme eigenvalues of Q over all Gauss points (closed
    # form on the device, eigvalsh in the oracle)
    lo, hi = assembly.q_spectral_bounds(prob)
    with api.igafd_setup(prob) as ctx:
        glo, ghi = api.igafd_spectral_bounds(ctx)
    assert abs(glo - lo) <= 1e-12 * abs(lo) and abs(ghi - hi) <= 1e-12 * abs(hi)


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_load_vector_matches_oracle(api, name, prob):
    with api.igafd_setup(prob) as ctx:
        for rhs in (synth.RHS_SINPROD, synth.RHS_PAPER_POLY, synth.RHS_BUBBLE):
            b = to_dev(np.zeros(ctx.N))
            api.igafd_load_vector(ctx, rhs, b)
            ref = assembly.assemble_load(prob, rhs)
            assert rel(to_host(b), ref) < 1e-13


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_precond_matches_oracle(api, name, prob, rng):
    _, F = oracle_of(name, prob)
    with api.igafd_setup(prob) as ctx:
        r = rng.standard_normal(ctx.N)
        ref = fd.fd_apply(F, r)
        s = to_dev(np.zeros(ctx.N))
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16", 5e-2)):
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            err = rel(to_host(s), ref)
            assert err < tol, (prec, err)


def test_precond_ragged_row_tiles(api, rng, monkeypatch):
    # n2 = 65, n3 = 66: the last MFMA row tile of those directions holds one or
    # two rows; applies against the oracle (also scaled) and the solve against
    # the six separate mode products
    prob = synth.uniform_problem(3, [10, 64, 65], 3, geometry=synth.warped_geometry(6),
                                 coefficient=synth.sincos_coefficient(0.3, 1, 1, 0.2, 0.4))
    F = fd.setup(prob)
    with api.igafd_setup(prob) as ctx:
        assert tuple(ctx.n[:3]) == (11, 65, 66) and api.igafd_get_shape(ctx)["fd_fused"] == 1
        r = rng.standard_normal(ctx.N)
        ref = fd.fd_apply(F, r)
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16", 5e-2)):
            s = to_dev(np.zeros(ctx.N))
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            assert rel(to_host(s), ref) < tol, prec
        S = np.exp(0.1 * rng.standard_normal(ctx.N))
        api.igafd_set_scaling(ctx, to_dev(S))
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(r), s)
        assert rel(to_host(s), S * fd.fd_apply(F, S * r)) < 1e-11
        api.igafd_set_scaling(ctx, None)
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, b, u)
    # the same solve with the six separate mode products
    monkeypatch.setenv("IGAFD_FD_FUSED", "0")
    with api.igafd_setup(prob) as ctx6:
        assert api.igafd_get_shape(ctx6)["fd_fused"] == 0
        u6 = to_dev(np.zeros(ctx6.N))
        info6 = api.igafd_solve(ctx6, b, u6)
    assert info["iters"] == info6["iters"] and rel(to_host(u), to_host(u6)) < 1e-10


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_solve_matches_oracle(api, name, prob):
    A, F = oracle_of(name, prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.pcg(lambda v: A @ v, lambda r: fd.fd_apply(F, r), b, rtol=1e-8)
    with api.igafd_setup(prob) as ctx:
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, rtol=1e-8, history=True)
        assert info["status"] == "OK"
        assert abs(info["iters"] - info_or["iters"]) <= 1
        assert info["true_relres"] <= 1e-8
        assert rel(to_host(u), u_or) <= 1e-7
        np.testing.assert_allclose(info["history"][: len(info_or["history"])][:5], info_or["history"][:5],
                                   rtol=1e-6, atol=1e-12)


def test_identity_map_converges_in_one_iteration(api):
    # P = A on the unit square (Sec. 3): CG with the exact inverse needs one step
    prob = synth.square_2d(E=24, p=3)
    with api.igafd_setup(prob) as ctx:
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, b, u)
        assert info["iters"] == 1 and info["true_relres"] < 1e-12


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_mixed_precision_flexible_solve(api, prec):
    # parity unpinned (no exact value for an inexact preconditioner): judged by
    # the FP64 true residual and the distance to the FP64 oracle solution
    prob = synth.uniform_problem(3, [10, 8, 12], 3, geometry=synth.warped_geometry(3),
                                 coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.0, 0.0))
    A, F = oracle_of("3d_warped_kappa_p3", prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.pcg(lambda v: A @ v, lambda r: fd.fd_apply(F, r), b, rtol=1e-8)
    with api.igafd_setup(prob) as ctx:
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, precision=prec)
        assert info["true_relres"] <= 1e-8
        assert info["iters"] <= info_or["iters"] + 3
        assert rel(to_host(u), u_or) <= 1e-6


def test_flexible_fp64_equals_standard(api):
    prob = synth.thick_ring(E=12, p=3)
    with api.igafd_setup(prob) as ctx:
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u1, u2 = to_dev(np.zeros(ctx.N)), to_dev(np.zeros(ctx.N))
        i1 = api.igafd_solve(ctx, b, u1, flexible=False)
        i2 = api.igafd_solve(ctx, b, u2, flexible=True)
        assert i1["iters"] == i2["iters"]
        assert rel(to_host(u2), to_host(u1)) < 1e-9


def test_bitwise_reproducible(api):
    prob = synth.warped_cube(E=9, p=3, seed=3)
    with api.igafd_setup(prob) as ctx:
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        us = []
        for _ in range(2):
            u = to_dev(np.zeros(ctx.N))
            api.igafd_solve(ctx, b, u)
            us.append(to_host(u))
        assert np.array_equal(us[0], us[1])


def test_scaling_identity_is_plain(api, rng):
    prob = synth.thick_ring(E=10, p=2)
    _, F = oracle_of("ring10p2", prob)
    with api.igafd_setup(prob) as ctx:
        r = to_dev(rng.standard_normal(ctx.N))
        s0, s1 = to_dev(np.zeros(ctx.N)), to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", r, s0)
        api.igafd_set_scaling(ctx, to_dev(np.ones(ctx.N)))
        api.igafd_apply_precond(ctx, "fp64", r, s1)
        assert np.array_equal(to_host(s0), to_host(s1))
        S = rng.uniform(0.5, 2.0, ctx.N)
        api.igafd_set_scaling(ctx, to_dev(S))
        api.igafd_apply_precond(ctx, "fp64", r, s1)
        ref = fd.fd_apply(F, to_host(r), scaling=S)
        assert rel(to_host(s1), ref) < 1e-11
        api.igafd_set_scaling(ctx, None)


def test_edge_cases(api):
    from paper_1602_01636_amd import IgafdError
    # one dof per direction, and a degree larger than the element count
    for prob in (synth.uniform_problem(3, 2, 1), synth.uniform_problem(2, 1, 3), synth.uniform_problem(3, [1, 2, 3], 3)):
        A = assembly.assemble_matrix(prob)
        F = fd.setup(prob)
        b = assembly.assemble_load(prob, synth.RHS_SINPROD)
        with api.igafd_setup(prob) as ctx:
            assert ctx.N == A.shape[0]
            y = to_dev(np.zeros(ctx.N))
            x = np.linspace(1, 2, ctx.N)
            api.igafd_apply_A(ctx, to_dev(x), y)
            assert rel(to_host(y), A @ x) < 1e-13
            s = to_dev(np.zeros(ctx.N))
            api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
            assert rel(to_host(s), fd.fd_apply(F, x)) < 1e-12
            u = to_dev(np.zeros(ctx.N))
            info = api.igafd_solve(ctx, to_dev(b), u)
            assert info["true_relres"] <= 1e-8
    prob = synth.thick_ring(E=6, p=2)
    with api.igafd_setup(prob) as ctx:
        # zero right-hand side: zero iterations, zero solution
        u = to_dev(np.ones(ctx.N))
        info = api.igafd_solve(ctx, to_dev(np.zeros(ctx.N)), u)
        assert info["iters"] == 0 and np.all(to_host(u) == 0)
        # iteration cap
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        info = api.igafd_solve(ctx, b, u, maxit=2)
        assert info["status"] == "NOT_CONVERGED" and info["iters"] == 2
        # NaN in the right-hand side -> breakdown reported, no hang
        bn = to_host(b).copy()
        bn[3] = np.nan
        with pytest.raises(IgafdError):
            api.igafd_solve(ctx, to_dev(bn), u)
        # mixed precision without the flexible form is rejected
        with pytest.raises(IgafdError):
            api.igafd_solve(ctx, b, u, precision="bf16", flexible=False)
    # folded map: det J <= 0 at a Gauss point
    g = {"kind": "warped", "amp": 2.0, "c": np.array([[1.0, 1.0, 1.0]]), "m": np.array([[1, 1, 1]])}
    with pytest.raises(IgafdError):
        api.igafd_setup(synth.uniform_problem(3, 3, 1, geometry=g))
    with pytest.raises(IgafdError):
        api.igafd_setup(synth.make_problem(3, 2, [synth.uniform_knots(3, 2)] * 3, quad=5))


GEMM_2D = [
    ("2d_ragged_p3", synth.uniform_problem(2, [37, 70], 3, geometry=synth.warped_geometry(4, dim=2),
                                           coefficient=synth.sincos_coefficient(0.3, 1, 2, 0.1, 0.2))),
    ("2d_jittered_p5", synth.make_problem(2, 5, [synth.jittered_knots(150, 5, 3), synth.jittered_knots(21, 5, 4)])),
    ("2d_annulus_p1", synth.uniform_problem(2, [130, 129], 1, geometry={"kind": "ring"})),
]


@pytest.mark.parametrize("name,prob", GEMM_2D, ids=[g[0] for g in GEMM_2D])
def test_2d_tiled_products(api, name, prob, rng, monkeypatch):
    """The 2D apply by tiled products (forced on at sizes whose tiles are all
    ragged): applies against the oracle, plain and scaled, and the solve
    (whose (r, s) partials come from the last product's epilogue) against
    the per-strip products."""
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    monkeypatch.setenv("IGAFD_FD_GEMM", "1")
    with api.igafd_setup(prob) as ctx:
        r = rng.standard_normal(ctx.N)
        ref = fd.fd_apply(F, r)
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16", 5e-2)):
            s = to_dev(np.full(ctx.N, 3.0))
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            assert rel(to_host(s), ref) < tol, prec
        S = np.exp(0.1 * rng.standard_normal(ctx.N))
        api.igafd_set_scaling(ctx, to_dev(S))
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(r), s)
        assert rel(to_host(s), S * fd.fd_apply(F, S * r)) < 1e-11
        u = to_dev(np.zeros(ctx.N))
        info_s = api.igafd_solve(ctx, to_dev(A @ r), u, use_scaling=True)
        assert info_s["true_relres"] <= 1e-8
        api.igafd_set_scaling(ctx, None)
        b = A @ rng.standard_normal(ctx.N)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u)
        u32 = to_dev(np.zeros(ctx.N))
        info32 = api.igafd_solve(ctx, to_dev(b), u32, precision="fp32")
    assert info["true_relres"] <= 1e-8 and info32["true_relres"] <= 1e-8
    monkeypatch.setenv("IGAFD_FD_GEMM", "0")
    with api.igafd_setup(prob) as ctx0:
        u0 = to_dev(np.zeros(ctx0.N))
        info0 = api.igafd_solve(ctx0, to_dev(b), u0)
    assert info["iters"] == info0["iters"] and rel(to_host(u), to_host(u0)) < 1e-10
