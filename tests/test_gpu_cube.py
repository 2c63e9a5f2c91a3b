"""GPU parity of the 3D fast-diagonalisation apply by tiled MFMA products
(Sec. 5.1 Alg. 3, transposes as in Alg. 1) and of the preconditioner-only
context; full size: the FD direct solver on the unit cube (P = A, Sec. 3) at
the sizes of the paper's Table cube.

Tolerances as for the other FD applies: FP64 1e-11 relative to the oracle,
FP32 mode products 1e-4, BF16 inputs 5e-2.  On the cube the exact solution is
known: s* is drawn, r = P s* by the oracle's banded Kronecker-sum product, and
the GPU's P^-1 r must return s* (the oracle's own FD apply does so to 1e-14 at
h^-1 = 512).  Such an r weights the modes of large eigenvalue sums heavily;
rounding in the forward products spreads over all modes and is divided by the
smallest sums, so the error relative to s* is bounded by u kappa (kappa the
largest ratio lam_max / lam_min of a direction, u the unit roundoff): FP32
mode products reach 1.7e-4 at h^-1 = 128, p = 6 (kappa = 9.9e4) when emulated
with numpy's FP32 products, 1.7e-6 at p = 3.  Tolerances: FP64 max(1e-11,
u64 kappa), FP32 max(1e-4, u32 kappa).
"""
import numpy as np
import pytest

import synth
from helpers import rel, to_dev, to_host
from oracle import assembly, fd

pytestmark = pytest.mark.gpu

GEMM_3D = [
    # forced onto the tiled products (IGAFD_FD_GEMM=1): every tile ragged
    ("ring_ragged_p2", synth.make_problem(3, 2, [synth.jittered_knots(E, 2, 30 + E) for E in (19, 35, 16)],
                                          geometry={"kind": "ring"}), "1"),
    ("warped_kappa_p5", synth.uniform_problem(3, [4, 6, 3], 5, geometry=synth.warped_geometry(6),
                                              coefficient=synth.sincos_coefficient(0.4, 1, 2, 0.2, 0.0)), "1"),
    # a direction longer than the fused passes take: tiled products by default
    ("ring_long_dir1_p3", synth.uniform_problem(3, [170, 5, 4], 3, geometry={"kind": "ring"}), None),
    ("ring_long_dir3_p1", synth.uniform_problem(3, [6, 7, 200], 1, geometry={"kind": "ring"}), None),
]


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


@pytest.mark.parametrize("name,prob,force", GEMM_3D, ids=[g[0] for g in GEMM_3D])
def test_3d_tiled_products(api, name, prob, force, rng, monkeypatch):
    """Applies against the oracle (plain and scaled), and solves whose (r, s)
    partials come from the last product's epilogue against the solve with the
    per-strip / fused products."""
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    if force:
        monkeypatch.setenv("IGAFD_FD_GEMM", force)
    else:
        monkeypatch.delenv("IGAFD_FD_GEMM", raising=False)
    with api.igafd_setup(prob) as ctx:
        assert api.igafd_get_shape(ctx)["fd_fused"] == 0
        r = rng.standard_normal(ctx.N)
        ref = fd.fd_apply(F, r)
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16", 5e-2), ("bf16x3", 6e-4)):
            s = to_dev(np.full(ctx.N, 3.0))
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            assert rel(to_host(s), ref) < tol, prec
        S = np.exp(0.1 * rng.standard_normal(ctx.N))
        api.igafd_set_scaling(ctx, to_dev(S))
        for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4), ("bf16x3", 6e-4)):
            s = to_dev(np.zeros(ctx.N))
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            assert rel(to_host(s), S * fd.fd_apply(F, S * r)) < tol, prec
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


def test_precond_only_context(api, rng):
    prob = synth.make_problem(3, 3, [synth.jittered_knots(E, 3, 60 + E) for E in (9, 7, 8)],
                              geometry={"kind": "ring"})
    with api.igafd_setup_precond(prob) as pc, api.igafd_setup(prob) as full:
        assert pc.band_bytes == 0 and full.band_bytes > 0
        assert (pc.N, pc.nnz, tuple(pc.n)) == (full.N, full.nnz, tuple(full.n))
        r = to_dev(rng.standard_normal(pc.N))
        for prec in ("fp64", "fp32", "bf16", "bf16x3"):
            s1, s2 = to_dev(np.zeros(pc.N)), to_dev(np.zeros(pc.N))
            api.igafd_apply_precond(pc, prec, r, s1)
            api.igafd_apply_precond(full, prec, r, s2)
            assert np.array_equal(to_host(s1), to_host(s2)), prec
        b1, b2 = to_dev(np.zeros(pc.N)), to_dev(np.zeros(pc.N))
        api.igafd_load_vector(pc, synth.RHS_SINPROD, b1)
        api.igafd_load_vector(full, synth.RHS_SINPROD, b2)
        assert np.array_equal(to_host(b1), to_host(b2))
        assert api.igafd_spectral_bounds(pc) == api.igafd_spectral_bounds(full)
        for d in range(3):
            U1, l1 = api.igafd_get_eigen(pc, d)
            U2, l2 = api.igafd_get_eigen(full, d)
            assert np.array_equal(U1, U2) and np.array_equal(l1, l2)
        assert api.igafd_set_adi(pc, 0.1) == api.igafd_set_adi(full, 0.1)
        s1, s2 = to_dev(np.zeros(pc.N)), to_dev(np.zeros(pc.N))
        api.igafd_apply_precond(pc, "fp64", r, s1)
        api.igafd_apply_precond(full, "fp64", r, s2)
        assert np.array_equal(to_host(s1), to_host(s2))
        api.igafd_set_adi(pc, 0)
        x, y = to_dev(np.ones(pc.N)), to_dev(np.zeros(pc.N))
        calls = [lambda: api.igafd_apply_A(pc, x, y), lambda: api.igafd_solve(pc, x, y),
                 lambda: api.igafd_solve_batched([pc], [x], [y]), lambda: api.igafd_diagonals(pc, y, None),
                 lambda: api.igafd_features(pc, to_dev(np.zeros(8 * pc.N)).float()),
                 lambda: api.igafd_scaling_targets(pc, to_dev(np.zeros(pc.N)).float()),
                 lambda: api.igafd_set_scaling_diag_ratio(pc), lambda: api.igafd_autotune(pc),
                 lambda: api.igafd_autotune(pc, spmv_rows=2)]
        for k, call in enumerate(calls):
            with pytest.raises(api.IgafdError):
                call()
        api.igafd_autotune(pc, fd_tiles=3)   # the FD shape alone is allowed
        s1 = to_dev(np.zeros(pc.N))
        api.igafd_apply_precond(pc, "fp64", r, s1)
        F = fd.setup(prob)
        assert rel(to_host(s1), fd.fd_apply(F, to_host(r))) < 1e-11


@pytest.mark.parametrize("E,p", [(128, 6), (256, 3), (512, 3)])
def test_cube_direct_solver(api, E, p):
    """Unit cube, P = A: the FD apply is the direct solve.  s* drawn, r = P s*
    by the oracle, P^-1 r on the GPU must return s* (FP64, FP32 and split BF16,
    whose error per product is at most about 3 * 2^-16 relative)."""
    prob = synth.unit_cube(E, p)
    F = fd.setup(prob)
    n = len(F[0]["lam"])
    kappa = max(f["lam"].max() / f["lam"].min() for f in F)
    x = np.random.default_rng(E + p).standard_normal(n ** 3)
    r = fd.apply_P(F, x)
    print(f"cube E={E} p={p} n={n}: r = P s* done", flush=True)
    with api.igafd_setup_precond(prob) as ctx:
        assert ctx.N == n ** 3 and ctx.band_bytes == 0
        rd = to_dev(r)
        del r
        s = to_dev(np.zeros(ctx.N))
        for prec, tol in (("fp64", max(1e-11, 2.0 ** -53 * kappa)), ("fp32", max(1e-4, 2.0 ** -24 * kappa)),
                          ("bf16x3", max(6e-4, 3 * 2.0 ** -16 * kappa))):
            api.igafd_apply_precond(ctx, prec, rd, s)
            err = rel(to_host(s), x)
            print(f"{prec}: rel. error {err:.3g} (tolerance {tol:.3g})", flush=True)
            assert err < tol, prec
