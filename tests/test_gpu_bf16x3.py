"""GPU parity of the split-BF16 preconditioner apply (IGAFD_BF16X3: each FP32
operand held as hi + lo BF16 parts, three BF16 MFMAs per product; Henry, Tang
and Heinecke 2019) against the FP64 oracle, on every apply path: the fused 3D
passes, the six separate 3D mode products, the 3D and 2D tiled products, the
small-2D mode products, the scaled apply S P^-1 S and the L-shaped Schwarz
apply.

Tolerance: the BF16 tests allow 5e-2 for a unit roundoff of 2^-8; the split
form's error per product is at most about 3 * 2^-16 relative (lo rounded
to BF16 on each operand, the dropped lo_a lo_b term; checked on the host in
test_split_bf16_bound.py), 3/256 of that, so the same scaling gives 5.9e-4;
the tests allow 6e-4.  On every case the split
apply's error must also be at least 30x below the plain BF16 apply's on the
same input.  Solves use the flexible CG and must match the oracle's FP64
solution to 1e-7 at rtol 1e-8, like every other precision.
"""
import numpy as np
import pytest

import synth
from helpers import rel, small_problems, to_dev, to_host
from oracle import assembly, fd, pcg
from oracle import multipatch as mp

pytestmark = pytest.mark.gpu

TOL_X3 = 6e-4
PROBLEMS = small_problems()
IDS = [p[0] for p in PROBLEMS]


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


def apply_err(api, ctx, prec, r, ref, fill=0.0):
    s = to_dev(np.full(ctx.N, fill))
    api.igafd_apply_precond(ctx, prec, to_dev(r), s)
    return rel(to_host(s), ref)


def check_both(api, ctx, r, ref):
    e3 = apply_err(api, ctx, "bf16x3", r, ref, 7.0)
    e1 = apply_err(api, ctx, "bf16", r, ref, 7.0)
    assert e3 < TOL_X3 and e3 * 30 < e1, (e3, e1)
    return e3


@pytest.mark.parametrize("name,prob", PROBLEMS, ids=IDS)
def test_split_apply_matches_oracle(api, name, prob, rng):
    F = fd.setup(prob)
    with api.igafd_setup(prob) as ctx:
        r = rng.standard_normal(ctx.N)
        check_both(api, ctx, r, fd.fd_apply(F, r))
        # the scaled preconditioner S P^-1 S
        S = np.exp(0.1 * rng.standard_normal(ctx.N))
        api.igafd_set_scaling(ctx, to_dev(S))
        e = apply_err(api, ctx, "bf16x3", r, S * fd.fd_apply(F, S * r))
        assert e < TOL_X3, e
        api.igafd_set_scaling(ctx, None)


@pytest.mark.parametrize("force", ["fused0", "gemm1"])
def test_split_apply_other_3d_paths(api, rng, monkeypatch, force):
    # n = (11, 65, 66): ragged last row tiles; the six separate mode products
    # and the 3D tiled products (forced on, every tile ragged)
    prob = synth.uniform_problem(3, [10, 64, 65], 3, geometry=synth.warped_geometry(6),
                                 coefficient=synth.sincos_coefficient(0.3, 1, 1, 0.2, 0.4))
    F = fd.setup(prob)
    if force == "fused0":
        monkeypatch.setenv("IGAFD_FD_FUSED", "0")
    else:
        monkeypatch.setenv("IGAFD_FD_GEMM", "1")
    with api.igafd_setup(prob) as ctx:
        shape = api.igafd_get_shape(ctx)
        if force == "fused0":
            assert shape["fd_fused"] == 0
        r = rng.standard_normal(ctx.N)
        check_both(api, ctx, r, fd.fd_apply(F, r))


def test_split_apply_2d_tiled(api, rng, monkeypatch):
    prob = synth.uniform_problem(2, [37, 45], 3, geometry={"kind": "ring"})
    F = fd.setup(prob)
    monkeypatch.setenv("IGAFD_FD_GEMM", "1")
    with api.igafd_setup(prob) as ctx:
        r = rng.standard_normal(ctx.N)
        check_both(api, ctx, r, fd.fd_apply(F, r))


@pytest.mark.parametrize("gemm", ["0", "1"])
def test_split_apply_lshape(api, monkeypatch, gemm):
    monkeypatch.setenv("IGAFD_FD_GEMM", gemm)
    knots, p = synth.uniform_knots(24, 3), 3
    L = mp.LShape(knots, p)
    Sch = mp.Schwarz(L)
    pos, n = L.square_index()
    with api.igafd_lshape_setup(knots, p) as ctx:
        r = synth.random_vector(n * n, 35)
        ref = Sch.ias(r[pos])
        errs = {}
        for prec in ("bf16x3", "bf16"):
            s = to_dev(np.full(n * n, 5.0))
            api.igafd_apply_precond(ctx, prec, to_dev(r), s)
            sg = to_host(s)
            errs[prec] = rel(sg[pos], ref)
            mask = np.ones(n * n, dtype=bool)
            mask[pos] = False
            assert np.all(sg[mask] == 0.0), prec
        assert errs["bf16x3"] < TOL_X3 and errs["bf16x3"] * 30 < errs["bf16"], errs


@pytest.mark.parametrize("name", ["3d_warped_kappa_p3", "2d_warped_kappa_p4", "3d_ring_p2"])
def test_split_solve_matches_oracle(api, name):
    prob = dict(PROBLEMS)[name]
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.pcg(lambda v: A @ v, lambda r: fd.fd_apply(F, r), b, rtol=1e-8)
    with api.igafd_setup(prob) as ctx:
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, rtol=1e-8, precision="bf16x3")
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert rel(to_host(u), u_or) <= 1e-7
        # the split apply is close enough to FP64 that the iteration count stays
        # within one of the oracle's FP64 count (plain BF16 may need more)
        assert abs(info["iters"] - info_or["iters"]) <= 1, (info["iters"], info_or["iters"])
        with pytest.raises(api.IgafdError):
            api.igafd_solve(ctx, to_dev(b), u, precision="bf16x3", flexible=False)
