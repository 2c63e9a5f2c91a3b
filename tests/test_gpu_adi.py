"""GPU parity of the three-variable ADI preconditioner P_J (Sec. 5.2 Alg.
'3D ADI method', Sec. 4.2 Thm. ADIprec) against the oracle.

The parameters (count J, omega_j, rho_J = ||T_J||) must agree with the
oracle's rule; one apply s_J = P_J^-1 r within 1e-11 relative (the same FP64
bound as the FD apply: the steps are products and solves with matrices of
condition ~ that of M_d^-1 K_d); CG + P_J within 1e-7 of the oracle's
solution and +-1 iteration.  Full size: the thick ring 128^3, p = 3, against
the oracle's closed form (the steps themselves are pinned to it at small
sizes), FP64 tolerance max(1e-11, eps kappa) as for the FD apply.
"""
import numpy as np
import pytest

import synth
from helpers import rel, to_dev, to_host
from oracle import adi, assembly, fd, pcg

pytestmark = pytest.mark.gpu

CASES = [
    ("uniform_p2", synth.uniform_problem(3, [6, 7, 5], 2)),
    ("jittered_p3", synth.make_problem(3, 3, [synth.jittered_knots(E, 3, 20 + E) for E in (8, 6, 7)],
                                       geometry={"kind": "ring"})),
    ("warped_p4", synth.uniform_problem(3, [9, 8, 10], 4, geometry=synth.warped_geometry(2))),
    ("ragged_p1", synth.uniform_problem(3, [17, 19, 7], 1)),
    ("small_p5", synth.uniform_problem(3, [4, 5, 6], 5)),
    ("small_p6", synth.uniform_problem(3, [3, 4, 2], 6)),
]
IDS = [c[0] for c in CASES]


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


@pytest.mark.parametrize("name,prob", CASES, ids=IDS)
def test_adi_parameters_and_apply(api, name, prob):
    F = fd.setup(prob)
    w, r_or, J0 = adi.parameters(F, 0.1)
    with api.igafd_setup(prob) as ctx:
        J, rho = api.igafd_set_adi(ctx, 0.1)
        g = api.igafd_get_adi(ctx)
        assert J == len(w) == g["J"] and g["J0"] == J0
        assert np.allclose(g["omegas"], w, rtol=1e-12, atol=0)
        assert abs(rho - r_or) <= 1e-10 * r_or and g["rho"] == rho
        x = synth.random_vector(ctx.N, 7)
        s = to_dev(np.full(ctx.N, 2.0))
        api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
        ref = adi.apply(F, x, w)
        assert rel(to_host(s), ref) < 1e-11
        assert rel(to_host(s), adi.closed_form(F, x, w)) < 1e-11


@pytest.mark.parametrize("name,prob", CASES[:4], ids=IDS[:4])
def test_adi_solve(api, name, prob):
    F = fd.setup(prob)
    w, _, _ = adi.parameters(F, 0.1)
    A = assembly.assemble_matrix(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.pcg(lambda v: A @ v, lambda v: adi.apply(F, v, w), b, rtol=1e-8)
    with api.igafd_setup(prob) as ctx:
        api.igafd_set_adi(ctx, 0.1)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, rtol=1e-8)
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert abs(info["iters"] - info_or["iters"]) <= 1, (info["iters"], info_or["iters"])
        assert rel(to_host(u), u_or) <= 1e-7
        # back to the exact FD apply
        api.igafd_set_adi(ctx, 0)
        assert api.igafd_get_adi(ctx)["J"] == 0
        x = synth.random_vector(ctx.N, 8)
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
        assert rel(to_host(s), fd.fd_apply(F, x)) < 1e-11


def test_adi_rejects(api):
    prob = CASES[0][1]
    with api.igafd_setup(prob) as ctx:
        for eps in (-0.1, 1.0, 2.0):
            with pytest.raises(api.IgafdError):
                api.igafd_set_adi(ctx, eps)
        api.igafd_set_adi(ctx, 0.1)
        x, s = to_dev(np.ones(ctx.N)), to_dev(np.zeros(ctx.N))
        for prec in ("fp32", "bf16"):
            with pytest.raises(api.IgafdError):
                api.igafd_apply_precond(ctx, prec, x, s)
            with pytest.raises(api.IgafdError):
                api.igafd_solve(ctx, x, s, precision=prec)
        with pytest.raises(api.IgafdError):
            api.igafd_solve_batched([ctx], [x], [s])
    with api.igafd_setup(synth.square_2d(E=6, p=2)) as c2:
        with pytest.raises(api.IgafdError):
            api.igafd_set_adi(c2, 0.1)


def test_adi_thick_ring_128_p3(api):
    prob = synth.thick_ring(E=128, p=3)
    F = fd.setup(prob)
    w, r_or, _ = adi.parameters(F, 0.1)
    kappa = max(f["lam"].max() / f["lam"].min() for f in F)
    with api.igafd_setup(prob) as ctx:
        J, rho = api.igafd_set_adi(ctx, 0.1)
        assert J == len(w) and np.allclose(api.igafd_get_adi(ctx)["omegas"], w, rtol=1e-12, atol=0)
        x = np.random.default_rng(9).standard_normal(ctx.N)
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
        assert rel(to_host(s), adi.closed_form(F, x, w)) < max(1e-11, 2.2e-16 * kappa)
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, b, u, rtol=1e-8)
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        api.igafd_set_adi(ctx, 0)
        u2 = to_dev(np.zeros(ctx.N))
        info_fd = api.igafd_solve(ctx, b, u2, rtol=1e-8)
        # Thm. ADIprec: kappa grows by at most (1+eps)/(1-eps) = 1.22, so CG needs
        # at most ~11% more iterations (plus one for rounding)
        assert info["iters"] <= int(np.ceil(info_fd["iters"] * np.sqrt(1.1 / 0.9))) + 1
        assert rel(to_host(u), to_host(u2)) <= 1e-6


@pytest.mark.parametrize("name,prob", CASES[:4], ids=IDS[:4])
def test_adi_greedy_parameters_and_solve(api, name, prob):
    """Greedy parameters (eq. greedy1/2) against the oracle's rule: the same
    count, the parameters and rho_J to rounding; the apply against the
    closed form; CG + P_J against the oracle's CG with those parameters."""
    F = fd.setup(prob)
    w, r_or, J0 = adi.greedy_parameters(F, 0.1)
    A = assembly.assemble_matrix(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.pcg(lambda v: A @ v, lambda v: adi.apply(F, v, w), b, rtol=1e-8)
    with api.igafd_setup(prob) as ctx:
        J, rho = api.igafd_set_adi_greedy(ctx, 0.1)
        g = api.igafd_get_adi(ctx)
        assert J == len(w) and g["J0"] == J0
        assert np.allclose(g["omegas"], w, rtol=1e-9, atol=0)
        assert abs(rho - r_or) <= 1e-9 * r_or and rho <= 0.1
        x = synth.random_vector(ctx.N, 17)
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
        assert rel(to_host(s), adi.closed_form(F, x, w)) < 1e-11
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, to_dev(b), u, rtol=1e-8)
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert abs(info["iters"] - info_or["iters"]) <= 1, (info["iters"], info_or["iters"])
        assert rel(to_host(u), u_or) <= 1e-7


def test_adi_greedy_thick_ring_128_p3(api):
    """Full size: greedy parameters against the oracle's, the apply against the
    closed form, and CG + P_J within the Thm. ADIprec bound of CG + P."""
    prob = synth.thick_ring(E=128, p=3)
    F = fd.setup(prob)
    w, r_or, _ = adi.greedy_parameters(F, 0.1)
    kappa = max(f["lam"].max() / f["lam"].min() for f in F)
    with api.igafd_setup(prob) as ctx:
        J, rho = api.igafd_set_adi_greedy(ctx, 0.1)
        assert J == len(w) and np.allclose(api.igafd_get_adi(ctx)["omegas"], w, rtol=1e-9, atol=0)
        x = np.random.default_rng(19).standard_normal(ctx.N)
        s = to_dev(np.zeros(ctx.N))
        api.igafd_apply_precond(ctx, "fp64", to_dev(x), s)
        assert rel(to_host(s), adi.closed_form(F, x, w)) < max(1e-11, 2.2e-16 * kappa)
        b = to_dev(np.zeros(ctx.N))
        api.igafd_load_vector(ctx, synth.RHS_SINPROD, b)
        u = to_dev(np.zeros(ctx.N))
        info = api.igafd_solve(ctx, b, u, rtol=1e-8)
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        api.igafd_set_adi(ctx, 0)
        u2 = to_dev(np.zeros(ctx.N))
        info_fd = api.igafd_solve(ctx, b, u2, rtol=1e-8)
        assert info["iters"] <= int(np.ceil(info_fd["iters"] * np.sqrt(1.1 / 0.9))) + 1
        assert rel(to_host(u), to_host(u2)) <= 1e-6
