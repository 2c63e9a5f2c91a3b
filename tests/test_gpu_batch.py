"""GPU: batched solves of uneven problems (grouped launches or a stream pool,
graph-captured chunks) give the same iterates as one-at-a-time solves (same
kernel bodies, same reduction order: bitwise), and match the oracle."""
import numpy as np
import pytest

import synth
from helpers import rel, to_dev, to_host
from oracle import assembly, fd, pcg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import paper_1602_01636_amd as api
    api.lib()
    return api


def _batch_problems():
    rng = np.random.default_rng(11)
    out = []
    for k in range(6):
        p = int(rng.integers(2, 6))
        m = rng.integers(p + 6, p + 16, size=3)
        geom = {"kind": "ring"} if k % 2 == 0 else synth.warped_geometry(1000 + k)
        out.append(synth.uniform_problem(3, [int(mm) - p for mm in m], p, geometry=geom))
    return out


@pytest.mark.parametrize("graph,grouped", [(True, True), (False, True), (True, False)])
def test_batched_equals_individual(api, graph, grouped, monkeypatch):
    """Grouped launches (every step one launch over all problems) and the
    stream pool, with and without graph capture: bitwise the single solves."""
    import torch
    if not graph:
        monkeypatch.setenv("IGAFD_NO_GRAPH", "1")
    if not grouped:
        monkeypatch.setenv("IGAFD_BATCH_GROUPED", "0")
    probs = _batch_problems()
    ctxs = [api.igafd_setup(pr) for pr in probs]
    bs, us, ref = [], [], []
    for c in ctxs:
        b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
        api.igafd_load_vector(c, synth.RHS_SINPROD, b)
        u = torch.zeros_like(b)
        info = api.igafd_solve(c, b, u)
        ref.append((info, u.clone()))
        bs.append(b)
        us.append(torch.full_like(b, 3.0))
    infos, wall = api.igafd_solve_batched(ctxs, bs, us)
    assert wall > 0
    for (info_ref, u_ref), info, u in zip(ref, infos, us):
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert info["iters"] == info_ref["iters"]
        assert torch.equal(u, u_ref)
    for c in ctxs:
        c.close()


def test_batched_mixed_tile_blocks_equals_individual(api, monkeypatch):
    """Problems whose tiled A products run 512-thread blocks next to ones with
    256 (separate grouped launches): bitwise the single solves."""
    import torch
    probs = _batch_problems()
    ctxs = []
    for k, pr in enumerate(probs):
        monkeypatch.setenv("IGAFD_SPMV_TILE", "2x2x512" if k % 2 == 0 else "2x2")
        ctxs.append(api.igafd_setup(pr))
    threads = [api.igafd_get_shape(c)["tile_threads"] for c in ctxs]
    assert threads[0::2] == [512] * 3 and all(t == 256 for t in threads[1::2])
    bs, us, ref = [], [], []
    for c in ctxs:
        b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
        api.igafd_load_vector(c, synth.RHS_SINPROD, b)
        u = torch.zeros_like(b)
        info = api.igafd_solve(c, b, u)
        ref.append((info, u.clone()))
        bs.append(b)
        us.append(torch.zeros_like(b))
    infos, _ = api.igafd_solve_batched(ctxs, bs, us)
    for (info_ref, u_ref), info, u in zip(ref, infos, us):
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert info["iters"] == info_ref["iters"]
        assert torch.equal(u, u_ref)
    for c in ctxs:
        c.close()


def test_batched_split_bf16_equals_individual(api):
    """The batched (graph-captured) path with split-BF16 applies in the
    flexible CG: bitwise the individual solves, converged in FP64."""
    import torch
    probs = _batch_problems()[:4]
    ctxs = [api.igafd_setup(pr) for pr in probs]
    bs, us, ref = [], [], []
    for c in ctxs:
        b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
        api.igafd_load_vector(c, synth.RHS_SINPROD, b)
        u = torch.zeros_like(b)
        info = api.igafd_solve(c, b, u, precision="bf16x3")
        ref.append((info, u.clone()))
        bs.append(b)
        us.append(torch.zeros_like(b))
    infos, _ = api.igafd_solve_batched(ctxs, bs, us, precision="bf16x3")
    for (info_ref, u_ref), info, u in zip(ref, infos, us):
        assert info["status"] == "OK" and info["true_relres"] <= 1e-8
        assert info["iters"] == info_ref["iters"]
        assert torch.equal(u, u_ref)
    for c in ctxs:
        c.close()


def test_batched_matches_oracle_and_autotune(api):
    import torch
    prob = synth.uniform_problem(3, [7, 9, 6], 3, geometry=synth.warped_geometry(1001))
    A = assembly.assemble_matrix(prob)
    F = fd.setup(prob)
    b = assembly.assemble_load(prob, synth.RHS_SINPROD)
    u_or, info_or = pcg.solve(prob, A, F, b)
    with api.igafd_setup(prob) as c1, api.igafd_setup(synth.thick_ring(E=9, p=2)) as c2:
        api.igafd_autotune(c1)
        api.igafd_autotune(c2, fd_tiles=1, spmv_rows=4)
        b2 = torch.zeros(c2.N, dtype=torch.float64, device="cuda")
        api.igafd_load_vector(c2, synth.RHS_SINPROD, b2)
        u1, u2 = to_dev(np.zeros(c1.N)), torch.zeros_like(b2)
        infos, _ = api.igafd_solve_batched([c1, c2], [to_dev(b), b2], [u1, u2])
        assert abs(infos[0]["iters"] - info_or["iters"]) <= 1
        assert rel(to_host(u1), u_or) <= 1e-7
        assert infos[1]["true_relres"] <= 1e-8


def test_batched_scaled_equals_individual(api):
    """S P^-1 S in the grouped batch (the scaling in the first and last FD
    passes of each problem's jobs): bitwise the single scaled solves."""
    import torch
    probs = _batch_problems()[:4]
    ctxs = [api.igafd_setup(pr) for pr in probs]
    try:
        bs, us, ref = [], [], []
        for c in ctxs:
            api.igafd_set_scaling_diag_ratio(c)
            b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
            api.igafd_load_vector(c, synth.RHS_SINPROD, b)
            u = torch.zeros_like(b)
            info = api.igafd_solve(c, b, u, use_scaling=True)
            ref.append((info, u.clone()))
            bs.append(b)
            us.append(torch.zeros_like(b))
        infos, _ = api.igafd_solve_batched(ctxs, bs, us, use_scaling=True)
        for (info_ref, u_ref), info, u in zip(ref, infos, us):
            assert info["status"] == "OK" and info["true_relres"] <= 1e-8
            assert info["iters"] == info_ref["iters"]
            assert torch.equal(u, u_ref)
    finally:
        for c in ctxs:
            c.close()


def test_batched_edge_cases(api):
    """A problem with b = 0 (stops at the start: no iteration, u = 0) among
    others in the grouped batch, and a batch mixing 2D and 3D problems (the
    stream-pool path): bitwise the single solves."""
    import torch
    probs = _batch_problems()[:3]
    ctxs = [api.igafd_setup(pr) for pr in probs]
    try:
        bs, us, ref = [], [], []
        for k, c in enumerate(ctxs):
            b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
            if k != 1:
                api.igafd_load_vector(c, synth.RHS_SINPROD, b)
            u = torch.zeros_like(b)
            info = api.igafd_solve(c, b, u)
            ref.append((info, u.clone()))
            bs.append(b)
            us.append(torch.full_like(b, 2.0))
        infos, _ = api.igafd_solve_batched(ctxs, bs, us)
        assert infos[1]["iters"] == 0 and infos[1]["status"] == "OK" and not torch.any(us[1])
        for (info_ref, u_ref), info, u in zip(ref, infos, us):
            assert info["iters"] == info_ref["iters"]
            assert torch.equal(u, u_ref)
    finally:
        for c in ctxs:
            c.close()
    mixed = [synth.uniform_problem(2, [20, 17], 3, geometry={"kind": "ring"}), _batch_problems()[0]]
    ctxs = [api.igafd_setup(pr) for pr in mixed]
    try:
        bs, us, ref = [], [], []
        for c in ctxs:
            b = torch.zeros(c.N, dtype=torch.float64, device="cuda")
            api.igafd_load_vector(c, synth.RHS_SINPROD, b)
            u = torch.zeros_like(b)
            info = api.igafd_solve(c, b, u)
            ref.append((info, u.clone()))
            bs.append(b)
            us.append(torch.zeros_like(b))
        infos, _ = api.igafd_solve_batched(ctxs, bs, us)
        for (info_ref, u_ref), info, u in zip(ref, infos, us):
            assert info["status"] == "OK" and info["true_relres"] <= 1e-8
            assert info["iters"] == info_ref["iters"]
            assert torch.equal(u, u_ref)
    finally:
        for c in ctxs:
            c.close()
