"""Shared helpers of the GPU parity tests: run the library through its C ABI
binding and the oracle on the same seeded inputs."""
import numpy as np

import synth


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    torch = torch_cuda()
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    """Relative distance of a from the reference b, in the 2-norm and entry by
    entry: max(||a - b||_2 / ||b||_2, ||a - b||_inf / ||b||_inf).  Every
    `rel(..) < tol` check in the GPU tests therefore bounds both the global
    error and the largest single-entry error (a wrong block holding a few
    percent of the norm fails the second)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b
    r2 = np.linalg.norm(d) / max(np.linalg.norm(b), 1e-300)
    rinf = np.abs(d).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)
    return float(max(r2, rinf))


def small_problems():
    """Small 2D/3D problems spanning several 256-row blocks, ragged mode tiles,
    nonuniform knots, every map and the coefficient."""
    P = []
    P.append(("2d_identity_p2", synth.make_problem(2, 2, [synth.jittered_knots(19, 2, 1), synth.jittered_knots(23, 2, 2)])))
    P.append(("2d_annulus_p3", synth.uniform_problem(2, [21, 18], 3, geometry={"kind": "ring"})))
    P.append(("2d_warped_kappa_p4", synth.uniform_problem(2, [17, 20], 4, geometry=synth.warped_geometry(5, dim=2),
                                                          coefficient=synth.sincos_coefficient(0.4, 1, 2, 0.3, 0.1))))
    P.append(("3d_ring_p2", synth.make_problem(3, 2, [synth.jittered_knots(E, 2, 10 + E) for E in (9, 11, 13)],
                                                 geometry={"kind": "ring"})))
    P.append(("3d_warped_kappa_p3", synth.uniform_problem(3, [10, 8, 12], 3, geometry=synth.warped_geometry(3),
                                                          coefficient=synth.sincos_coefficient(0.5, 1, 1, 0.0, 0.0))))
    P.append(("3d_identity_p1", synth.uniform_problem(3, [17, 19, 7], 1)))
    P.append(("3d_warped_p5", synth.uniform_problem(3, [6, 7, 5], 5, geometry=synth.warped_geometry(7))))
    return P
