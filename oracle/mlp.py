"""FP64 reference of the learned diagonal scaling (test infrastructure only).

The paper leaves better preconditioning of complicated geometry to future work
(Sec. 3, remarks after Prop. 1).  The scaled preconditioner S P^-1 S uses a
diagonal S > 0.  Its "exact" diagonal-ratio choice is
S_i = sqrt(P_ii / A_ii) (so that diag(S^-1 P S^-1) = diag(A)); the network
predicts t_i = log S_i = 1/2 log(P_ii / A_ii) from local statistics:

    features_i = sum_t w_t B_i(t) g(t) / sum_t w_t B_i(t)   (quadrature points of supp B_i)
    g = (G11, G22, G33, G12, G13, G23, kappa),  G = |det J| J^-1 J^-T   (= Q / kappa, eq. Q)
    plus the degree p as an eighth input.

Network: z1 = W1 f + b1, h1 = tanh z1, z2 = W2 h1 + b2, h2 = tanh z2,
t = w3 . h2 + b3, inputs normalised as (f - mean) / std.  Loss L = mean (t - t*)^2.
Parameter vector layout: W1 (64 x 8 row-major), b1, W2 (64 x 64), b2, w3, b3.

Parity: gradients are pinned by central finite differences of this FP64
loss; features by their definition on tiny meshes and by the identity map
(G = I, kappa = 1).
"""
from __future__ import annotations

import numpy as np

from . import assembly, fd, geometry

NIN, NH = 8, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, k = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + size], dtype=np.float64).reshape(shape)
        k += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SIZES])


def forward(theta, mean, inv_std, feat):
    """Returns t and the activations (normalised inputs f, h1, h2)."""
    P = unpack(theta)
    f = (np.asarray(feat, np.float64) - mean) * inv_std
    h1 = np.tanh(f @ P["W1"].T + P["b1"])
    h2 = np.tanh(h1 @ P["W2"].T + P["b2"])
    t = h2 @ P["w3"] + P["b3"][0]
    return t, (f, h1, h2)


def loss_and_grad(theta, mean, inv_std, feat, target):
    """L = mean (t - target)^2 and dL/dtheta by back-propagation."""
    P = unpack(theta)
    t, (f, h1, h2) = forward(theta, mean, inv_std, feat)
    n = len(t)
    e = t - target
    L = float(np.mean(e * e))
    dt = 2.0 * e / n
    g = {"w3": h2.T @ dt, "b3": np.array([dt.sum()])}
    dz2 = np.outer(dt, P["w3"]) * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ f
    g["b1"] = dz1.sum(axis=0)
    return L, pack(g)


def features(problem):
    """Per-dof inputs (N x 8) by their definition: B_i-weighted averages over
    the Gauss points of supp B_i of G's six entries and kappa, then p."""
    mesh = assembly._Mesh(problem)
    d = mesh.d
    acc = np.zeros((mesh.N, 8))
    for part in assembly._chunks(mesh.all_elements(), 2048):
        xi, w, vals, _, dofs = mesh.element_data(part)
        C, T = w.shape
        x, J = geometry.map_and_jacobian(problem["geometry"], xi.reshape(-1, d))
        det = np.abs(np.linalg.det(J))
        Jinv = np.linalg.inv(J)
        G = det[:, None, None] * (Jinv @ np.swapaxes(Jinv, 1, 2))
        G3 = np.zeros((len(det), 3, 3))
        G3[:, :d, :d] = G
        kap = geometry.kappa(problem["coefficient"], x)
        g = np.stack([G3[:, 0, 0], G3[:, 1, 1], G3[:, 2, 2], G3[:, 0, 1], G3[:, 0, 2], G3[:, 1, 2], kap,
                      np.ones_like(kap)], axis=1).reshape(C, T, 8)
        contrib = np.einsum("et,eta,etc->eac", w, vals, g)
        ok = dofs >= 0
        np.add.at(acc, dofs[ok], contrib[ok])
    out = acc[:, :7] / acc[:, 7:8]
    return np.concatenate([out, np.full((mesh.N, 1), float(problem["degree"]))], axis=1)


def targets(problem, A=None):
    """t_i = 1/2 log(P_ii / A_ii)."""
    if A is None:
        A = assembly.assemble_matrix(problem)
    dP = fd.diag_P(fd.setup(problem))
    return 0.5 * np.log(dP / A.diagonal())
