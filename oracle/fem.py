"""Linear-tet kinematics and elastic energy (oracle, FP64, test infrastructure).

Per tet e = (i0, i1, i2, i3):  Dm = [X1-X0 | X2-X0 | X3-X0],  V_e = det(Dm)/6,
Ds = the same with current positions, F = Ds Dm^-1 (the deformation gradient
fed to Eq. 2).  The elastic energy is sum_e V_e Psi(F_e); its gradient and
Hessian follow from dF/dx, written out as the 9x12 matrix D below.
"""
from __future__ import annotations

import numpy as np

from . import material


def rest_data(X, tets):
    """Dm^-1 [T,3,3] and V_e [T]; raises on a non-positive volume."""
    Dm = np.stack([X[tets[:, k]] - X[tets[:, 0]] for k in (1, 2, 3)], axis=2)
    vol = np.linalg.det(Dm) / 6.0
    if np.any(vol <= 0.0):
        raise ValueError("tet with non-positive rest volume")
    return np.linalg.inv(Dm), vol


def shape_gradients(Dminv):
    """G[e, a, :] = dF/dx_a row: rows of Dm^-1 for a = 1..3, minus their sum
    for a = 0, so that F = sum_a x_a (outer) G_a."""
    G = np.empty(Dminv.shape[:-2] + (4, 3))
    G[..., 1:, :] = Dminv
    G[..., 0, :] = -Dminv.sum(axis=-2)
    return G


def deformation_gradient(x, tets, Dminv):
    Ds = np.stack([x[tets[:, k]] - x[tets[:, 0]] for k in (1, 2, 3)], axis=2)
    return Ds @ Dminv


def dF_dx(G):
    """D[e, 3 i + j, 3 a + k] = delta_ik G[e, a, j]  (9 x 12 per tet)."""
    T = G.shape[0]
    D = np.zeros((T, 3, 3, 4, 3))
    for i in range(3):
        D[:, i, :, :, i] = np.swapaxes(G, 1, 2)
    return D.reshape(T, 9, 12)


def elastic_energy(x, tets, Dminv, vol, mu, lam, alpha):
    """Per-tet V_e Psi(F_e) (mu, lam, alpha scalars or per-tet arrays)."""
    F = deformation_gradient(x, tets, Dminv)
    return vol * material.energy_density(F, mu, lam, alpha)


def elastic_gradient(x, tets, Dminv, vol, mu, lam, alpha):
    """Per-tet 12-vector dE_e/dx: V_e P G_a for each local vertex a."""
    F = deformation_gradient(x, tets, Dminv)
    P = material.first_piola(F, mu, lam, alpha)
    G = shape_gradients(Dminv)
    g = np.einsum("eij,eaj->eai", P, G) * vol[:, None, None]
    return g.reshape(-1, 12)


def elastic_hessian(x, tets, Dminv, vol, mu, lam, alpha, project=True):
    """Per-tet 12x12 V_e D^T (d^2 Psi / dF^2) D, PSD-projected in F-space."""
    F = deformation_gradient(x, tets, Dminv)
    H = material.energy_hessian(F, mu, lam, alpha)
    if project:
        H = material.project_psd(H)
    D = dF_dx(shape_gradients(Dminv))
    return vol[:, None, None] * np.einsum("epa,epq,eqb->eab", D, H, D)


def scatter_vector(tets, g_e, n_verts):
    """Sum per-tet 12-vectors into a [V,3] array."""
    out = np.zeros((n_verts, 3))
    g = g_e.reshape(-1, 4, 3)
    for a in range(4):
        np.add.at(out, tets[:, a], g[:, a])
    return out
