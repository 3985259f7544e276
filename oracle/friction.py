"""Lagged smoothed Coulomb friction against the rigid indenters (oracle,
FP64, test infrastructure).

Sec. III-B configures the contact solver with a friction ratio (0.5) and a
velocity threshold eps_v (0.01 m/s).  The paper prints no formula; this is
the incremental-potential contact friction model that configuration names,
written per contact vertex k and indenter m:

  lagged at the start of the step (positions x_t, previous indenter pose):
      lambda_km = -kappa A_k b'(d_km / d_hat)     normal force magnitude [N]
      n_km      = grad(phi_m)(x_t,k)              contact normal
  the indenter's material point at x_t,k moves over the step by
      w_km = R_new R_old^T (x_t,k - c_old) + c_new - x_t,k
  relative tangential displacement over the step
      u_km = (I - n n^T) ((x_k - x_t,k) - w_km),  y = |u_km|
  dissipation potential, added to the step's potential with the same h^2
  weight as the elastic and barrier energies
      E_f = h^2 mu sum_km lambda_km f0(y),   eps = eps_v h  [m]
      f0(y) = -y^3 / (3 eps^2) + y^2 / eps + eps / 3   (y < eps),  y  (y >= eps)
      f1 = f0' :  -y^2 / eps^2 + 2 y / eps  (y < eps),   1  (y >= eps)
  gradient  h^2 mu lambda f1(y) u / y
  Hessian   h^2 mu lambda P [ f1(y)/y (I - uu^T/y^2) + f1'(y) uu^T/y^2 ] P,
            P = I - n n^T; PSD since f1 >= 0 and f1' >= 0 on [0, eps].
The contact force of Alg. 2 (f = -g / dt^2) then carries the friction force
-mu lambda f1(y) u / y, tangential to the lagged normal, of magnitude at most
mu lambda (Coulomb's bound, reached when sliding, y >= eps).
"""
from __future__ import annotations

import numpy as np

from . import contact


def f0(y, eps):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < eps, -y ** 3 / (3 * eps ** 2) + y ** 2 / eps + eps / 3, y)


def f1(y, eps):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < eps, -y ** 2 / eps ** 2 + 2 * y / eps, 1.0)


def f1_prime(y, eps):
    y = np.asarray(y, dtype=np.float64)
    return np.where(y < eps, -2 * y / eps ** 2 + 2 / eps, 0.0)


def f1_over_y(y, eps):
    """f1(y) / y, finite at y = 0 (limit 2 / eps)."""
    y = np.asarray(y, dtype=np.float64)
    safe = np.where(y > 0, y, 1.0)
    return np.where(y < eps, -y / eps ** 2 + 2 / eps, 1.0 / safe)


def indenter_motion(ind_old, ind_new, p):
    """Displacement over the step of the indenter material point at p."""
    R_old = np.asarray(ind_old.R, float)
    R_new = np.asarray(ind_new.R, float)
    local = (np.atleast_2d(p) - np.asarray(ind_old.c)[None]) @ R_old     # R_old^T (p - c_old)
    return local @ R_new.T + np.asarray(ind_new.c)[None] - p


def lag(inds_old, inds_new, x_t_c, area, dhat, kappa, mesh_pairs=False):
    """Per (indenter, candidate): lambda [M,C], n [M,C,3], w [M,C,3].
    lambda n is the barrier's contact force on the vertex at x_t under the
    previous pose: -kappa A b'(phi / d_hat) grad phi, or, for a rigid mesh
    with mesh_pairs, -kappa A sum_t b'(d_t / d_hat) grad d_t over the
    triangles within d_hat; lambda is its length and n its direction (a
    unit vector, so that I - n n^T projects)."""
    lam, nrm, w = [], [], []
    for old, new in zip(inds_old, inds_new):
        if mesh_pairs and old.shape == contact.MESH:
            _, g, _ = contact.barrier_terms([old], x_t_c, np.ones(len(x_t_c)), dhat, 1.0, project=False,
                                            mesh_pairs=True)
            mag = np.linalg.norm(g, axis=1)
            lam.append(kappa * area * mag)
            nrm.append(-g / np.where(mag > 0, mag, 1.0)[:, None])
        else:
            # the unit normal and the force's length: the texture plate's phi
            # is not a distance (|grad phi| < 1 off its extrema)
            phi, n, _ = contact.sdf(old, x_t_c)
            gn = np.linalg.norm(n, axis=1)
            lam.append(-kappa * area * contact.barrier_d1(phi / dhat) * gn)
            nrm.append(n / np.where(gn > 0, gn, 1.0)[:, None])
        w.append(indenter_motion(old, new, x_t_c))
    return np.array(lam), np.array(nrm), np.array(w)


def terms(lagged, x_c, x_t_c, mu, eps, h2):
    """Friction energy (scalar), gradient [C,3], Hessian [C,3,3]."""
    lam, nrm, w = lagged
    C = x_c.shape[0]
    E = 0.0
    g = np.zeros((C, 3))
    H = np.zeros((C, 3, 3))
    for m in range(lam.shape[0]):
        n = nrm[m]
        P = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
        rel = (x_c - x_t_c) - w[m]
        u = np.einsum("kij,kj->ki", P, rel)
        y = np.linalg.norm(u, axis=1)
        c = h2 * mu * lam[m]
        E += float(np.sum(c * f0(y, eps)))
        fy = f1_over_y(y, eps)
        g += (c * fy)[:, None] * u
        safe = np.where(y > 0, y, 1.0)
        uh = np.where((y > 0)[:, None], u / safe[:, None], 0.0)
        UU = uh[:, :, None] * uh[:, None, :]
        Hk = fy[:, None, None] * (np.eye(3)[None] - UU) + f1_prime(y, eps)[:, None, None] * UU
        H += c[:, None, None] * (P @ Hk @ P)
    return E, g, H
