"""Stable Neo-Hookean constitutive law (oracle, FP64, test infrastructure).

Eq. 1: Lame parameters from (E, nu).
Eq. 2: first Piola stress P = mu F + lambda (J - alpha) J F^-T.  As printed the
       shift is alpha = 1, which leaves a rest stress P(I) = mu I; the
       rest-stable shift alpha = 1 + mu / lambda gives P(I) = 0.  Both are
       available; the default is the rest-stable one.
Energy density whose derivative is Eq. 2:
       Psi(F) = mu/2 (tr F^T F - 3) + lambda/2 (J - alpha)^2.
Eq. 3: sigma = J^-1 P F^T;  Eq. 4: sigma = (mu / J) F F^T + lambda (J - alpha) I.

All functions take stacks of 3x3 matrices F[..., 3, 3] (row index i, column j).
The 9x9 Hessians use the row-major flattening vec(F)[3 i + j] = F[i, j].
"""
from __future__ import annotations

import numpy as np


def lame(E, nu):
    """Eq. 1: mu = E / (2 (1 + nu)), lambda = E nu / ((1 + nu)(1 - 2 nu))."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam


def rest_shift(mu, lam, literal=False):
    """alpha in (J - alpha): 1 as printed in Eq. 2, else 1 + mu / lambda."""
    return 1.0 if literal else 1.0 + mu / lam


def cofactor(F):
    """cof F = J F^-T, columns = cross products of the columns of F."""
    f0, f1, f2 = F[..., :, 0], F[..., :, 1], F[..., :, 2]
    return np.stack([np.cross(f1, f2), np.cross(f2, f0), np.cross(f0, f1)], axis=-1)


def det(F):
    return np.linalg.det(F)


def _m(a):
    """Per-tet scalar -> broadcastable against [..., 3, 3]."""
    return np.asarray(a, dtype=np.float64)[..., None, None]


def energy_density(F, mu, lam, alpha):
    """Psi(F) = mu/2 (||F||_F^2 - 3) + lambda/2 (J - alpha)^2."""
    J = det(F)
    return 0.5 * mu * (np.sum(F * F, axis=(-2, -1)) - 3.0) + 0.5 * lam * (J - alpha) ** 2


def first_piola(F, mu, lam, alpha):
    """Eq. 2: P = mu F + lambda (J - alpha) cof F, with cof F = J F^-T."""
    J = det(F)
    return _m(mu) * F + _m(lam * (J - alpha)) * cofactor(F)


# Levi-Civita symbol
EPS = np.zeros((3, 3, 3))
for _i, _j, _k in ((0, 1, 2), (1, 2, 0), (2, 0, 1)):
    EPS[_i, _j, _k] = 1.0
    EPS[_i, _k, _j] = -1.0


def det_hessian(F):
    """d^2 J / dF_ij dF_kl = sum_{n,q} eps_ikn eps_jlq F_nq, as 9x9."""
    H = np.einsum("ikn,jlq,...nq->...ijkl", EPS, EPS, F)
    return H.reshape(F.shape[:-2] + (9, 9))


def energy_hessian(F, mu, lam, alpha):
    """d^2 Psi / dF^2 = mu I_9 + lambda vec(cof F) vec(cof F)^T
                        + lambda (J - alpha) d^2 J / dF^2   (9x9, unprojected)."""
    J = det(F)
    g = cofactor(F).reshape(F.shape[:-2] + (9,))
    H = _m(mu) * np.eye(9) + _m(lam) * g[..., :, None] * g[..., None, :]
    return H + _m(lam * (J - alpha)) * det_hessian(F)


def project_psd(H):
    """Symmetric eigen-decomposition, negative eigenvalues clamped to zero."""
    w, Q = np.linalg.eigh(0.5 * (H + np.swapaxes(H, -1, -2)))
    return (Q * np.maximum(w, 0.0)[..., None, :]) @ np.swapaxes(Q, -1, -2)


def cauchy_from_piola(F, mu, lam, alpha):
    """Eq. 3: sigma = J^-1 P F^T."""
    J = det(F)
    return first_piola(F, mu, lam, alpha) @ np.swapaxes(F, -1, -2) / J[..., None, None]


def cauchy(F, mu, lam, alpha):
    """Eq. 4: sigma = (mu / J) b + lambda (J - alpha) I, b = F F^T."""
    J = det(F)
    b = F @ np.swapaxes(F, -1, -2)
    return _m(mu / J) * b + _m(lam * (J - alpha)) * np.eye(3)
