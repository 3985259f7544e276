"""IPC log barrier against analytic rigid indenters (oracle, FP64).

Sec. III-B configures the incremental-potential contact solver with a barrier
distance threshold d_hat.  The barrier itself is IPC's clamped log barrier,
written here per candidate vertex k against indenter signed distance d_k:

    b(s)  = -(s - 1)^2 ln s   for 0 < s < 1,   0 for s >= 1,   +inf for s <= 0
    E_b   = kappa * sum_k A_k d_hat b(d_k / d_hat)          (kappa in Pa)
    dE_b/dx_k   = kappa A_k b'(s) grad(phi)
    d2E_b/dx_k2 = kappa A_k [ b''(s) / d_hat grad(phi) grad(phi)^T + b'(s) hess(phi) ]

Indenters are rigid: local coordinates y = R^T (x - c).  Signed distances
(local frame, solid on the negative side):
    sphere   |y| - r
    cylinder axis z, radius r, half-height a: q = (|y_xy| - r, |y_z| - a),
             phi = |max(q, 0)| + min(max(q_x, q_y), 0)
    box      half extents a: q = |y| - a, phi = |max(q, 0)| + min(max_i q_i, 0)
    torus    axis z: |(|y_xy| - R_t, y_z)| - r_t
    texture  plate occupying y_z >= eta(y_x, y_y), eta = A sin(k y_x) sin(k y_y),
             k = 2 pi / lambda:  phi = (eta - y_z) / sqrt(1 + (k A)^2)
             (a 1-Lipschitz lower bound of the distance).
    mesh     closed triangle mesh (V, F) in the local frame: signed distance
             to its surface (meshsdf).
"""
from __future__ import annotations

import numpy as np

from . import meshsdf

SPHERE, CYLINDER, BOX, TORUS, TEXTURE, MESH = 0, 1, 2, 3, 4, 5

_MESHES = {}


def _mesh_data(mesh):
    """Tables of a rigid mesh indenter's (V, F), built once per mesh object."""
    hit = _MESHES.get(id(mesh))
    if hit is None or hit[0] is not mesh:
        hit = (mesh, meshsdf.MeshData(*mesh))
        _MESHES[id(mesh)] = hit
    return hit[1]


def barrier(s):
    """b(s) = -(s-1)^2 ln s on (0,1); 0 for s >= 1; inf for s <= 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    inside = (s > 0) & (s < 1)
    si = s[inside]
    out[inside] = -(si - 1.0) ** 2 * np.log(si)
    out[s <= 0] = np.inf
    return out


def barrier_d1(s):
    """b'(s) = -2 (s-1) ln s - (s-1)^2 / s on (0,1), else 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    m = (s > 0) & (s < 1)
    si = s[m]
    out[m] = -2.0 * (si - 1.0) * np.log(si) - (si - 1.0) ** 2 / si
    return out


def barrier_d2(s):
    """b''(s) = -2 ln s - 4 (s-1)/s + (s-1)^2 / s^2 on (0,1), else 0."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    m = (s > 0) & (s < 1)
    si = s[m]
    out[m] = -2.0 * np.log(si) - 4.0 * (si - 1.0) / si + (si - 1.0) ** 2 / si ** 2
    return out


def _radial_frame(y):
    rho = np.hypot(y[:, 0], y[:, 1])
    safe = np.where(rho > 0, rho, 1.0)
    e_rho = np.stack([y[:, 0] / safe, y[:, 1] / safe, np.zeros_like(rho)], axis=1)
    e_rho[rho == 0] = (1.0, 0.0, 0.0)
    Ixy = np.diag([1.0, 1.0, 0.0])
    # Hessian of rho = |y_xy|
    H_rho = (Ixy[None] - e_rho[:, :, None] * e_rho[:, None, :]) / safe[:, None, None]
    return rho, e_rho, H_rho


def _outer(a, b):
    return a[:, :, None] * b[:, None, :]


def sdf_local(shape, prm, y):
    """phi [N], grad [N,3], hess [N,3,3] in the indenter's local frame."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    N = y.shape[0]
    if shape == SPHERE:
        r = prm[0]
        L = np.linalg.norm(y, axis=1)
        n = y / L[:, None]
        H = (np.eye(3)[None] - _outer(n, n)) / L[:, None, None]
        return L - r, n, H
    if shape == CYLINDER:
        r, a = prm[0], prm[1]
        rho, e_rho, H_rho = _radial_frame(y)
        sz = np.where(y[:, 2] >= 0, 1.0, -1.0)
        e_z = np.stack([np.zeros(N), np.zeros(N), sz], axis=1)
        qx, qy = rho - r, np.abs(y[:, 2]) - a
        phi = np.empty(N); g = np.empty((N, 3)); H = np.zeros((N, 3, 3))
        edge = (qx > 0) & (qy > 0)
        side = (qx > 0) & ~edge
        cap = (qy > 0) & ~edge
        inner = ~(edge | side | cap)
        if edge.any():
            L = np.hypot(qx[edge], qy[edge])
            er, ez = e_rho[edge], e_z[edge]
            phi[edge] = L
            g[edge] = (qx[edge, None] * er + qy[edge, None] * ez) / L[:, None]
            prr = (qy[edge] ** 2 / L ** 3)[:, None, None]
            pzz = (qx[edge] ** 2 / L ** 3)[:, None, None]
            prz = (-qx[edge] * qy[edge] / L ** 3)[:, None, None]
            H[edge] = (prr * _outer(er, er) + pzz * _outer(ez, ez)
                       + prz * (_outer(er, ez) + _outer(ez, er))
                       + (qx[edge] / L)[:, None, None] * H_rho[edge])
        for m, radial in ((side, True), (cap, False)):
            if m.any():
                phi[m] = qx[m] if radial else qy[m]
                g[m] = e_rho[m] if radial else e_z[m]
                H[m] = H_rho[m] if radial else 0.0
        if inner.any():
            radial = qx[inner] >= qy[inner]
            phi[inner] = np.maximum(qx[inner], qy[inner])
            g[inner] = np.where(radial[:, None], e_rho[inner], e_z[inner])
            H[inner] = np.where(radial[:, None, None], H_rho[inner], 0.0)
        return phi, g, H
    if shape == BOX:
        a = np.asarray(prm[:3], dtype=np.float64)
        s = np.where(y >= 0, 1.0, -1.0)
        q = np.abs(y) - a[None]
        pos = q > 0
        npos = pos.sum(axis=1)
        phi = np.empty(N); g = np.zeros((N, 3)); H = np.zeros((N, 3, 3))
        out = npos >= 2
        if out.any():
            qp = np.where(pos[out], q[out], 0.0)
            L = np.linalg.norm(qp, axis=1)
            n = qp * s[out] / L[:, None]
            P = np.zeros((out.sum(), 3, 3))
            for i in range(3):
                P[:, i, i] = pos[out][:, i]
            phi[out] = L
            g[out] = n
            H[out] = (P - _outer(n, n)) / L[:, None, None]
        one = ~out
        if one.any():
            i = np.argmax(q[one], axis=1)
            rows = np.nonzero(one)[0]
            phi[one] = q[rows, i]
            g[rows, i] = s[rows, i]
        return phi, g, H
    if shape == TORUS:
        Rt, rt = prm[0], prm[1]
        rho, e_rho, H_rho = _radial_frame(y)
        w0, w1 = rho - Rt, y[:, 2]
        L = np.hypot(w0, w1)
        e_z = np.tile(np.array([0.0, 0.0, 1.0]), (N, 1))
        g = (w0[:, None] * e_rho + w1[:, None] * e_z) / L[:, None]
        prr = (w1 ** 2 / L ** 3)[:, None, None]
        pzz = (w0 ** 2 / L ** 3)[:, None, None]
        prz = (-w0 * w1 / L ** 3)[:, None, None]
        H = (prr * _outer(e_rho, e_rho) + pzz * _outer(e_z, e_z)
             + prz * (_outer(e_rho, e_z) + _outer(e_z, e_rho))
             + (w0 / L)[:, None, None] * H_rho)
        return L - rt, g, H
    if shape == TEXTURE:
        A, lam = prm[0], prm[1]
        k = 2.0 * np.pi / lam
        c = np.sqrt(1.0 + (k * A) ** 2)
        sx, cx = np.sin(k * y[:, 0]), np.cos(k * y[:, 0])
        sy, cy = np.sin(k * y[:, 1]), np.cos(k * y[:, 1])
        eta = A * sx * sy
        ex, ey = A * k * cx * sy, A * k * sx * cy
        exx, eyy, exy = -k * k * eta, -k * k * eta, A * k * k * cx * cy
        g = np.stack([ex, ey, -np.ones(N)], axis=1) / c
        H = np.zeros((N, 3, 3))
        H[:, 0, 0], H[:, 1, 1] = exx / c, eyy / c
        H[:, 0, 1] = H[:, 1, 0] = exy / c
        return (eta - y[:, 2]) / c, g, H
    raise ValueError(f"unknown indenter shape {shape}")


def sdf(ind, x):
    """World-frame phi, grad, hess for indenter `ind` (shape, prm, R, c)."""
    R = np.asarray(ind.R, dtype=np.float64)
    y = (np.atleast_2d(x) - np.asarray(ind.c)[None]) @ R     # = R^T (x - c)
    if ind.shape == MESH:
        phi, g, H = meshsdf.sdf_local(_mesh_data(ind.mesh), y)
    else:
        phi, g, H = sdf_local(ind.shape, ind.prm, y)
    return phi, g @ R.T, R[None] @ H @ R.T[None]


def barrier_terms(indenters, x_c, area, dhat, kappa, project=True, mesh_pairs=False):
    """Barrier energy (scalar), gradient [C,3] and Hessian [C,3,3] of E_b over
    candidate positions x_c with rest areas `area`, summed over indenters.
    The per-vertex 3x3 Hessian is PSD-projected (eigenvalues clamped at 0)
    unless project=False.

    mesh_pairs: a rigid mesh's barrier is summed over its triangles nearer
    than d_hat, kappa A_k d_hat sum_t b(d_t / d_hat) with d_t the distance to
    triangle t (IPC's point-triangle pairs, Sec. III-B), instead of taken at
    the distance to the whole mesh."""
    C = x_c.shape[0]
    E = 0.0
    g = np.zeros((C, 3))
    H = np.zeros((C, 3, 3))
    for ind in indenters:
        if mesh_pairs and ind.shape == MESH:
            R = np.asarray(ind.R, dtype=np.float64)
            y = (x_c - np.asarray(ind.c)[None]) @ R
            k, _, d, gl, Hl = meshsdf.pair_distances(_mesh_data(ind.mesh), y, dhat)
            s = d / dhat
            w = kappa * area[k]
            b1, b2 = barrier_d1(s), barrier_d2(s)
            n = gl @ R.T
            E += float(np.sum(w * dhat * barrier(s)))
            np.add.at(g, k, (w * b1)[:, None] * n)
            np.add.at(H, k, w[:, None, None] * ((b2 / dhat)[:, None, None] * _outer(n, n)
                                                + b1[:, None, None] * (R[None] @ Hl @ R.T[None])))
            continue
        phi, n, Hphi = sdf(ind, x_c)
        s = phi / dhat
        E += float(np.sum(kappa * area * dhat * barrier(s)))
        b1, b2 = barrier_d1(s), barrier_d2(s)
        g += (kappa * area * b1)[:, None] * n
        H += (kappa * area)[:, None, None] * ((b2 / dhat)[:, None, None] * _outer(n, n)
                                              + b1[:, None, None] * Hphi)
    if not project:
        return E, g, H
    w, Q = np.linalg.eigh(H)
    Hp = (Q * np.maximum(w, 0.0)[:, None, :]) @ np.swapaxes(Q, 1, 2)
    return E, g, Hp
