"""Signed distance to a closed rigid triangle mesh (oracle, FP64, test
infrastructure).

The paper's rigid objects (the Franka-held test objects of Sec. IV-E, and
the rigid bodies of the contact solver of Sec. III-B) are triangle meshes.
Against a rigid mesh the contact measure of a pad vertex is its distance to
the mesh surface, which this module computes by brute force:

  d(y) = min over triangles T of dist(y, T)
  closest point on T: the projection of y onto T's plane when it falls
  inside T (face), else the nearest point over T's three edge segments
  (edge interior, or an end point = vertex);
  sign s = +1 outside, -1 inside, from the angle-weighted pseudonormal of the
  closest feature (Baerentzen and Aanaes, IEEE TVCG 2005): face normal, sum
  of the two face normals at an edge, angle-weighted sum at a vertex;
  phi = s d,  grad phi = s (y - c) / d   (c the closest point),
  hess phi = 0 (face), s (I - t t^T - grad grad^T) / d (edge of direction
  t), s (I - grad grad^T) / d (vertex).

The mesh must be closed and consistently oriented with outward normals
(counter-clockwise seen from outside).
"""
from __future__ import annotations

import numpy as np

FACE, EDGE, VERTEX = 0, 1, 2


class MeshData:
    """Per-mesh tables: edge ids per triangle, pseudonormals."""

    def __init__(self, V, F):
        self.V = np.asarray(V, dtype=np.float64)
        self.F = np.asarray(F, dtype=np.int64)
        a, b, c = (self.V[self.F[:, k]] for k in range(3))
        cr = np.cross(b - a, c - a)
        self.fn = cr / np.linalg.norm(cr, axis=1)[:, None]
        edges = {}
        self.tri_edge = np.zeros((len(self.F), 3), np.int64)   # edge k joins corners k, k+1
        for t, tri in enumerate(self.F):
            for k in range(3):
                key = (min(tri[k], tri[(k + 1) % 3]), max(tri[k], tri[(k + 1) % 3]))
                self.tri_edge[t, k] = edges.setdefault(key, len(edges))
        self.edge_n = np.zeros((len(edges), 3))
        for t in range(len(self.F)):
            for k in range(3):
                self.edge_n[self.tri_edge[t, k]] += self.fn[t]
        self.vert_n = np.zeros_like(self.V)
        for t, tri in enumerate(self.F):
            for k in range(3):
                p, q, r = self.V[tri[k]], self.V[tri[(k + 1) % 3]], self.V[tri[(k + 2) % 3]]
                u, w = q - p, r - p
                ang = np.arccos(np.clip(u @ w / (np.linalg.norm(u) * np.linalg.norm(w)), -1.0, 1.0))
                self.vert_n[tri[k]] += ang * self.fn[t]


def _segment(y, p0, p1):
    """Nearest point on segments p0-p1 to points y (all [K,3]): point, t."""
    e = p1 - p0
    t = np.clip(np.einsum("ki,ki->k", y - p0, e) / np.einsum("ki,ki->k", e, e), 0.0, 1.0)
    return p0 + t[:, None] * e, t


def closest(mesh, y):
    """For points y [K,3]: distance d, closest point c, feature kind, feature
    id (triangle, edge or vertex index) and, for edges, the edge direction."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    K = y.shape[0]
    best = np.full(K, np.inf)
    cp = np.zeros((K, 3))
    kind = np.zeros(K, np.int64)
    fid = np.zeros(K, np.int64)
    tdir = np.zeros((K, 3))
    for t, tri in enumerate(mesh.F):
        a, b, c = mesh.V[tri[0]], mesh.V[tri[1]], mesh.V[tri[2]]
        n = mesh.fn[t]
        q = y - np.outer((y - a) @ n, n)
        # barycentric coordinates of the projection
        v0, v1, v2 = b - a, c - a, q - a
        d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
        d20, d21 = v2 @ v0, v2 @ v1
        den = d00 * d11 - d01 * d01
        l1 = (d11 * d20 - d01 * d21) / den
        l2 = (d00 * d21 - d01 * d20) / den
        inside = (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
        pt = q.copy()
        knd = np.full(K, FACE)
        idx = np.full(K, t)
        dr = np.zeros((K, 3))
        if not inside.all():
            out = ~inside
            yo = y[out]
            bd = np.full(yo.shape[0], np.inf)
            bp = np.zeros_like(yo)
            bk = np.zeros(yo.shape[0], np.int64)
            bi = np.zeros(yo.shape[0], np.int64)
            bdir = np.zeros_like(yo)
            corners = (a, b, c)
            for k in range(3):
                p0, p1 = corners[k], corners[(k + 1) % 3]
                P0 = np.broadcast_to(p0, yo.shape)
                P1 = np.broadcast_to(p1, yo.shape)
                pk, s = _segment(yo, P0, P1)
                dk = np.linalg.norm(yo - pk, axis=1)
                better = dk < bd
                bd = np.where(better, dk, bd)
                bp[better] = pk[better]
                at0, at1 = s <= 0.0, s >= 1.0
                kk = np.where(at0 | at1, VERTEX, EDGE)
                ii = np.where(at0, tri[k], np.where(at1, tri[(k + 1) % 3], mesh.tri_edge[t, k]))
                bk = np.where(better, kk, bk)
                bi = np.where(better, ii, bi)
                e = (p1 - p0) / np.linalg.norm(p1 - p0)
                bdir[better] = e
            pt[out], knd[out], idx[out], dr[out] = bp, bk, bi, bdir
        dist = np.linalg.norm(y - pt, axis=1)
        better = dist < best
        best = np.where(better, dist, best)
        cp[better], kind[better], fid[better], tdir[better] = pt[better], knd[better], idx[better], dr[better]
    return best, cp, kind, fid, tdir


def sdf_local(mesh, y):
    """phi [K], grad [K,3], hess [K,3,3] in the mesh's frame."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    d, c, kind, fid, tdir = closest(mesh, y)
    N = np.where((kind == FACE)[:, None], mesh.fn[np.where(kind == FACE, fid, 0)],
                 np.where((kind == EDGE)[:, None], mesh.edge_n[np.minimum(np.where(kind == EDGE, fid, 0),
                                                                           len(mesh.edge_n) - 1)],
                          mesh.vert_n[np.where(kind == VERTEX, fid, 0)]))
    diff = y - c
    s = np.where(np.einsum("ki,ki->k", diff, N) >= 0, 1.0, -1.0)
    safe = np.where(d > 0, d, 1.0)
    g = s[:, None] * diff / safe[:, None]
    I = np.eye(3)[None]
    gg = g[:, :, None] * g[:, None, :]
    tt = tdir[:, :, None] * tdir[:, None, :]
    H = np.where((kind == FACE)[:, None, None], 0.0,
                 np.where((kind == EDGE)[:, None, None], I - tt - gg, I - gg))
    H = (s / safe)[:, None, None] * H
    return s * d, g, H
