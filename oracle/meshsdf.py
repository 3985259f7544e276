"""Signed distance to a closed rigid triangle mesh (oracle, FP64, test
infrastructure).

The paper's rigid objects (the Franka-held test objects of Sec. IV-D, and
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


def _pairs_block(mesh, y):
    """Closest point on every triangle for a block of points: distance [K,M],
    point [K,M,3], feature kind [K,M], feature id [K,M], edge direction
    [K,M,3] (zero unless kind is EDGE)."""
    K = y.shape[0]
    A, B, Cc = (mesh.V[mesh.F[:, k]][None] for k in range(3))          # [1,M,3]
    n = mesh.fn[None]
    Y = y[:, None, :]                                                   # [K,1,3]
    q = Y - np.einsum("kmi,kmi->km", Y - A, np.broadcast_to(n, (K,) + n.shape[1:]))[..., None] * n
    # barycentric coordinates of the projection onto each triangle's plane
    v0, v1 = B - A, Cc - A
    v2 = q - A
    d00 = np.einsum("kmi,kmi->km", v0, v0)
    d01 = np.einsum("kmi,kmi->km", v0, v1)
    d11 = np.einsum("kmi,kmi->km", v1, v1)
    d20 = np.einsum("kmi,kmi->km", v2, np.broadcast_to(v0, v2.shape))
    d21 = np.einsum("kmi,kmi->km", v2, np.broadcast_to(v1, v2.shape))
    den = d00 * d11 - d01 * d01
    l1 = (d11 * d20 - d01 * d21) / den
    l2 = (d00 * d21 - d01 * d20) / den
    inside = (l1 >= 0) & (l2 >= 0) & (l1 + l2 <= 1)
    M = mesh.F.shape[0]
    pt = q.copy()
    kind = np.full((K, M), FACE)
    fid = np.broadcast_to(np.arange(M)[None], (K, M)).copy()
    tdir = np.zeros((K, M, 3))
    # outside the triangle: nearest point over the three edge segments
    best = np.full((K, M), np.inf)
    corners = (A, B, Cc)
    for k in range(3):
        p0, p1 = corners[k], corners[(k + 1) % 3]
        e = p1 - p0
        t = np.clip(np.einsum("kmi,kmi->km", Y - p0, np.broadcast_to(e, (K,) + e.shape[1:]))
                    / np.einsum("kmi,kmi->km", e, e), 0.0, 1.0)
        pk = p0 + t[..., None] * e
        dk = np.linalg.norm(Y - pk, axis=2)
        better = (~inside) & (dk < best)
        best = np.where(better, dk, best)
        pt = np.where(better[..., None], pk, pt)
        vert = np.where(t <= 0.0, mesh.F[None, :, k], mesh.F[None, :, (k + 1) % 3])
        kk = np.where((t <= 0.0) | (t >= 1.0), VERTEX, EDGE)
        ii = np.where(kk == VERTEX, vert, mesh.tri_edge[None, :, k])
        kind = np.where(better, kk, kind)
        fid = np.where(better, ii, fid)
        ed = e / np.linalg.norm(e, axis=2, keepdims=True)
        tdir = np.where(better[..., None], np.broadcast_to(ed, tdir.shape), tdir)
    dist = np.linalg.norm(Y - pt, axis=2)
    return dist, pt, kind, fid, tdir


def _closest_block(mesh, y):
    """closest() for a block of points, all triangles at once ([K, M] pairs)."""
    dist, pt, kind, fid, tdir = _pairs_block(mesh, y)
    j = np.argmin(dist, axis=1)
    r = np.arange(y.shape[0])
    return dist[r, j], pt[r, j], kind[r, j], fid[r, j], tdir[r, j]


def closest(mesh, y, block=128):
    """For points y [K,3]: distance d, closest point c, feature kind, feature
    id (triangle, edge or vertex index) and, for edges, the edge direction.
    Every triangle is tried (brute force); the first of equal distances wins."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    parts = [_closest_block(mesh, y[i:i + block]) for i in range(0, y.shape[0], block)]
    return tuple(np.concatenate([p[k] for p in parts]) for k in range(5))


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


def pair_distances(mesh, y, dmax, block=128):
    """Every (point, triangle) pair nearer than dmax: the unsigned distance
    to the closed triangle and its derivatives in the mesh's frame.
    Returns (point index [P], triangle [P], d [P], grad [P,3], hess [P,3,3])
    with grad = (y - c) / d and hess = 0 (face), (I - t t^T - grad grad^T)
    / d (edge of direction t), (I - grad grad^T) / d (vertex): the distance
    to one triangle is C1 off the triangle, unlike the distance to the whole
    mesh, which has a kink on the bisector plane of every concave edge."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    out = []
    for i0 in range(0, y.shape[0], block):
        yb = y[i0:i0 + block]
        dist, pt, kind, _, tdir = _pairs_block(mesh, yb)
        ki, ti = np.nonzero(dist < dmax)
        d = dist[ki, ti]
        safe = np.where(d > 0, d, 1.0)
        g = (yb[ki] - pt[ki, ti]) / safe[:, None]
        I = np.eye(3)[None]
        gg = g[:, :, None] * g[:, None, :]
        t = tdir[ki, ti]
        tt = t[:, :, None] * t[:, None, :]
        k = kind[ki, ti]
        H = np.where((k == FACE)[:, None, None], 0.0, np.where((k == EDGE)[:, None, None], I - tt - gg, I - gg))
        out.append((ki + i0, ti, d, g, H / safe[:, None, None]))
    return tuple(np.concatenate([o[j] for o in out]) for j in range(5))
