"""Surface topology and per-vertex setup (oracle, FP64, test infrastructure).

Alg. 1 (surface extraction) (Sec. III-C-2): extract the boundary triangles of the tet
mesh and the parent tetrahedron of each.  Sec. III-A: the thinnest bounding
box axis is the pad thickness and a 15 % thickness band marks the contact
surface (here the face opposite the fixed base; see `contact_face_labels`).
"""
from __future__ import annotations

import numpy as np

# Outward faces of a positively oriented tet (v0, v1, v2, v3): each face is
# listed so that (b - a) x (c - a) points away from the opposite vertex.
LOCAL_FACES = ((1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1))


def surface_triangles(tets):
    """Alg. 1 (surface extraction).  A face is on the surface iff its vertex set occurs
    in exactly one tet.  Returns (tris int32 [S,3] with outward winding,
    parent int32 [S]) in ascending (tet id, local face) order."""
    tets = np.asarray(tets, dtype=np.int64)
    T = tets.shape[0]
    faces = np.stack([tets[:, list(f)] for f in LOCAL_FACES], axis=1)  # T,4,3
    flat = faces.reshape(-1, 3)
    key = np.sort(flat, axis=1)
    _, inverse, counts = np.unique(key, axis=0, return_inverse=True,
                                   return_counts=True)
    once = counts[inverse.ravel()] == 1
    idx = np.nonzero(once)[0]          # ascending = (tet, face) order
    tris = flat[idx].astype(np.int32)
    parent = (idx // 4).astype(np.int32)
    return tris, parent


def thickness_axis(X):
    """Sec. III-A: the thinnest bounding-box axis is the thickness."""
    ext = X.max(axis=0) - X.min(axis=0)
    return int(np.argmin(ext)), ext


def default_fixed(X):
    """Base of the pad (minimum along the thickness axis) fully fixed:
    per-vertex xyz bitmask, 7 = all three components fixed."""
    a, ext = thickness_axis(X)
    lo = X[:, a].min()
    base = X[:, a] <= lo + 1e-9 * ext[a]
    return np.where(base, 7, 0).astype(np.uint8)


def tri_normals_areas(P, tris):
    """Unit normal (e1 x e2 / |e1 x e2|) and area of each triangle."""
    v0, v1, v2 = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    c = np.cross(v1 - v0, v2 - v0)
    L = np.linalg.norm(c, axis=1)
    return c / L[:, None], 0.5 * L


def contact_face_labels(X, tris):
    """Contact surface (Sec. III-A labels the face of the pad that meets
    objects, located along the thinnest bounding-box axis): here the surface
    triangles whose rest outward normal has a component >= 0.5 along the
    thickness axis, on the side opposite the fixed base.  On flat pads this is
    exactly the top face (the 15 % thickness band of the sizing rule selects
    the same triangles); on domed pads it keeps the whole cap."""
    a, _ = thickness_axis(X)
    n, _ = tri_normals_areas(X, tris)
    return (n[:, a] >= 0.5).astype(np.uint8)


def candidates(tris, fixed, n_verts):
    """Contact vertices of Alg. 2 and barrier candidates (Sec. III-B runs the
    IPC barrier over the pad's surface): every vertex of a surface triangle
    with at least one free component, ascending id.  Vertices of the side
    faces are included, so an indenter that reaches past the contact face
    still meets a barrier."""
    on_face = np.zeros(n_verts, dtype=bool)
    on_face[np.asarray(tris).ravel()] = True
    return np.nonzero(on_face & (np.asarray(fixed) != 7))[0].astype(np.int32)


def vertex_areas(P, tris, verts):
    """A_k = 1/3 of the summed areas of the given triangles incident to k."""
    _, area = tri_normals_areas(P, tris)
    acc = np.zeros(P.shape[0])
    for c in range(3):
        np.add.at(acc, tris[:, c], area / 3.0)
    return acc[verts]


def vertex_normals(P, tris, verts):
    """Area-weighted unit normal at each vertex: normalised sum of the given
    incident triangles' e1 x e2, whose length is twice the triangle's area."""
    v0, v1, v2 = P[tris[:, 0]], P[tris[:, 1]], P[tris[:, 2]]
    c = np.cross(v1 - v0, v2 - v0)
    acc = np.zeros_like(P)
    for k in range(3):
        np.add.at(acc, tris[:, k], c)
    n = acc[verts]
    return n / np.linalg.norm(n, axis=1)[:, None]


def contact_vertex_tris(tris, is_top, verts, n_verts):
    """The triangles whose share a contact vertex takes (its barrier weight
    at rest, and Alg. 2's vertex normal and area): the incident
    contact-face triangles for a vertex on the contact face, else all its
    incident surface triangles (a vertex of the side faces only).  Returns a
    boolean mask [len(verts)] of the vertices on the contact face."""
    top = np.asarray(is_top).astype(bool)
    on_top = np.zeros(n_verts, dtype=bool)
    on_top[np.asarray(tris)[top].ravel()] = True
    return on_top[verts]


def contact_vertex_geometry(P, tris, is_top, verts):
    """Unit normal and area of each contact vertex from the triangles
    `contact_vertex_tris` gives it (positions P)."""
    tris = np.asarray(tris)
    top = np.asarray(is_top).astype(bool)
    sel = contact_vertex_tris(tris, is_top, verts, P.shape[0])
    A = vertex_areas(P, tris, verts)
    n = np.zeros((len(verts), 3))
    if (~sel).any():
        n[~sel] = vertex_normals(P, tris, verts[~sel])
    if sel.any():
        A[sel] = vertex_areas(P, tris[top], verts[sel])
        n[sel] = vertex_normals(P, tris[top], verts[sel])
    return n, A


def lumped_mass(X, tets, density):
    """m_a = sum over tets e containing a of density * V_e / 4."""
    Dm = np.stack([X[tets[:, k]] - X[tets[:, 0]] for k in (1, 2, 3)], axis=2)
    vol = np.linalg.det(Dm) / 6.0
    m = np.zeros(X.shape[0])
    for k in range(4):
        np.add.at(m, tets[:, k], density * vol / 4.0)
    return m
