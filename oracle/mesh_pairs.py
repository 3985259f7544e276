"""Rigid-mesh vertices against the pad's surface triangles, and rigid-mesh
edges against the pad's surface edges (oracle, FP64, test infrastructure).

Sec. III-B runs IPC contact between the pad and rigid objects.  IPC's
primitive pairs are point-triangle and edge-edge, both ways between two
surfaces.  With mesh_contact 2 a rigid mesh indenter adds, to the pad-vertex
against mesh-triangle pairs (contact.barrier_terms with mesh_pairs), the two
kinds whose pad side is a triangle or an edge (reading):

  vertex-face  kappa a_y d_hat b(d(y, t) / d_hat)
               y a mesh vertex, a_y a third of the area of its incident mesh
               triangles, t a pad surface triangle, d the distance from y to
               the closed triangle;
  edge-edge    kappa w d_hat m(c) b(d(e, f) / d_hat),  w = |e|_0 |f|_0 / 4
               e a mesh edge, f a pad surface edge (rest lengths), d the
               distance between the closed segments, c = |e x f|^2 and IPC's
               mollifier m(c) = (2 - c / c0) c / c0 below c0 = 1e-3 |e|_0^2
               |f|_0^2, 1 above: the term vanishes smoothly as the edges turn
               parallel, where their closest points stop being unique.

b is contact.barrier.  A mesh corner or edge can then no longer pass between
pad vertices unseen.  Gradients on the pad vertices follow from the envelope
theorem: with q = sum_a lam_a x_a the pad's closest point and u = (p - q) / d
the unit vector to the mesh's closest point p, dd/dx_a = -lam_a u.  For the
mollifier, dc/dx1 = 2 (|e|^2 f - (e.f) e) for c = |e x (x1 - x0)|^2, and its
negative at x0.  The Hessian is Gauss-Newton, w m b''(s) / d_hat
(grad d)(grad d)^T, positive semi-definite; the minimiser does not depend on
it.

Tunnelling: the indenter jumps to its new pose at every step, which can carry
a mesh corner or edge through a pad triangle or edge that the unsigned
distances above cannot see.  signed_pairs gives the pairs whose mesh feature
lies on the inner side of the pad surface within a window (the mesh's
travel over the step plus d_hat), which the feasible start pushes back.
"""
from __future__ import annotations

import numpy as np

from . import contact


def closest_on_triangles(y, a, b, c):
    """Distance from points y to the closed triangles (a, b, c) (all [N, 3])
    and the barycentric weights [N, 3] of the closest points.  The projection
    onto the plane when it falls inside the triangle, else the nearest of the
    clamped projections onto the three edges."""
    e0, e1, w = b - a, c - a, y - a
    d00 = np.einsum("ni,ni->n", e0, e0)
    d01 = np.einsum("ni,ni->n", e0, e1)
    d11 = np.einsum("ni,ni->n", e1, e1)
    d20 = np.einsum("ni,ni->n", w, e0)
    d21 = np.einsum("ni,ni->n", w, e1)
    den = d00 * d11 - d01 * d01
    u = (d11 * d20 - d01 * d21) / den
    v = (d00 * d21 - d01 * d20) / den
    lam = np.stack([1.0 - u - v, u, v], axis=1)
    inside = (u >= 0) & (v >= 0) & (u + v <= 1)
    q = a + u[:, None] * e0 + v[:, None] * e1
    dist = np.where(inside, np.linalg.norm(y - q, axis=1), np.inf)
    corners = (a, b, c)
    for k in range(3):
        p0, p1 = corners[k], corners[(k + 1) % 3]
        e = p1 - p0
        t = np.clip(np.einsum("ni,ni->n", y - p0, e) / np.einsum("ni,ni->n", e, e), 0.0, 1.0)
        dk = np.linalg.norm(y - (p0 + t[:, None] * e), axis=1)
        better = (~inside) & (dk < dist)
        dist = np.where(better, dk, dist)
        lk = np.zeros_like(lam)
        lk[:, k] = 1.0 - t
        lk[:, (k + 1) % 3] = t
        lam = np.where(better[:, None], lk, lam)
    return dist, lam


def closest_on_segments(p0, p1, q0, q1):
    """Distance between the closed segments p0p1 and q0q1 (all [N, 3]) and
    the parameters (s, t) of the closest points p0 + s (p1 - p0) and
    q0 + t (q1 - q0).  The squared distance is a convex quadratic over the
    unit square: its minimum is the interior stationary point when that lies
    in the square, else on one of the four sides, where the one-dimensional
    minimum is a clamped projection."""
    d1, d2, r = p1 - p0, q1 - q0, p0 - q0
    a = np.einsum("ni,ni->n", d1, d1)
    e = np.einsum("ni,ni->n", d2, d2)
    b = np.einsum("ni,ni->n", d1, d2)
    c = np.einsum("ni,ni->n", d1, r)
    f = np.einsum("ni,ni->n", d2, r)
    den = a * e - b * b
    safe = np.where(den > 1e-14 * a * e, den, 1.0)
    s_in = (b * f - c * e) / safe
    t_in = (a * f - b * c) / safe
    ok_in = (den > 1e-14 * a * e) & (s_in >= 0) & (s_in <= 1) & (t_in >= 0) & (t_in <= 1)
    cands = [(np.zeros_like(a), np.clip(f / e, 0, 1)), (np.ones_like(a), np.clip((b + f) / e, 0, 1)),
             (np.clip(-c / a, 0, 1), np.zeros_like(a)), (np.clip((b - c) / a, 0, 1), np.ones_like(a))]
    best = np.full(a.shape, np.inf)
    s_best, t_best = np.zeros_like(a), np.zeros_like(a)

    def dist(s, t):
        return np.linalg.norm(r + s[:, None] * d1 - t[:, None] * d2, axis=1)

    dd = np.where(ok_in, dist(np.where(ok_in, s_in, 0), np.where(ok_in, t_in, 0)), np.inf)
    best = np.where(ok_in, dd, best)
    s_best, t_best = np.where(ok_in, s_in, s_best), np.where(ok_in, t_in, t_best)
    for s, t in cands:
        dk = dist(s, t)
        better = dk < best
        best = np.where(better, dk, best)
        s_best = np.where(better, s, s_best)
        t_best = np.where(better, t, t_best)
    return best, s_best, t_best


def mollifier(c, c0):
    """IPC's edge-edge mollifier and its derivative dm/dc."""
    x = c / c0
    m = np.where(x < 1.0, (2.0 - x) * x, 1.0)
    dm = np.where(x < 1.0, (2.0 - 2.0 * x) / c0, 0.0)
    return m, dm


def surface_edges(tris):
    """Unique edges of the surface triangles, sorted (i < j), ascending."""
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0).astype(np.int64)


def mesh_tables(V, F):
    """A rigid mesh's vertex areas (a third of the incident triangle areas)
    and unique edges (local frame)."""
    V = np.asarray(V, dtype=np.float64)
    F = np.asarray(F, dtype=np.int64)
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1)
    va = np.zeros(V.shape[0])
    for k in range(3):
        np.add.at(va, F[:, k], area / 3.0)
    return va, surface_edges(F)


def _world(ind):
    V, F = ind.mesh
    R = np.asarray(ind.R, dtype=np.float64)
    return np.asarray(V, dtype=np.float64) @ R.T + np.asarray(ind.c)[None], np.asarray(F, dtype=np.int64)


def _near_boxes(P, lo, hi, dmax):
    """Index pairs (i, j) with point P[i] within dmax of the box [lo_j, hi_j]
    in every coordinate: a superset of the pairs nearer than dmax (a point
    farther than dmax from a feature's bounding box is farther from the
    feature), taken in order of i, then j."""
    if not np.isfinite(dmax):
        return np.repeat(np.arange(P.shape[0]), lo.shape[0]), np.tile(np.arange(lo.shape[0]), P.shape[0])
    near = np.all((P[:, None, :] >= lo[None] - dmax) & (P[:, None, :] <= hi[None] + dmax), axis=2)
    return np.nonzero(near)


def vf_pairs(Yw, x, tris, dmax):
    """Every (mesh vertex, pad triangle) pair nearer than dmax:
    (vertex [P], triangle [P], d [P], lam [P, 3], u [P, 3])."""
    corners = x[tris]
    iv, it = _near_boxes(Yw, corners.min(axis=1), corners.max(axis=1), dmax)
    d, lam = closest_on_triangles(Yw[iv], x[tris[it, 0]], x[tris[it, 1]], x[tris[it, 2]])
    keep = d < dmax
    iv, it, d, lam = iv[keep], it[keep], d[keep], lam[keep]
    q = np.einsum("pk,pki->pi", lam, x[tris[it]])
    u = (Yw[iv] - q) / np.where(d > 0, d, 1.0)[:, None]     # touching pairs (d = 0): no direction
    return iv, it, d, lam, u


def ee_pairs(Yw, medges, x, pedges, dmax):
    """Every (mesh edge, pad edge) pair nearer than dmax:
    (mesh edge [P], pad edge [P], d [P], s [P], t [P], u [P, 3])."""
    # the closest point of the mesh edge lies within dmax of the pad edge's
    # box, so some point of the mesh edge does: test the mesh edge's box
    # against the pad edge's box grown by dmax
    ends = x[pedges]
    elo, ehi = Yw[medges].min(axis=1), Yw[medges].max(axis=1)
    flo, fhi = ends.min(axis=1), ends.max(axis=1)
    if np.isfinite(dmax):
        near = np.all((elo[:, None, :] <= fhi[None] + dmax) & (ehi[:, None, :] >= flo[None] - dmax), axis=2)
        ie, jf = np.nonzero(near)
    else:
        ie = np.repeat(np.arange(medges.shape[0]), pedges.shape[0])
        jf = np.tile(np.arange(pedges.shape[0]), medges.shape[0])
    p0, p1 = Yw[medges[ie, 0]], Yw[medges[ie, 1]]
    q0, q1 = x[pedges[jf, 0]], x[pedges[jf, 1]]
    d, s, t = closest_on_segments(p0, p1, q0, q1)
    keep = d < dmax
    ie, jf, d, s, t = ie[keep], jf[keep], d[keep], s[keep], t[keep]
    p = Yw[medges[ie, 0]] + s[:, None] * (Yw[medges[ie, 1]] - Yw[medges[ie, 0]])
    q = x[pedges[jf, 0]] + t[:, None] * (x[pedges[jf, 1]] - x[pedges[jf, 0]])
    u = (p - q) / np.where(d > 0, d, 1.0)[:, None]
    return ie, jf, d, s, t, u


def pair_terms(ind, x, tris, pedges, pedge_len0, dhat, kappa):
    """Energy, gradient [V, 3] and Gauss-Newton Hessian blocks of the
    vertex-face and edge-edge pairs of one rigid mesh indenter at pad
    positions x.  Blocks: (rows [B], cols [B], 3x3 values [B, 3, 3]) in vertex
    indices, to be scattered into the assembled Hessian."""
    V0, F = ind.mesh
    va, medges = mesh_tables(V0, F)
    Yw, _ = _world(ind)
    E = 0.0
    g = np.zeros_like(x)
    rows, cols, vals = [], [], []
    # vertex-face
    iv, it, d, lam, u = vf_pairs(Yw, x, tris, dhat)
    s = d / dhat
    w = kappa * va[iv]
    E += float(np.sum(w * dhat * contact.barrier(s)))
    b1, b2 = contact.barrier_d1(s), contact.barrier_d2(s)
    for a in range(3):
        np.add.at(g, tris[it, a], (w * b1)[:, None] * (-lam[:, a:a + 1] * u))
    uu = u[:, :, None] * u[:, None, :]
    for a in range(3):
        for c in range(3):
            rows.append(tris[it, a])
            cols.append(tris[it, c])
            vals.append((w * b2 / dhat * lam[:, a] * lam[:, c])[:, None, None] * uu)
    # edge-edge
    len_e = np.linalg.norm(V0[medges[:, 1]] - V0[medges[:, 0]], axis=1)
    ie, jf, d, sp, tp, u = ee_pairs(Yw, medges, x, pedges, dhat)
    s = d / dhat
    ev = Yw[medges[ie, 1]] - Yw[medges[ie, 0]]
    fv = x[pedges[jf, 1]] - x[pedges[jf, 0]]
    cr = np.cross(ev, fv)
    cc = np.einsum("pi,pi->p", cr, cr)
    c0 = 1e-3 * len_e[ie] ** 2 * pedge_len0[jf] ** 2
    m, dm = mollifier(cc, c0)
    w = kappa * 0.25 * len_e[ie] * pedge_len0[jf]
    bb = contact.barrier(s)
    b1, b2 = contact.barrier_d1(s), contact.barrier_d2(s)
    E += float(np.sum(w * dhat * m * bb))
    # d c / d x1 = 2 (|e|^2 f - (e.f) e), d c / d x0 = -(the same)
    ee = np.einsum("pi,pi->p", ev, ev)
    ef = np.einsum("pi,pi->p", ev, fv)
    dc1 = 2.0 * (ee[:, None] * fv - ef[:, None] * ev)
    lam = np.stack([1.0 - tp, tp], axis=1)
    for a, sign in ((0, -1.0), (1, 1.0)):
        gd = -lam[:, a:a + 1] * u                       # d d / d x_a
        ga = (w * dhat)[:, None] * (dm[:, None] * bb[:, None] * sign * dc1 + (m * b1 / dhat)[:, None] * gd)
        np.add.at(g, pedges[jf, a], ga)
    uu = u[:, :, None] * u[:, None, :]
    for a in range(2):
        for c in range(2):
            rows.append(pedges[jf, a])
            cols.append(pedges[jf, c])
            vals.append((w * m * b2 / dhat * lam[:, a] * lam[:, c])[:, None, None] * uu)
    if rows:
        return E, g, (np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
    return E, g, (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3, 3)))


def _advance(dist_at, d0, pm, span=1.0):
    """Conservative advancement per pair (reading): every point of the
    moving pad feature moves at most alpha pm, so the pair's distance
    d(alpha) is Lipschitz with constant pm, and from a reached alpha the step
    (d(alpha) - 0.1 d0) / pm keeps it above 0.1 d0.  Advances until within
    0.1 % of that floor, 32 advances, or span; dist_at(alpha, mask) gives the
    distances of the masked pairs at their alphas."""
    al = np.zeros_like(d0)
    dc = d0.copy()
    floor = 0.1 * d0
    live = (pm > 0) & (d0 > 0)
    for _ in range(32):
        if not live.any():
            break
        al = np.where(live, al + (dc - floor) / np.where(pm > 0, pm, 1.0), al)
        hit = live & (al >= span)
        al = np.where(hit, span, al)
        live &= ~hit
        if not live.any():
            break
        dc = np.where(live, dist_at(al, live), dc)
        live &= dc - floor > 1e-3 * floor
    al = np.where(pm > 0, al, np.inf)
    return np.where(d0 > 0, al, 0.0)


def _separation_bound(d, pm, sep, pu):
    """With u the unit vector between a pair's closest points, sep = min
    over the mesh feature of w.u - max over the pad feature's vertices of
    x_a.u is the features' separation along u, a lower bound on their
    distance for any positions, and it shrinks at most by alpha pu with pu =
    max_a p_a.u: alpha <= 0.9 sep / pu keeps the pair apart (no bound when
    pu <= 0), whatever the motion across u."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(sep > 0, np.where(pu > 0, 0.9 * sep / pu, np.inf), 0.0)


def step_bound(ind, x, p, tris, pedges):
    """Largest safe step fraction (at most 1) for the pad's surface
    triangles and edges moving by alpha p against the rigid mesh: per pair
    the larger of two safe bounds (reading), conservative advancement
    (_advance) and the separation along the pair direction
    (_separation_bound); the minimum over all pairs."""
    V0, F = ind.mesh
    _, medges = mesh_tables(V0, F)
    Yw, _ = _world(ind)
    pn = np.linalg.norm(p, axis=1)
    a = 1.0
    big = np.inf
    iv, it, d, _, u = vf_pairs(Yw, x, tris, big)
    if iv.size:
        def vf_at(al, m):
            xa = x[tris[it]] + al[:, None, None] * p[tris[it]]
            return closest_on_triangles(Yw[iv], xa[:, 0], xa[:, 1], xa[:, 2])[0]
        sep = np.einsum("pi,pi->p", Yw[iv], u) - np.einsum("pki,pi->pk", x[tris[it]], u).max(axis=1)
        pu = np.einsum("pki,pi->pk", p[tris[it]], u).max(axis=1)
        ca = _advance(vf_at, d, pn[tris].max(axis=1)[it])
        a = min(a, float(np.min(np.maximum(ca, _separation_bound(d, None, sep, pu)))))
    ie, jf, d, _, _, u = ee_pairs(Yw, medges, x, pedges, big)
    if ie.size:
        def ee_at(al, m):
            xa = x[pedges[jf]] + al[:, None, None] * p[pedges[jf]]
            return closest_on_segments(Yw[medges[ie, 0]], Yw[medges[ie, 1]], xa[:, 0], xa[:, 1])[0]
        sep = np.einsum("pki,pi->pk", Yw[medges[ie]], u).min(axis=1) - np.einsum("pki,pi->pk", x[pedges[jf]], u).max(axis=1)
        pu = np.einsum("pki,pi->pk", p[pedges[jf]], u).max(axis=1)
        ca = _advance(ee_at, d, pn[pedges].max(axis=1)[jf])
        a = min(a, float(np.min(np.maximum(ca, _separation_bound(d, None, sep, pu)))))
    return a


def signed_pairs(ind, x, tris, pedges, window, below=0.0):
    """Pairs whose mesh feature sits on the inner side of the pad surface
    (tunnelled through it by the indenter's jump to its new pose), or less
    than `below` outside it, within `window` of it: vertex-face pairs whose
    closest point is inside the triangle, signed along its outward normal;
    edge-edge pairs with both closest points inside their segments, signed
    along the pad edge's outward direction (the sum of the normals of the
    pad triangles sharing the edge).  A pair counts only when the vector
    between its closest points lies within 60 degrees of the primitive's
    normal line (|signed distance| >= d / 2, always true for a vertex over
    a triangle's interior): next to a pad edge or corner, a mesh feature
    above one surface region can sit behind the plane of a neighbouring
    one (a side face's plane extends above the top face) without being
    inside the pad (reading).  Returns a list of
    (pad vertex ids [k], outward unit normal [3], signed distance,
    primitive) with primitive = triangle index for vertex-face pairs and
    number of triangles + edge index for edge-edge pairs."""
    V0, F = ind.mesh
    _, medges = mesh_tables(V0, F)
    Yw, _ = _world(ind)
    out = []
    iv, it, d, lam, _ = vf_pairs(Yw, x, tris, window)
    a, b, c = x[tris[it, 0]], x[tris[it, 1]], x[tris[it, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1)[:, None]
    sd = np.einsum("pi,pi->p", Yw[iv] - a, n)
    interior = (lam > 0).all(axis=1) & (np.abs(sd) >= 0.5 * d)
    for k in np.nonzero(interior & (sd < below))[0]:
        out.append((tris[it[k]], n[k], float(sd[k]), int(it[k])))
    # outward direction of each pad edge: sum of its triangles' normals
    tn = np.cross(x[tris[:, 1]] - x[tris[:, 0]], x[tris[:, 2]] - x[tris[:, 0]])
    tn /= np.linalg.norm(tn, axis=1)[:, None]
    key = {tuple(e): i for i, e in enumerate(pedges)}
    en = np.zeros((pedges.shape[0], 3))
    for t in range(tris.shape[0]):
        for k in range(3):
            e = tuple(sorted((int(tris[t, k]), int(tris[t, (k + 1) % 3]))))
            en[key[e]] += tn[t]
    en /= np.linalg.norm(en, axis=1)[:, None]
    ie, jf, d, s, t, _ = ee_pairs(Yw, medges, x, pedges, window)
    p = Yw[medges[ie, 0]] + s[:, None] * (Yw[medges[ie, 1]] - Yw[medges[ie, 0]])
    q = x[pedges[jf, 0]] + t[:, None] * (x[pedges[jf, 1]] - x[pedges[jf, 0]])
    sd = np.einsum("pi,pi->p", p - q, en[jf])
    interior = (s > 0) & (s < 1) & (t > 0) & (t < 1) & (np.abs(sd) >= 0.5 * d)
    for k in np.nonzero(interior & (sd < below))[0]:
        out.append((pedges[jf[k]], en[jf[k]], float(sd[k]), tris.shape[0] + int(jf[k])))
    return out
