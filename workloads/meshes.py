"""Synthetic gel-pad meshes (seeded input generators).

The paper meshes each sensor elastomer with a third-party tetrahedraliser
(Sec. III-A) whose sensor CAD is not available here.  These structured
stand-ins produce (V, T) arrays of the same shape class: a tensor-product
grid of hexahedral cells, each split into six tetrahedra along the common
main diagonal (Kuhn/Freudenthal split), so the mesh is conforming.

Everything in this module is input generation: node coordinates and
connectivity.  No part of the method (stress, contact, solve, extraction)
lives here; both the oracle and the GPU library receive these arrays as
plain inputs.

Units are metres throughout.
"""
from __future__ import annotations

import numpy as np

# The six monotone corner paths 000 -> 111 of a unit cube, one per
# permutation of the axes.  Each tet is the path
#   c, c + e[p0], c + e[p0] + e[p1], c + (1,1,1).
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))
# Odd permutations give a negatively oriented path; swapping the last two
# path vertices restores det(Dm) > 0.
ODD = (False, True, True, False, False, True)


def node_id(i, j, k, nx, ny):
    """Node (i, j, k) of an nx x ny x nz cell grid -> global vertex id."""
    return i + (nx + 1) * (j + (ny + 1) * k)


def kuhn_grid(xs, ys, zs):
    """Tensor-product grid with node coordinates xs (nx+1), ys, zs.

    Returns (X float64 [V,3], tets int32 [T,4]) with
      vertex id = i + (nx+1)(j + (ny+1) k)
      tet id    = 6 * cell + p,  cell = i + nx (j + ny k)
    """
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    zs = np.asarray(zs, dtype=np.float64)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    if min(nx, ny, nz) < 1:
        raise ValueError("grid needs at least one cell per axis")
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1),
                          np.arange(nx + 1), indexing="ij")
    X = np.stack([xs[I.ravel()], ys[J.ravel()], zs[K.ravel()]], axis=1)

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    ncell = ci.size
    tets = np.empty((ncell, 6, 4), dtype=np.int64)
    for p, perm in enumerate(PERMS):
        corner = np.zeros((ncell, 3), dtype=np.int64)
        path = [corner.copy()]
        for ax in perm:
            corner[:, ax] += 1
            path.append(corner.copy())
        ids = [node_id(ci + c[:, 0], cj + c[:, 1], ck + c[:, 2], nx, ny)
               for c in path]
        if ODD[p]:
            ids[2], ids[3] = ids[3], ids[2]
        tets[:, p, :] = np.stack(ids, axis=1)
    return X, tets.reshape(-1, 4).astype(np.int32)


def uniform_axis(length, n):
    """n equal cells over [0, length]."""
    return np.linspace(0.0, float(length), int(n) + 1)


def geometric_ratio(total, first, n):
    """Ratio r with first * (r**n - 1) / (r - 1) = total (bisection)."""
    if abs(first * n - total) <= 1e-15 * total:
        return 1.0
    lo, hi = (1.0 + 1e-15, 10.0) if first * n < total else (1e-6, 1.0 - 1e-15)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = first * (mid ** n - 1.0) / (mid - 1.0)
        if (s < total) == (first * n < total):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def graded_axis_top(length, n, top):
    """n layers over [0, length]; the top layer is `top` thick and layers
    grow geometrically downward (refinement toward the contact face)."""
    r = geometric_ratio(length, top, n)
    widths = top * r ** np.arange(n)          # widths[0] is the top layer
    zs_top_down = length - np.concatenate([[0.0], np.cumsum(widths)])
    zs = zs_top_down[::-1].copy()
    zs[0] = 0.0
    zs[-1] = float(length)
    return zs


def dome_map(X, thickness, cap_radius, centre_xy):
    """Stretch each vertical column so the top becomes a spherical cap.

    z' = z * (H + cap(x, y)) / H, cap = sqrt(Rc^2 - rho^2) - sqrt(Rc^2 - rho_max^2),
    rho = planar distance to the pad centre, rho_max = its maximum over the
    pad (so the cap is zero at the farthest corner)."""
    X = np.array(X, dtype=np.float64, copy=True)
    rho = np.hypot(X[:, 0] - centre_xy[0], X[:, 1] - centre_xy[1])
    rho_max = rho.max()
    cap = np.sqrt(cap_radius ** 2 - rho ** 2) - np.sqrt(cap_radius ** 2 - rho_max ** 2)
    X[:, 2] = X[:, 2] * (thickness + cap) / thickness
    return X


def cylinder_map(X, thickness, cap_radius, centre_x):
    """Stretch each vertical column so the top becomes a cylindrical cap
    curved along x (axis along y):

    z' = z * (H + cap(x)) / H, cap = sqrt(Rc^2 - u^2) - sqrt(Rc^2 - u_max^2),
    u = x - centre_x, u_max = its largest magnitude over the pad (so the cap
    is zero at the two curved edges)."""
    X = np.array(X, dtype=np.float64, copy=True)
    u = X[:, 0] - centre_x
    u_max = np.abs(u).max()
    cap = np.sqrt(cap_radius ** 2 - u ** 2) - np.sqrt(cap_radius ** 2 - u_max ** 2)
    X[:, 2] = X[:, 2] * (thickness + cap) / thickness
    return X


def cells_for_target(Lx, Ly, Lz, target_tets):
    """Cell counts nx:ny:nz ~ Lx:Ly:(2 Lz) closest to target_tets / 6."""
    cells = target_tets / 6.0
    s = (cells / (Lx * Ly * 2.0 * Lz)) ** (1.0 / 3.0)
    return (max(1, int(round(s * Lx))), max(1, int(round(s * Ly))),
            max(1, int(round(s * 2.0 * Lz))))


def sizing_profile_axis(length, centre, h_f, inner=0.4, band=0.2, ratio=8.0,
                        levels=(1.0, 2.0, 4.0, 8.0)):
    """1-D node positions whose spacing follows the radial sizing profile of
    the contact-refinement rule: fine spacing h_f inside `inner` x half-extent
    of the centre, coarse spacing ratio*h_f outside inner+band, cosine blend
    in the band, quantised to the nearest level (in log2) of h_f*levels.

    Nodes are marched outward from `centre` in both directions and the last
    cell on each side is stretched/shrunk to land on 0 and `length`."""
    half = 0.5 * length
    r_c, r_t = inner * half, band * half
    lv = np.asarray(levels)

    def spacing(r):
        if r <= r_c:
            q = 1.0
        elif r >= r_c + r_t:
            q = ratio
        else:
            t = (r - r_c) / r_t
            q = 1.0 + (ratio - 1.0) * 0.5 * (1.0 - np.cos(np.pi * t))
        return h_f * lv[np.argmin(np.abs(np.log2(lv) - np.log2(q)))]

    def march(limit):
        pts, r = [], 0.0
        while True:
            h = spacing(r)
            if r + h >= limit - 0.5 * h:
                pts.append(limit)
                return pts
            r += h
            pts.append(r)

    right = [centre + r for r in march(length - centre)]
    left = [centre - r for r in march(centre)]
    xs = np.unique(np.array(left + [centre] + right, dtype=np.float64))
    xs[0], xs[-1] = 0.0, float(length)
    return xs


def fan_prisms(n, radius, height, nz):
    """A disc pad of n triangular prism sectors around its vertical axis,
    nz layers, each prism split into 3 tets conformingly (each quad face
    cut by the diagonal through its smallest vertex index, Dompierre et
    al. 1999).  The axis vertices touch every sector: a row of the assembled
    Hessian with about 2n blocks.  Returns (X [V,3], tets [T,4])."""
    th = 2 * np.pi * np.arange(n) / n
    X = []
    for k in range(nz + 1):
        z = height * k / nz
        X.append([0.0, 0.0, z])
        X += [[radius * np.cos(t), radius * np.sin(t), z] for t in th]
    X = np.array(X)

    def vid(k, j):
        return k * (n + 1) + j

    def split(a, b):
        m = int(np.argmin(a + b))
        if m >= 3:
            a, b, m = b, a, m - 3
        a, b = a[m:] + a[:m], b[m:] + b[:m]
        (a0, a1, a2), (b0, b1, b2) = a, b
        if min(a1, b2) < min(a2, b1):
            return [[a0, a1, a2, b2], [a0, a1, b2, b1], [a0, b1, b2, b0]]
        return [[a0, a1, a2, b1], [a0, b1, a2, b2], [a0, b1, b2, b0]]
    T = []
    for k in range(nz):
        for i in range(n):
            j = (i + 1) % n
            T += split([vid(k, 0), vid(k, 1 + i), vid(k, 1 + j)], [vid(k + 1, 0), vid(k + 1, 1 + i), vid(k + 1, 1 + j)])
    T = np.array(T, np.int64)
    e1, e2, e3 = (X[T[:, c]] - X[T[:, 0]] for c in (1, 2, 3))
    neg = np.einsum("ij,ij->i", np.cross(e1, e2), e3) < 0
    T[neg] = T[neg][:, [0, 2, 1, 3]]
    return X, T.astype(np.int32)


# ----------------------------------------------------------------------------
# closed triangle surfaces for rigid mesh indenters (local frame, outward
# counter-clockwise triangles, every edge shared by exactly two triangles)

def box_surface(a, b, c):
    """Box of half extents (a, b, c): 8 vertices, 12 triangles."""
    V = np.array([[sx * a, sy * b, sz * c] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)], float)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    F = []
    for q in quads:
        F += [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
    return V, np.array(F, np.int32)


def cylinder_surface(r, a, n):
    """Closed cylinder about the local z axis (radius r, half length a): an
    n-gon prism with vertices on the circle, caps fanned from their centres."""
    th = 2 * np.pi * np.arange(n) / n
    ring = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    V = np.concatenate([np.column_stack([ring, np.full(n, -a)]), np.column_stack([ring, np.full(n, a)]),
                        [[0.0, 0.0, -a], [0.0, 0.0, a]]])
    F = []
    for i in range(n):
        j = (i + 1) % n
        F += [(i, j, n + j), (i, n + j, n + i), (2 * n, j, i), (2 * n + 1, n + i, n + j)]
    return V, np.array(F, np.int32)


def icosphere(r, level):
    """Sphere of radius r: icosahedron subdivided `level` times, vertices
    pushed to the sphere."""
    t = (1 + 5 ** 0.5) / 2
    V = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = [np.array(v, float) / np.linalg.norm(v) for v in V]
    for _ in range(level):
        mid = {}

        def midpoint(i, j):
            key = (min(i, j), max(i, j))
            if key not in mid:
                m = V[i] + V[j]
                V.append(m / np.linalg.norm(m))
                mid[key] = len(V) - 1
            return mid[key]
        G = []
        for a, b, c in F:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            G += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = G
    return r * np.array(V), np.array(F, np.int32)


def torus_surface(R, r, nu, nv, phase=0.0):
    """Torus about the local z axis (ring radius R, tube radius r), nu x nv
    quads split into triangles; the tube polygon starts `phase` segments
    round (0.5 puts a facet, not a polygon edge, at the bottom)."""
    V = []
    for i in range(nu):
        u = 2 * np.pi * i / nu
        for j in range(nv):
            v = 2 * np.pi * (j + phase) / nv
            V.append(((R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)))
    F = []
    for i in range(nu):
        for j in range(nv):
            a = i * nv + j
            b = ((i + 1) % nu) * nv + j
            c = ((i + 1) % nu) * nv + (j + 1) % nv
            d = i * nv + (j + 1) % nv
            F += [(a, b, c), (a, c, d)]
    return np.array(V, float), np.array(F, np.int32)
