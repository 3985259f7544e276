"""Conforming adaptive refinement of a tet mesh by terminal-edge bisection,
driven by the contact sizing field of Sec. III-A (oracle, FP64, test
infrastructure; plain Python loops, small meshes only).

Sizing field h(p) (Sec. III-A): the thickness axis k is the thinnest
bounding-box axis; points within `band` x thickness of the contact face are
the contact band.  In the band a radial profile over the planar axes (u, v)
applies, with the radius normalised by the planar half-extents,
    rho = |((p_u - c_u) / h_u, (p_v - c_v) / h_v)|:
h = l_c for rho <= inner, l_g for rho >= inner + transition, and in between
the cosine blend h = l_g + (l_c - l_g) (1 + cos(pi (rho - inner) /
transition)) / 2.  Outside the band h = l_g.

The paper imposes the field inside WildMeshing's Delaunay optimisation;
here it drives bisection of a given conforming mesh (the reading of this
build), with h read as a cell size: edge ab is too long when
|x_a - x_b|^2 > 3 h(m)^2, m its midpoint (the body diagonal of a cube of
side h).

Procedure (its order fixes the result):
  edges are ordered by (squared length, smaller vertex id, larger vertex id);
  the longest edge of a tet is its largest in that order;
  tets are visited first-in first-out, starting with 0 .. T-1;
  while the visited tet t has a too-long edge:
      e = longest edge of t;
      walk: e' = the largest longest-edge among the tets sharing e;
            repeat with e = e' until e' == e (a terminal edge);
      bisect e = (a, b), a < b: new vertex m = 0.5 (x_a + x_b), appended;
      every tet s sharing e, in ascending index, keeps index s with b
      replaced by m, and a new tet (a replaced by m, same material) is
      appended; s and the new tet are queued in that order.
Bisection at the terminal edge keeps the mesh conforming and every tet
positively oriented.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np

_PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


class Sizing:
    def __init__(self, X, band=0.15, inner=0.4, transition=0.2, l_contact=0.8e-3, l_global=3.2e-3,
                 axis=-1, side=1, centre=None):
        lo, hi = X.min(axis=0), X.max(axis=0)
        ext = hi - lo
        self.k = int(np.argmin(ext)) if axis < 0 else int(axis)
        self.u, self.v = [i for i in range(3) if i != self.k]
        self.side = side
        self.lo, self.hi, self.H = lo, hi, ext[self.k]
        self.half = 0.5 * ext
        c = (0.5 * (lo + hi)) if centre is None else None
        self.cu = c[self.u] if centre is None else centre[0]
        self.cv = c[self.v] if centre is None else centre[1]
        self.band, self.inner, self.trans = band, inner, transition
        self.lc, self.lg = l_contact, l_global

    def h(self, p):
        depth = (self.hi[self.k] - p[self.k]) if self.side > 0 else (p[self.k] - self.lo[self.k])
        if depth > self.band * self.H:
            return self.lg
        du = (p[self.u] - self.cu) / self.half[self.u]
        dv = (p[self.v] - self.cv) / self.half[self.v]
        rho = math.sqrt(du * du + dv * dv)
        if rho <= self.inner:
            return self.lc
        if rho >= self.inner + self.trans:
            return self.lg
        w = 0.5 * (1.0 + math.cos(math.pi * (rho - self.inner) / self.trans))
        return self.lg + (self.lc - self.lg) * w


def refine(X, tets, sizing, mat=None, max_tets=1 << 22):
    """Returns (X [V',3], tets [T',4], mat [T'])."""
    X = [tuple(float(c) for c in p) for p in np.asarray(X, dtype=np.float64)]
    T = [list(map(int, t)) for t in np.asarray(tets)]
    M = list(map(int, mat)) if mat is not None else [0] * len(T)
    around = {}                       # edge (a, b), a < b -> set of tets

    def edges(t):
        q = T[t]
        return [(min(q[i], q[j]), max(q[i], q[j])) for i, j in _PAIRS]

    def add(t):
        for e in edges(t):
            around.setdefault(e, set()).add(t)

    def remove(t):
        for e in edges(t):
            around[e].discard(t)
            if not around[e]:
                del around[e]

    def len2(e):
        a, b = X[e[0]], X[e[1]]
        dx, dy, dz = a[0] - b[0], a[1] - b[1], a[2] - b[2]
        return dx * dx + dy * dy + dz * dz

    def key(e):
        return (len2(e), e[0], e[1])

    def longest(t):
        return max(edges(t), key=key)

    def too_long(e):
        a, b = X[e[0]], X[e[1]]
        m = (0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]), 0.5 * (a[2] + b[2]))
        h = sizing.h(m)
        return len2(e) > 3.0 * h * h

    for t in range(len(T)):
        add(t)
    queue = deque(range(len(T)))
    while queue:
        t = queue.popleft()
        while any(too_long(e) for e in edges(t)):
            e = longest(t)
            while True:
                nxt = max((longest(s) for s in around[e]), key=key)
                if nxt == e:
                    break
                e = nxt
            a, b = e
            pa, pb = X[a], X[b]
            X.append((0.5 * (pa[0] + pb[0]), 0.5 * (pa[1] + pb[1]), 0.5 * (pa[2] + pb[2])))
            m = len(X) - 1
            for s in sorted(around[e]):
                if len(T) >= max_tets:
                    raise ValueError("refinement exceeds max_tets")
                remove(s)
                old = T[s]
                T[s] = [m if v == b else v for v in old]
                T.append([m if v == a else v for v in old])
                M.append(M[s])
                add(s)
                add(len(T) - 1)
                queue.append(s)
                queue.append(len(T) - 1)
    return np.array(X), np.array(T, dtype=np.int32), np.array(M, dtype=np.int32)
