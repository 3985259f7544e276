"""Stress and force extraction (oracle, FP64, test infrastructure).

Alg. 2 (the stress step): sigma_i per tet from Eq. 4 (with the same rest shift as
the energy).  Alg. 1: per surface triangle j, from current vertex positions,
n_j = e1 x e2 / |e1 x e2|, sigma of the parent tet, t_j = sigma n_j (Eq. 6/7),
p_n = t . n (Eq. 8, positive = tension), t_tau = t - p_n n (Eq. 9).
Alg. 2 "Contact": f_k = -(contact gradient) / dt^2, i.e. -dE_b/dx_k; vertex
normal and area from the incident contact-face triangles, or for a vertex of
the side faces only from its incident surface triangles (current positions);
f_n = (f . n) n, f_tau = f - f_n, p_k = |f_k| / A_k; the indenter reaction is
-sum_k f_k.
"""
from __future__ import annotations

import numpy as np

from . import contact, fem, friction, material, mesh_pairs, surface


def cauchy_per_tet(pad, x):
    """Eq. 4 for every tet -> [T,3,3]."""
    F = fem.deformation_gradient(x, pad.tets, pad.Dminv)
    return material.cauchy(F, pad.mu, pad.lam, pad.alpha)


def surface_traction(pad, x, sigma):
    """Alg. 1 loop body for every surface triangle.
    Returns t [S,3], p_n [S], t_tau [S,3], n [S,3], current area [S]."""
    n, area = surface.tri_normals_areas(x, pad.tris)
    s = sigma[pad.parent]
    t = np.einsum("sij,sj->si", s, n)
    pn = np.einsum("si,si->s", t, n)
    t_tau = t - pn[:, None] * n
    return t, pn, t_tau, n, area


def contact_forces(pad, x, inds, prm, fric=None):
    """Alg. 2 contact path per candidate vertex: f_k = -g_k / dt^2 with g the
    step potential's contact gradient (barrier, plus friction when `fric`,
    the step's lagged friction data, is given).
    Returns dict of f, n, area, f_n, f_tau, p, reaction."""
    _, gb, _ = contact.barrier_terms(inds, x[pad.cand], pad.area, prm.dhat, prm.kappa,
                                     mesh_pairs=bool(prm.mesh_pairs))
    f = -gb
    for ind in inds:
        if prm.mesh_pairs == 2 and ind.shape == contact.MESH:
            # the mesh-vertex/pad-triangle and edge-edge pairs' forces on the
            # pad's contact vertices
            f = f - mesh_pairs.pair_terms(ind, x, pad.tris, pad.pedges, pad.pedge_len0, prm.dhat,
                                          prm.kappa)[1][pad.cand]
    if fric is not None:
        lagged, x_t_c = fric
        f = f - friction.terms(lagged, x[pad.cand], x_t_c, prm.mu_f, prm.eps_v * prm.dt, 1.0)[1]
    n, A = surface.contact_vertex_geometry(x, pad.tris, pad.is_top, pad.cand)
    fn = np.einsum("ki,ki->k", f, n)[:, None] * n
    ft = f - fn
    p = np.linalg.norm(f, axis=1) / A
    return dict(f=f, n=n, area=A, f_n=fn, f_tau=ft, p=p, reaction=-f.sum(axis=0))


def top_traction_sum(pad, x, sigma):
    """sum over contact-face triangles of t_j * (current area_j)."""
    t, _, _, _, area = surface_traction(pad, x, sigma)
    top = pad.is_top.astype(bool)
    return (t[top] * area[top, None]).sum(axis=0)
