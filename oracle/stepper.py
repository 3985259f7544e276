"""One implicit incremental-potential step and its Newton minimiser
(oracle, FP64, test infrastructure).

Sec. III-B / Alg. 2 (the physics step): the pad advances by minimising, over the
free degrees of freedom,

    E(x) = 1/2 sum_a m_a |x_a - xhat_a|^2 + h^2 [ sum_e V_e Psi(F_e) + E_b(x) ],
    xhat = x_t + h v_t + h^2 g,

with the fixed components held at their rest positions.  The h^2 factor on
the potential is the one Alg. 2 undoes when it turns the contact gradient
into a force (f = -g / dt^2).  `quasi_static` drops the inertia term.

The minimiser (the paper caps Newton at 1024 iterations per step):
  1. initial guess x_t; any candidate closer than 0.1 d_hat to an indenter is
     pushed out along grad(phi) (at most 8 rounds; failure = infeasible);
  2. Newton direction p from the PSD-projected Hessian (sparse direct solve);
     converged when ||p||_inf <= tol * (rest bounding-box diagonal), in which
     case the filtered step is taken without a line search;
  3. step filter alpha <= 0.9 d_k / |p_k| for every candidate (valid because
     every distance function here is 1-Lipschitz);
  4. Armijo backtracking E(x + a p) <= E(x) + 1e-4 a g.p + 1e-12 |E(x)|, at
     most 40 halvings (the last term admits energy changes below what a
     float64 sum over the mesh resolves);
  5. x += a p.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import contact, fem, friction, material, mesh_pairs, surface


ENERGY_NOISE = 1e-12


class Infeasible(RuntimeError):
    pass


class LineSearchFailure(RuntimeError):
    pass


class NotConverged(RuntimeError):
    pass


@dataclasses.dataclass
class OraclePad:
    X: np.ndarray
    tets: np.ndarray
    mu: np.ndarray          # per tet
    lam: np.ndarray
    alpha: np.ndarray
    density: float
    Dminv: np.ndarray
    vol: np.ndarray
    mass: np.ndarray
    fixed: np.ndarray       # per-vertex xyz bitmask
    tris: np.ndarray
    parent: np.ndarray
    is_top: np.ndarray
    cand: np.ndarray
    area: np.ndarray        # rest areas of the candidates (surface.contact_vertex_geometry)
    pedges: np.ndarray      # surface edges (i < j), for rigid-mesh edge-edge pairs
    pedge_len0: np.ndarray  # their rest lengths
    L_diag: float
    free: np.ndarray        # [V,3] bool
    x: np.ndarray           # committed state
    v: np.ndarray


def make_pad(X, tets, E, nu, density, fixed=None, literal_alpha=False):
    """Setup: Eq. 1 Lame parameters, rest data, mass, surface (Alg. 1 1-3)."""
    X = np.asarray(X, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int32)
    T = tets.shape[0]
    E = np.broadcast_to(np.asarray(E, dtype=np.float64), (T,)).copy()
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (T,)).copy()
    mu, lam = material.lame(E, nu)
    alpha = np.array([material.rest_shift(m, l, literal_alpha) for m, l in zip(mu, lam)])
    Dminv, vol = fem.rest_data(X, tets)
    mass = surface.lumped_mass(X, tets, density)
    fixed = surface.default_fixed(X) if fixed is None else np.asarray(fixed, np.uint8)
    tris, parent = surface.surface_triangles(tets)
    is_top = surface.contact_face_labels(X, tris)
    cand = surface.candidates(tris, fixed, X.shape[0])
    area = surface.contact_vertex_geometry(X, tris, is_top, cand)[1]
    L = float(np.linalg.norm(X.max(axis=0) - X.min(axis=0)))
    free = np.stack([(fixed >> b) & 1 == 0 for b in range(3)], axis=1)
    pedges = mesh_pairs.surface_edges(tris)
    plen = np.linalg.norm(X[pedges[:, 1]] - X[pedges[:, 0]], axis=1)
    return OraclePad(X, tets, mu, lam, alpha, density, Dminv, vol, mass, fixed,
                     tris, parent, is_top, cand, area, pedges, plen, L, free, X.copy(), np.zeros_like(X))


@dataclasses.dataclass
class StepParams:
    dt: float = 1.0 / 60.0
    dhat: float = 1e-4
    kappa: float = 1e3
    newton_tol: float = 1e-6
    max_newton: int = 1024
    quasi_static: bool = False
    gravity: tuple = (0.0, 0.0, 0.0)
    max_halvings: int = 40
    mu_f: float = 0.0        # friction ratio (0 = frictionless)
    eps_v: float = 0.01      # friction velocity threshold [m/s]
    mesh_pairs: int = 0      # rigid meshes: 0 distance to the mesh; 1 barrier summed over the triangles
                             # nearer than d_hat; 2 that plus mesh-vertex/pad-triangle and edge-edge pairs


@dataclasses.dataclass
class StepResult:
    x: np.ndarray
    v: np.ndarray
    newton_iters: int
    energies: List[float]
    fric: object = None      # lagged friction data of the step (None: frictionless)


def friction_lag(pad, inds, prm, inds_prev=None):
    """Lagged friction data of a step from the committed state x_t and the
    previous indenter poses (None when friction is off)."""
    if prm.mu_f <= 0:
        return None
    prev = inds if inds_prev is None else inds_prev
    return (friction.lag(prev, inds, pad.x[pad.cand], pad.area, prm.dhat, prm.kappa,
                         mesh_pairs=bool(prm.mesh_pairs)),
            pad.x[pad.cand].copy())


def _friction(pad, x, prm, fric):
    lagged, x_t_c = fric
    return friction.terms(lagged, x[pad.cand], x_t_c, prm.mu_f, prm.eps_v * prm.dt, prm.dt ** 2)


def _pair_meshes(inds, prm):
    """Rigid mesh indenters that take the mesh-vertex/pad-triangle and
    edge-edge pairs (mesh_contact 2)."""
    return [ind for ind in inds if prm.mesh_pairs == 2 and ind.shape == contact.MESH]


def _pairs(pad, x, ind, prm):
    return mesh_pairs.pair_terms(ind, x, pad.tris, pad.pedges, pad.pedge_len0, prm.dhat, prm.kappa)


def energy(pad, x, xhat, inds, prm, fric=None):
    """E(x) of the incremental potential (inf if a candidate penetrates)."""
    h2 = prm.dt ** 2
    Eel = float(np.sum(fem.elastic_energy(x, pad.tets, pad.Dminv, pad.vol,
                                          pad.mu, pad.lam, pad.alpha)))
    Eb, _, _ = contact.barrier_terms(inds, x[pad.cand], pad.area, prm.dhat, prm.kappa,
                                     mesh_pairs=bool(prm.mesh_pairs))
    for ind in _pair_meshes(inds, prm):
        Eb += _pairs(pad, x, ind, prm)[0]
    Ein = 0.0 if prm.quasi_static else 0.5 * float(np.sum(pad.mass[:, None] * (x - xhat) ** 2))
    Ef = _friction(pad, x, prm, fric)[0] if fric is not None else 0.0
    return Ein + h2 * (Eel + Eb) + Ef


def gradient(pad, x, xhat, inds, prm, fric=None):
    """dE/dx as [V,3] (fixed components included, not masked)."""
    h2 = prm.dt ** 2
    ge = fem.elastic_gradient(x, pad.tets, pad.Dminv, pad.vol, pad.mu, pad.lam, pad.alpha)
    g = h2 * fem.scatter_vector(pad.tets, ge, x.shape[0])
    _, gb, _ = contact.barrier_terms(inds, x[pad.cand], pad.area, prm.dhat, prm.kappa,
                                     mesh_pairs=bool(prm.mesh_pairs))
    g[pad.cand] += h2 * gb
    for ind in _pair_meshes(inds, prm):
        g += h2 * _pairs(pad, x, ind, prm)[1]
    if fric is not None:
        g[pad.cand] += _friction(pad, x, prm, fric)[1]
    if not prm.quasi_static:
        g += pad.mass[:, None] * (x - xhat)
    return g


def hessian(pad, x, inds, prm, project=True, fric=None):
    """Assembled (3V x 3V) sparse Hessian of E; element and barrier parts
    PSD-projected unless project=False (then the exact Hessian)."""
    h2 = prm.dt ** 2
    V = x.shape[0]
    Ke = fem.elastic_hessian(x, pad.tets, pad.Dminv, pad.vol, pad.mu, pad.lam,
                             pad.alpha, project=project)
    dof = (3 * pad.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    rows = np.repeat(dof, 12, axis=1).ravel()
    cols = np.tile(dof, (1, 12)).ravel()
    vals = h2 * Ke.ravel()
    _, _, Hb = contact.barrier_terms(inds, x[pad.cand], pad.area, prm.dhat, prm.kappa, project=project,
                                     mesh_pairs=bool(prm.mesh_pairs))
    cd = (3 * pad.cand[:, None] + np.arange(3)[None, :])
    rows = np.concatenate([rows, np.repeat(cd, 3, axis=1).ravel()])
    cols = np.concatenate([cols, np.tile(cd, (1, 3)).ravel()])
    vals = np.concatenate([vals, h2 * Hb.ravel()])
    for ind in _pair_meshes(inds, prm):
        # Gauss-Newton blocks of the pairs (positive semi-definite)
        bi, bj, bv = _pairs(pad, x, ind, prm)[2]
        ri = (3 * bi[:, None, None] + np.arange(3)[None, :, None]) + 0 * np.arange(3)[None, None, :]
        ci = (3 * bj[:, None, None] + np.arange(3)[None, None, :]) + 0 * np.arange(3)[None, :, None]
        rows = np.concatenate([rows, ri.ravel()])
        cols = np.concatenate([cols, ci.ravel()])
        vals = np.concatenate([vals, h2 * bv.ravel()])
    if fric is not None:
        Hf = _friction(pad, x, prm, fric)[2]
        rows = np.concatenate([rows, np.repeat(cd, 3, axis=1).ravel()])
        cols = np.concatenate([cols, np.tile(cd, (1, 3)).ravel()])
        vals = np.concatenate([vals, Hf.ravel()])
    if not prm.quasi_static:
        d = np.arange(3 * V)
        rows = np.concatenate([rows, d])
        cols = np.concatenate([cols, d])
        vals = np.concatenate([vals, np.repeat(pad.mass, 3)])
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * V, 3 * V))


def candidate_distances(pad, x, inds):
    """min over indenters of phi at every candidate."""
    d = np.full(pad.cand.shape[0], np.inf)
    for ind in inds:
        phi, _, _ = contact.sdf(ind, x[pad.cand])
        d = np.minimum(d, phi)
    return d


def _travel(ind, ind_prev):
    """Largest displacement of a rigid mesh's vertices from the previous
    pose to this one."""
    if ind_prev is None:
        return 0.0
    V = np.asarray(ind.mesh[0], dtype=np.float64)
    a = V @ np.asarray(ind.R).T + np.asarray(ind.c)[None]
    b = V @ np.asarray(ind_prev.R).T + np.asarray(ind_prev.c)[None]
    return float(np.linalg.norm(a - b, axis=1).max())


def feasible_start(pad, x, inds, prm, inds_prev=None):
    """Initial guess: push candidates closer than 0.1 d_hat out along
    grad(phi), free components only, at most 8 rounds.  With mesh_contact 2,
    pad triangles and edges that a rigid mesh's vertex or edge came through
    (or nearer than 0.1 d_hat to, on their inner side) within the mesh's
    travel since the previous pose plus d_hat are pushed back along their
    outward normal in the same rounds (reading): a primitive asks its
    vertices to move by (sd - 0.1 d_hat) n for its deepest pair, and each
    vertex takes the largest push asked of it (the first primitive, in
    order, on ties; triangles before edges), so that pushes from the
    primitives around a vertex do not add up past the barrier's reach."""
    x = x.copy()
    d_safe = 0.1 * prm.dhat
    free_c = pad.free[pad.cand]
    prev = inds_prev if inds_prev is not None and len(inds_prev) == len(inds) else [None] * len(inds)
    for _ in range(8):
        moved = False
        for ind in inds:
            phi, n, _ = contact.sdf(ind, x[pad.cand])
            low = phi < d_safe * (1.0 - 1e-9)
            if low.any():
                moved = True
                x[pad.cand[low]] += ((d_safe - phi[low])[:, None] * n[low]) * free_c[low]
        for ind, ip in zip(inds, prev):
            if not (prm.mesh_pairs == 2 and ind.shape == contact.MESH):
                continue
            window = _travel(ind, ip) + prm.dhat
            deepest = {}
            for verts, n, sd, prim in mesh_pairs.signed_pairs(ind, x, pad.tris, pad.pedges, window,
                                                              below=d_safe * (1.0 - 1e-9)):
                if prim not in deepest or sd < deepest[prim][2]:
                    deepest[prim] = (verts, n, sd)
            push = {}
            for prim in sorted(deepest):
                verts, n, sd = deepest[prim]
                for v in verts:
                    if int(v) not in push or d_safe - sd > push[int(v)][0]:
                        push[int(v)] = (d_safe - sd, (sd - d_safe) * n)
            for v, (_, dv) in push.items():
                moved = True
                x[v] += dv * pad.free[v]
        if not moved:
            break
    if np.any(candidate_distances(pad, x, inds) <= 0.0):
        raise Infeasible("indenter pose leaves no feasible start")
    for ind, ip in zip(inds, prev):
        if prm.mesh_pairs == 2 and ind.shape == contact.MESH:
            if mesh_pairs.signed_pairs(ind, x, pad.tris, pad.pedges, _travel(ind, ip) + prm.dhat):
                raise Infeasible("a rigid mesh stays through the pad surface")
    return x


def step_filter(pad, x, p, inds, prm=None):
    """alpha_max = min(1, min_k 0.9 d_k / |p_k|), and with mesh_contact 2 the
    bound of the rigid meshes' vertex-face and edge-edge pairs."""
    d = candidate_distances(pad, x, inds)
    pk = np.linalg.norm(p[pad.cand], axis=1)
    moving = pk > 0
    a = 1.0
    if moving.any():
        a = float(min(1.0, np.min(0.9 * d[moving] / pk[moving])))
    if prm is not None:
        for ind in _pair_meshes(inds, prm):
            a = min(a, mesh_pairs.step_bound(ind, x, p, pad.tris, pad.pedges))
    return a


def step(pad, inds, prm, solver="direct", cg_tol=1e-12, verbose=False, inds_prev=None):
    """Advance the pad one step under the end-of-step indenter poses `inds`
    (friction lagged under the previous poses `inds_prev`, default `inds`).
    Returns StepResult; pad.x / pad.v are NOT modified (commit separately)."""
    h = prm.dt
    x_t, v_t = pad.x, pad.v
    xhat = x_t + h * v_t + h * h * np.asarray(prm.gravity)[None]
    fric = friction_lag(pad, inds, prm, inds_prev)
    x = feasible_start(pad, x_t, inds, prm, inds_prev)
    free = pad.free.ravel()
    tol = prm.newton_tol * pad.L_diag
    energies = [energy(pad, x, xhat, inds, prm, fric)]
    for it in range(1, prm.max_newton + 1):
        g = gradient(pad, x, xhat, inds, prm, fric).ravel()
        H = hessian(pad, x, inds, prm, fric=fric)
        Hff = H[free][:, free]
        if solver == "direct":
            pf = spla.spsolve(Hff.tocsc(), -g[free])
        else:
            dinv = 1.0 / Hff.diagonal()
            pf, info = spla.cg(Hff, -g[free], rtol=cg_tol, maxiter=100000,
                               M=sp.diags(dinv))
        p = np.zeros_like(g)
        p[free] = pf
        P3 = p.reshape(-1, 3)
        a = step_filter(pad, x, P3, inds, prm)
        pinf = float(np.max(np.abs(p))) if p.size else 0.0
        if pinf <= tol:
            x = x + a * P3
            energies.append(energy(pad, x, xhat, inds, prm, fric))
            v = (x - x_t) / h
            return StepResult(x, v, it, energies, fric)
        E0 = energies[-1]
        gTp = float(g @ p)
        for _ in range(prm.max_halvings + 1):
            E1 = energy(pad, x + a * P3, xhat, inds, prm, fric)
            if E1 <= E0 + 1e-4 * a * gTp + ENERGY_NOISE * abs(E0):
                break
            a *= 0.5
        else:
            raise LineSearchFailure(f"no decrease at Newton iteration {it}")
        x = x + a * P3
        energies.append(E1)
        if verbose:
            print(f"  newton {it}: |p|inf={pinf:.3e} a={a:.3e} E={E1:.6e}")
    raise NotConverged("Newton did not converge")


def commit(pad, res):
    pad.x = res.x.copy()
    pad.v = res.v.copy()
