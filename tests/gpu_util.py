"""Shared helpers of the GPU tests (not collected by pytest)."""
from __future__ import annotations

import functools
import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_2606_20426_amd as tc  # noqa: E402
from oracle import contact, extract, stepper, surface  # noqa: E402


def log(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=1)
def context():
    return tc.Context(0)


def gpu_pad(ctx, pad, precision="fp64", fixed=None, **kw):
    params = tc.make_params(precision=precision, **kw)
    return tc.Pad(ctx, pad.X, pad.tets, dict(E=pad.material.E, nu=pad.material.nu,
                                              density=pad.material.density),
                  params, fixed=fixed if fixed is not None else pad.fixed)


def oracle_pad(pad, fixed=None):
    return stepper.make_pad(pad.X, pad.tets, pad.material.E, pad.material.nu,
                            pad.material.density, fixed=fixed if fixed is not None else pad.fixed)


def oracle_episode(ep, steps, tol=1e-10, quasi_static=False):
    """Oracle states after each step: list of dict(x, sigma, t, pn, tt, cf)."""
    op = oracle_pad(ep.pad)
    prm = stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa,
                             newton_tol=tol, quasi_static=quasi_static)
    out = []
    for s in range(1, steps + 1):
        ind = ep.pose(s)
        res = stepper.step(op, [ind], prm)
        stepper.commit(op, res)
        out.append(outputs(op, op.x, [ind], prm))
        out[-1]["newton"] = res.newton_iters
    return op, out


def outputs(op, x, inds, prm):
    sig = extract.cauchy_per_tet(op, x)
    t, pn, tt, n, area = extract.surface_traction(op, x, sig)
    cf = extract.contact_forces(op, x, inds, prm)
    return dict(x=x.copy(), sigma=sig, t=t, pn=pn, tt=tt, n=n, area=area, cf=cf,
                tsum=extract.top_traction_sum(op, x, sig))


def voigt_to_mat(s6):
    s6 = np.asarray(s6, dtype=np.float64)
    S = np.empty(s6.shape[:-1] + (3, 3))
    S[..., 0, 0], S[..., 1, 1], S[..., 2, 2] = s6[..., 0], s6[..., 1], s6[..., 2]
    S[..., 1, 2] = S[..., 2, 1] = s6[..., 3]
    S[..., 0, 2] = S[..., 2, 0] = s6[..., 4]
    S[..., 0, 1] = S[..., 1, 0] = s6[..., 5]
    return S


def errors(gp, ref, X, top):
    """Parity norms: displacement-normalised positions, Frobenius-max sigma,
    pressure over the contact face."""
    x = gp.read("positions")
    sig = voigt_to_mat(gp.read("sigma"))
    pn = gp.read("pressure").astype(np.float64)
    e_pos = np.abs(x - ref["x"]).max() / max(np.abs(ref["x"] - X).max(), 1e-300)
    e_sig = np.linalg.norm(sig - ref["sigma"], axis=(1, 2)).max() / max(
        np.linalg.norm(ref["sigma"], axis=(1, 2)).max(), 1e-300)
    e_pn = np.abs(pn[top] - ref["pn"][top]).max() / max(np.abs(ref["pn"][top]).max(), 1e-300)
    return e_pos, e_sig, e_pn


_SURF_VERTS = {}


def free_surface_vertices(tets, fixed):
    """Vertices of surface triangles with a free component (side faces
    included): the set the barrier must keep outside every indenter."""
    tets = np.ascontiguousarray(tets)
    key = hashlib.sha1(tets.tobytes()).hexdigest()
    if key not in _SURF_VERTS:
        tris, _ = surface.surface_triangles(tets)
        _SURF_VERTS[key] = np.unique(tris)
    verts = _SURF_VERTS[key]
    return verts[np.asarray(fixed)[verts] != 7]


def surface_gap(verts, x, inds):
    """Smallest signed distance from the given vertices at positions x to
    any indenter (the no-penetration invariant of the step).  For a rigid
    mesh only the vertices inside its bounding sphere (plus 1 mm) take the
    brute-force distance; the others are at least their distance to that
    sphere away, which is what they contribute."""
    gap = np.inf
    for ind in inds:
        pts = x[verts]
        if getattr(ind, "mesh", None) is not None:
            rb = float(np.linalg.norm(np.asarray(ind.mesh[0]), axis=1).max())
            r = np.linalg.norm(pts - np.asarray(ind.c)[None], axis=1)
            near = r < rb + 1e-3
            if (~near).any():
                gap = min(gap, float((r[~near] - rb).min()))
            pts = pts[near]
        for lo in range(0, pts.shape[0], 4096):
            gap = min(gap, float(contact.sdf(ind, pts[lo:lo + 4096])[0].min()))
    return gap


def min_surface_gap(op, x, inds):
    """surface_gap over every free surface vertex of an oracle pad."""
    return surface_gap(free_surface_vertices(op.tets, op.fixed), x, inds)
