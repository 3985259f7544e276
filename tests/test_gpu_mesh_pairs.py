"""Vertex-face and edge-edge pairs against rigid meshes (mesh_contact 2) on
the GPU against the oracle: a cube corner pressed down between the vertices
of a coarse pad, where only the pairs whose pad side is a triangle or an
edge see the contact, step by step in both precisions (including the first
step, whose start has the corner on the pad surface and needs the
primitives' push); the gradient and Newton direction at a state with
active pairs; the same scene with mesh_contact 1 passes through the surface
on both sides."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_util import context, errors, log, outputs, tc
from oracle import mesh_pairs, stepper
from workloads import scenes

pytestmark = pytest.mark.gpu


def _gpu_ind(mid, ind):
    return dict(shape=tc.MESH, prm=(0.0,), R=ind.R, c=ind.c, mesh_id=mid)


def _oracle_prm(ep, mode, **kw):
    return stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa, newton_tol=1e-10,
                              mesh_pairs=mode, **kw)


def _oracle_pad(ep):
    m = ep.pad.material
    return stepper.make_pad(ep.pad.X, ep.pad.tets, m.E, m.nu, m.density, fixed=ep.pad.fixed)


def _oracle_run(mode):
    ep = scenes.corner_press_episode()
    op = _oracle_pad(ep)
    prm = _oracle_prm(ep, mode)
    refs = []
    for s in range(1, ep.n_steps + 2):     # the ramp, then one step held
        ind = ep.pose(s)
        res = stepper.step(op, [ind], prm, inds_prev=[ep.pose(s - 1)] if s > 1 else None)
        stepper.commit(op, res)
        ref = outputs(op, op.x, [ind], prm)
        ref["newton"] = res.newton_iters
        refs.append(ref)
    return ep, op, refs


@pytest.fixture(scope="module")
def corner():
    return _oracle_run(2)


def _gpu_pad(ctx, ep, prec, mode, **kw):
    m = ep.pad.material
    return tc.Pad(ctx, ep.pad.X, ep.pad.tets, [dict(E=m.E, nu=m.nu, density=m.density)],
                  tc.make_params(precision=prec, mesh_contact=mode, **kw), fixed=ep.pad.fixed)


def _tunnelled(op, x, ind):
    return [p for p in mesh_pairs.signed_pairs(ind, x, op.tris, op.pedges, 1e-3) if p[2] < 0]


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-7, 1e-4, 1e-4)])
def test_corner_press_matches_oracle(corner, prec, newton_tol, cg_rel_tol, tol):
    ep, op, refs = corner
    ctx = context()
    mid = ctx.add_mesh(*ep.indenter.mesh)
    gp = _gpu_pad(ctx, ep, prec, 2, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol)
    top = op.is_top.astype(bool)
    worst = np.zeros(5)
    for s, ref in enumerate(refs, start=1):
        ind = ep.pose(s)
        st = gp.step([_gpu_ind(mid, ind)])
        assert st.status == 0, st
        e = np.array(errors(gp, ref, ep.pad.X, top))
        R, Rref = gp.read("reaction"), ref["cf"]["reaction"]
        eR = np.abs(R - Rref).max() / max(np.abs(Rref).max(), 1e-12)
        f, fref = gp.read("contact_force"), ref["cf"]["f"]
        ef = np.abs(f - fref).max() / max(np.abs(fref).max(), 1e-12)
        x = gp.read("positions")
        tun = _tunnelled(op, x, ind)
        log(f"{prec} step {s}: {st} oracle newton {ref['newton']} err pos {e[0]:.2e} sigma {e[1]:.2e} "
            f"p_n {e[2]:.2e} f {ef:.2e} reaction {R} ref {Rref} tunnelled {len(tun)}")
        assert not tun
        worst = np.maximum(worst, np.concatenate([e, [ef, eR]]))
    assert (worst[:3] < tol).all() and (worst[3:] < 10 * tol).all(), worst
    assert refs[-1]["cf"]["reaction"][2] > 0.5      # the corner is held by the pad
    gp.close()
    ctx.remove_mesh(mid)


def test_corner_press_without_triangle_pairs_passes_through():
    """mesh_contact 1 (pad-vertex pairs only) on the same scene: the corner
    crosses a top triangle unseen, on the GPU as in the oracle: no force,
    the pad at rest, the corner behind the surface."""
    ep, op, refs = _oracle_run(1)
    ctx = context()
    mid = ctx.add_mesh(*ep.indenter.mesh)
    gp = _gpu_pad(ctx, ep, "fp64", 1, newton_tol=1e-9, cg_rel_tol=1e-9)
    for s, ref in enumerate(refs, start=1):
        st = gp.step([_gpu_ind(mid, ep.pose(s))])
        assert st.status == 0
    x = gp.read("positions")
    assert np.abs(gp.read("reaction")).max() == 0.0 and np.abs(refs[-1]["cf"]["reaction"]).max() == 0.0
    assert np.abs(x - ep.pad.X).max() < 1e-15
    assert _tunnelled(op, x, ep.pose(len(refs)))
    gp.close()
    ctx.remove_mesh(mid)


def _oracle_direction(op, x, inds, prm):
    g = stepper.gradient(op, x, x, inds, prm)
    H = stepper.hessian(op, x, inds, prm)
    free = op.free.ravel()
    gf = g.ravel().copy()
    gf[~free] = 0.0
    p = np.zeros(gf.size)
    p[free] = spla.spsolve(H[free][:, free].tocsc(), -gf[free])
    return p.reshape(-1, 3), gf.reshape(-1, 3)


@pytest.mark.parametrize("prec,tol_d,tol_g", [("fp64", 1e-7, 1e-11), ("mixed", 2e-3, 1e-5)])
def test_pair_newton_direction_matches_oracle(corner, prec, tol_d, tol_g):
    """Gradient and Newton direction (Gauss-Newton pair blocks on and off
    the diagonal) at the state after step 2 under the pose of step 3, where
    vertex-face and edge-edge pairs are active."""
    ep, op0, refs = corner
    op = _oracle_pad(ep)
    prm = _oracle_prm(ep, 2, quasi_static=True)
    pose = ep.pose(3)
    x0 = stepper.feasible_start(op, refs[1]["x"], [pose], prm, inds_prev=[ep.pose(2)])
    _, _, (rows, _, _) = mesh_pairs.pair_terms(pose, x0, op.tris, op.pedges, op.pedge_len0, prm.dhat, prm.kappa)
    assert rows.size > 0
    p_ref, g_ref = _oracle_direction(op, x0, [pose], prm)
    ctx = context()
    mid = ctx.add_mesh(*ep.indenter.mesh)
    gp = _gpu_pad(ctx, ep, prec, 2, quasi_static=1, cg_rel_tol=1e-12 if prec == "fp64" else 1e-6, cg_forcing=0)
    gp.write("positions", x0)
    gp.write("velocities", np.zeros_like(x0))
    d, g = gp.newton_direction([_gpu_ind(mid, pose)])
    eg = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    ed = np.abs(d - p_ref).max() / np.abs(p_ref).max()
    log(f"{prec}: {rows.size} pair blocks, |p| {np.abs(p_ref).max():.3e} gradient err {eg:.2e} direction err {ed:.2e}")
    assert eg < tol_g
    assert ed < tol_d
    gp.close()
    ctx.remove_mesh(mid)
