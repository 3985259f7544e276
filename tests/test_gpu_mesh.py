"""Rigid triangle-mesh indenters (TC_MESH): signed distance to the mesh over
a bounding-volume hierarchy on the GPU against the oracle's brute-force
distance, step by step; a box given as 12 triangles against the analytic
box; the mesh registry."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import context, errors, log, outputs, tc
from oracle import contact, extract, stepper
from workloads import meshes, scenes

pytestmark = pytest.mark.gpu

MM = 1e-3


def _gpu_inds(ids, inds):
    out = []
    for ind in inds:
        if ind.shape == scenes.MESH:
            out.append(dict(shape=tc.MESH, prm=(0.0,), R=ind.R, c=ind.c, mesh_id=ids[id(ind.mesh)]))
        else:
            out.append(ind)
    return out


def _oracle_run(name, mu_f, pairs=False):
    pad, params, poses = getattr(scenes, name)()
    m = pad.material
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density, fixed=pad.fixed)
    prm = stepper.StepParams(dt=params.dt, dhat=params.dhat, kappa=params.kappa, newton_tol=1e-10,
                             mu_f=mu_f, eps_v=0.01, mesh_pairs=pairs)
    refs = []
    for s, ind in enumerate(poses, start=1):
        prev = [poses[s - 2]] if s > 1 else None
        res = stepper.step(op, [ind], prm, inds_prev=prev)
        stepper.commit(op, res)
        ref = outputs(op, op.x, [ind], prm)
        ref["cf"] = extract.contact_forces(op, op.x, [ind], prm, fric=res.fric)
        ref["newton"] = res.newton_iters
        refs.append(ref)
    return pad, poses, op, refs


@pytest.fixture(scope="module")
def press():
    return _oracle_run("mesh_press_episode", 0.0)


@pytest.fixture(scope="module")
def slide():
    return _oracle_run("mesh_slide_episode", 0.5)


@pytest.fixture(scope="module")
def press_pairs():
    return _oracle_run("mesh_press_episode", 0.0, pairs=True)


@pytest.fixture(scope="module")
def slide_pairs():
    return _oracle_run("mesh_slide_episode", 0.5, pairs=True)


def _compare(run, prec, newton_tol, cg_rel_tol, mu_f, pairs=0):
    pad, poses, op, refs = run
    ctx = context()
    mesh = poses[0].mesh
    ids = {id(mesh): ctx.add_mesh(*mesh)}
    m = pad.material
    gp = tc.Pad(ctx, pad.X, pad.tets, [dict(E=m.E, nu=m.nu, density=m.density)],
                tc.make_params(precision=prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol,
                               friction=mu_f, eps_v=0.01, mesh_contact=pairs), fixed=pad.fixed)
    top = op.is_top.astype(bool)
    worst = np.zeros(4)
    for s, (ind, ref) in enumerate(zip(poses, refs), start=1):
        st = gp.step(_gpu_inds(ids, [ind]))
        e = np.array(errors(gp, ref, pad.X, top))
        f, fref = gp.read("contact_force"), ref["cf"]["f"]
        ef = np.abs(f - fref).max() / max(np.abs(fref).max(), 1e-12)
        log(f"{prec} step {s}: {st} oracle newton {ref['newton']} err pos {e[0]:.2e} sigma {e[1]:.2e} "
            f"p_n {e[2]:.2e} f {ef:.2e} reaction {gp.read('reaction')} ref {ref['cf']['reaction']}")
        worst = np.maximum(worst, np.append(e, ef))
    gp.close()
    ctx.remove_mesh(ids[id(mesh)])
    return worst


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4)])
def test_torus_mesh_press_matches_oracle(press, prec, newton_tol, cg_rel_tol, tol):
    worst = _compare(press, prec, newton_tol, cg_rel_tol, 0.0)
    assert (worst[:3] < tol).all() and worst[3] < 10 * tol, worst


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-7, 1e-4, 1e-4)])
def test_torus_mesh_pair_barrier_matches_oracle(press_pairs, prec, newton_tol, cg_rel_tol, tol):
    """mesh_contact 1: the barrier summed over the triangles within d_hat.
    The mixed run stops at 1e-7 of the bounding box: at the first contact
    step the displacement is small, and 1e-6 leaves 1.8e-4 of it."""
    worst = _compare(press_pairs, prec, newton_tol, cg_rel_tol, 0.0, pairs=1)
    assert (worst[:3] < tol).all() and worst[3] < 10 * tol, worst


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-7, 1e-4, 1e-4)])
def test_icosphere_slide_pair_barrier_with_friction_matches_oracle(slide_pairs, prec, newton_tol, cg_rel_tol, tol):
    """mesh_contact 1 with friction: the lag takes the summed pair force."""
    worst = _compare(slide_pairs, prec, newton_tol, cg_rel_tol, 0.5, pairs=1)
    assert (worst[:3] < tol).all() and worst[3] < 10 * tol, worst


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4)])
def test_icosphere_slide_with_friction_matches_oracle(slide, prec, newton_tol, cg_rel_tol, tol):
    worst = _compare(slide, prec, newton_tol, cg_rel_tol, 0.5)
    assert (worst[:3] < tol).all() and worst[3] < 10 * tol, worst


def test_box_mesh_equals_analytic_box():
    """The same pad pressed by a face-down, slightly tilted cube given as 12
    triangles and as the analytic box: the same minimiser, by the same
    Newton path (a convex mesh's step bound is the convex shapes')."""
    pad = scenes.config1().pad
    ctx = context()
    a = 3 * MM
    V, F = meshes.box_surface(a, a, a)
    mid = ctx.add_mesh(V, F)
    R = scenes._rot_z(0.3) @ scenes._rot_x(0.05)
    low = a * (np.cos(0.05) + np.sin(0.05))
    c = np.array([9 * MM, 7 * MM, 4 * MM + low + 1e-4])
    pads = [tc.Pad(ctx, pad.X, pad.tets, dict(E=0.3e6, nu=0.45, density=1000.0),
                   tc.make_params(precision="fp64", newton_tol=1e-9, cg_rel_tol=1e-9), fixed=pad.fixed)
            for _ in range(2)]
    for s in range(1, 5):
        cc = c - np.array([0, 0, 0.15 * MM * s])
        sa = pads[0].step([dict(shape=tc.BOX, prm=(a, a, a), R=R, c=cc)])
        sm = pads[1].step([dict(shape=tc.MESH, prm=(0.0,), R=R, c=cc, mesh_id=mid)])
        xa, xm = pads[0].read("positions"), pads[1].read("positions")
        disp = np.abs(xa - pad.X).max()
        log(f"step {s}: box {sa} mesh {sm} diff {np.abs(xa - xm).max() / disp:.2e}")
        assert np.abs(xa - xm).max() <= 1e-6 * disp
        # a convex mesh takes the convex shapes' step bound: the same path
        assert sa.newton_iters == sm.newton_iters
        ra, rm = pads[0].read("reaction"), pads[1].read("reaction")
        assert np.abs(ra - rm).max() <= 1e-5 * np.abs(ra).max()
    assert disp > 0.2 * MM
    for p in pads:
        p.close()
    ctx.remove_mesh(mid)


def test_mesh_registry():
    ctx = tc.Context(0)
    used0 = ctx.memory()[0]
    V, F = meshes.icosphere(2 * MM, 2)
    ids = [ctx.add_mesh(V, F) for _ in range(3)]
    mesh_bytes = ctx.memory()[0] - used0
    assert len(set(ids)) == 3 and mesh_bytes > 0
    pad = scenes.config1().pad
    gp = tc.Pad(ctx, pad.X, pad.tets, dict(E=0.3e6, nu=0.45, density=1000.0),
                tc.make_params(precision="mixed"), fixed=pad.fixed)
    far = dict(shape=tc.MESH, prm=(0.0,), R=np.eye(3), c=(9 * MM, 7 * MM, 20 * MM), mesh_id=ids[1])
    gp.step([far])
    assert np.array_equal(gp.read("positions"), pad.X)       # out of reach: rest state exactly
    ctx.remove_mesh(ids[1])
    with pytest.raises(tc.TcError) as e:
        gp.step([far])
    assert e.value.status == -1                                # TC_E_INVALID_ARG
    with pytest.raises(tc.TcError):
        ctx.remove_mesh(ids[1])
    assert ctx.add_mesh(V, F) == ids[1]                       # the freed slot is reused
    with pytest.raises(tc.TcError):
        ctx.add_mesh(V, F[:, ::-1])                            # inward normals
    gp.close()
    before = ctx.memory()[0]
    for i in ids:
        ctx.remove_mesh(i)
    assert before - ctx.memory()[0] == mesh_bytes
    ctx.close()


def test_pair_mode_served_and_extracted():
    """Rigid-mesh pads in pair mode (mesh_contact 1) through the server end
    bitwise equal to synchronous stepping; standalone extraction at the
    final state gives the oracle's pair-barrier contact forces."""
    import time
    pad, params, poses = scenes.mesh_press_episode()
    mesh = poses[0].mesh
    ctx = tc.Context(0)
    mid = ctx.add_mesh(*mesh)
    m = pad.material
    shifts = [0.0, 1.0 * MM, -1.0 * MM]
    eps = [[dict(shape=tc.MESH, prm=(0.0,), R=p.R, c=p.c + np.array([d, 0, 0]), mesh_id=mid) for p in poses]
           for d in shifts]

    def make():
        return tc.Pad(ctx, pad.X, pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                      tc.make_params(precision="mixed", mesh_contact=1), fixed=pad.fixed)
    alone = []
    for ep in eps:
        g = make()
        for ind in ep:
            assert g.step([ind]).status == 0
        alone.append(g.read("positions"))
        g.close()
    pads = [make() for _ in eps]
    srv = tc.Server(ctx, 2)
    results = []
    for s in range(len(poses)):
        for k, ep in enumerate(eps):
            srv.submit(pads[k], [ep[s]], tag=100 * k + s)
        results += srv.poll()
    t0 = time.perf_counter()
    while len(results) < len(eps) * len(poses):
        results += srv.poll(wait_us=2000)
        assert time.perf_counter() - t0 < 60, "server did not finish"
    srv.close()
    assert all(r["status"] == 0 for r in results)
    for k, g in enumerate(pads):
        assert np.array_equal(g.read("positions"), alone[k]), k
    # standalone extraction against the oracle at the GPU's positions
    g = pads[0]
    g.extract([eps[0][-1]])
    x = g.read("positions")
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density, fixed=pad.fixed)
    prm = stepper.StepParams(dt=params.dt, dhat=params.dhat, kappa=params.kappa, mesh_pairs=True)
    ref = extract.contact_forces(op, x, [poses[-1]], prm)
    f = g.read("contact_force")
    err = np.abs(f - ref["f"]).max() / np.abs(ref["f"]).max()
    log(f"served pair-mode pads bitwise equal; extraction contact forces vs oracle {err:.2e}")
    assert err < 1e-9 and np.abs(ref["f"]).max() > 0
    for g in pads:
        g.close()
    ctx.remove_mesh(mid)
    ctx.close()
