"""Edge cases of the step: no indenter at all, the maximum number of
indenters at once (against the oracle), a pad without contact vertices (alone
and inside a batch), and friction pads on the server (their previous poses
advance with served steps exactly as with synchronous ones)."""
from __future__ import annotations

import time

import numpy as np
import pytest

from gpu_util import context, errors, gpu_pad, log, oracle_pad, outputs, tc
from oracle import stepper, surface
from workloads import scenes

pytestmark = pytest.mark.gpu

MM = scenes.MM


@pytest.mark.parametrize("friction", [0.0, 0.5])
def test_empty_indenter_list_keeps_rest_state(friction):
    ep = scenes.config1()
    gp = gpu_pad(context(), ep.pad, "mixed", friction=friction)
    for _ in range(3):
        st = gp.step([])
        assert st.status == 0 and st.newton_iters >= 1
    assert np.array_equal(gp.read("positions"), ep.pad.X)
    assert np.abs(gp.read("reaction")).max() == 0.0
    # and the pad steps normally afterwards (the previous pose count differs:
    # the friction lag takes the current pose)
    st = gp.step([ep.pose(1)])
    assert st.status == 0
    gp.close()


def _five_indenters(pad):
    spots = [(3.5, 3.5), (14.5, 3.5), (3.5, 10.5), (14.5, 10.5), (9.0, 7.0)]
    shapes = [scenes.SPHERE, scenes.CYLINDER, scenes.SPHERE, scenes.TORUS, scenes.BOX]
    radii = [2.0, None, 2.5, None, None]
    out = []
    for (x, y), sh, r in zip(spots, shapes, radii):
        out.append(scenes.place_indenter(pad, sh, (x * MM, y * MM), 1e-4,
                                         sphere_radius=None if r is None else r * MM))
    return out


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4)])
def test_five_indenters_match_oracle(prec, newton_tol, cg_rel_tol, tol):
    ep = scenes.config1()
    starts = _five_indenters(ep.pad)
    assert len(starts) == tc._abi.MAX_INDENTERS
    op = oracle_pad(ep.pad)
    prm = stepper.StepParams(newton_tol=1e-10)
    gp = gpu_pad(context(), ep.pad, prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol)
    top = op.is_top.astype(bool)
    worst = np.zeros(3)
    for s in range(1, 5):
        inds = [i.at_depth(0.1 * MM * s) for i in starts]
        res = stepper.step(op, inds, prm)
        stepper.commit(op, res)
        ref = outputs(op, op.x, inds, prm)
        st = gp.step(inds)
        e = np.array(errors(gp, ref, ep.pad.X, top))
        R, Rref = gp.read("reaction"), ref["cf"]["reaction"]
        log(f"{prec} step {s}: {st} oracle newton {res.newton_iters} err {e} reaction {R} ref {Rref}")
        assert np.abs(R - Rref).max() <= 1e-3 * np.abs(Rref).max()
        worst = np.maximum(worst, e)
    assert (worst < tol).all(), worst
    assert np.abs(gp.read("reaction").ravel()[2]) > 0
    gp.close()


def test_pad_without_contact_vertices():
    """Every surface vertex fixed: no candidates, nothing moves; in a
    batch with a normal pad the other pad's result is the same as alone."""
    ep = scenes.config1()
    X = ep.pad.X
    tris, _ = surface.surface_triangles(ep.pad.tets)
    fixed = np.zeros(X.shape[0], np.uint8)
    fixed[np.unique(tris)] = 7
    ctx = context()
    held = gpu_pad(ctx, ep.pad, "mixed", fixed=fixed)
    assert held.info["n_candidates"] == 0
    st = held.step([ep.pose(3)])
    assert st.status == 0
    assert np.array_equal(held.read("positions"), X)
    a = gpu_pad(ctx, ep.pad, "mixed")
    b = gpu_pad(ctx, ep.pad, "mixed")
    for s in (1, 2):
        a.step([ep.pose(s)])
        tc.step_batch(ctx, [held, b], [[ep.pose(s)], [ep.pose(s)]])
    assert np.array_equal(a.read("positions"), b.read("positions"))
    assert np.array_equal(held.read("positions"), X)
    for g in (held, a, b):
        g.close()


def test_server_friction_pads_equal_synchronous():
    """Served steps keep each pad's previous pose like synchronous steps:
    press-slide episodes with friction, interleaved on a server, end bitwise
    equal to the same episodes stepped one call at a time."""
    pad, params, poses = scenes.press_slide_episode()
    shifts = [0.0, 1.5 * MM, -1.5 * MM]
    eps = [[scenes.Indenter(p.shape, p.prm, p.R, p.c + np.array([0, d, 0])) for p in poses] for d in shifts]
    ctx = tc.Context(0)
    alone = []
    for ep in eps:
        g = gpu_pad(ctx, pad, "mixed", friction=0.5)
        for ind in ep:
            g.step([ind])
        alone.append(g.read("positions"))
        g.close()
    pads = [gpu_pad(ctx, pad, "mixed", friction=0.5) for _ in eps]
    srv = tc.Server(ctx, 2)
    results = []
    for s in range(len(poses)):
        for k, ep in enumerate(eps):
            srv.submit(pads[k], [ep[s]], tag=100 * k + s)
        time.sleep(0.001)
        results += srv.poll()
    t0 = time.perf_counter()
    while len(results) < len(eps) * len(poses):
        results += srv.poll(wait_us=2000)
        assert time.perf_counter() - t0 < 60, "server did not finish"
    srv.close()
    assert all(r["status"] == 0 for r in results)
    for k, g in enumerate(pads):
        assert np.array_equal(g.read("positions"), alone[k]), k
        g.close()
    ctx.close()


def test_autotune_keeps_state_and_stepping_valid():
    """The launch-shape autotuner picks shapes from its candidate sets, leaves
    every pad's committed state (and friction pose) untouched, and stepping
    afterwards reaches the same minimiser as the default launch shape."""
    eps = scenes.config3(n_envs=4)
    ctxs = [tc.Context(0), tc.Context(0)]
    pads = [[gpu_pad(c, e.pad, "mixed", newton_tol=1e-6, cg_rel_tol=1e-4) for e in eps] for c in ctxs]
    for s in (1, 2):
        for c, ps in zip(ctxs, pads):
            tc.step_batch(c, ps, [[e.pose(s)] for e in eps])
    before = [p.read("positions") for p in pads[1]]
    chosen = ctxs[1].autotune(pads[1], [[e.pose(3)] for e in eps])
    log(f"autotune chose {chosen}")
    assert chosen[0] in (128, 256, 512, 1024) and chosen[1] in (64, 128, 256)
    assert chosen[2] % 64 == 0 and 64 <= chosen[2] <= 1024 and chosen[3] in (8, 12, 16, 24)
    assert 1 <= chosen[4] <= 2                      # 4 pads: at most 2 streams of 2 pads
    for p, x in zip(pads[1], before):
        assert np.array_equal(p.read("positions"), x)
    for s in (3, 4):
        for c, ps in zip(ctxs, pads):
            st = tc.step_batch(c, ps, [[e.pose(s)] for e in eps])
            assert all(x.status == 0 for x in st)
    for e, pa, pb in zip(eps, *pads):
        xa, xb = pa.read("positions"), pb.read("positions")
        disp = np.abs(xa - e.pad.X).max()
        tol = max(1e-3 * disp, 2e-6 * np.linalg.norm(e.pad.X.max(0) - e.pad.X.min(0)))
        assert np.abs(xa - xb).max() <= tol
    for ps in pads:
        for p in ps:
            p.close()
    for c in ctxs:
        c.close()


def test_runtime_switches_relayout_scratch():
    """Turning friction on or off for a live pad changes its step scratch
    layout: the next steps run on the new layout and reach the same
    minimiser as a pad configured that way from the start."""
    ep = scenes.config1()
    ref_ctx, ctx = tc.Context(0), tc.Context(0)
    kw = dict(newton_tol=1e-6, cg_rel_tol=1e-4)
    ref = gpu_pad(ref_ctx, ep.pad, "mixed", friction=0.5, **kw)
    pad = gpu_pad(ctx, ep.pad, "mixed", **kw)
    other = gpu_pad(ctx, ep.pad, "mixed", friction=0.5, **kw)
    ref.step([ep.pose(1)])
    pad.step([ep.pose(1)])
    other.step([ep.pose(1)])
    pad.set_params(tc.make_params(precision="mixed", friction=0.5, **kw))   # friction on: new layout
    for s in (2, 3):
        ref.step([ep.pose(s)])
        st = tc.step_batch(ctx, [pad, other], [[ep.pose(s)], [ep.pose(s)]])
        assert all(x.status == 0 for x in st)
    pad.set_params(tc.make_params(precision="mixed", friction=0.5, **kw))   # unchanged layout
    for s in (4, 5):
        ref.step([ep.pose(s)])
        tc.step_batch(ctx, [pad, other], [[ep.pose(s)], [ep.pose(s)]])
    xr = ref.read("positions")
    tol = 2e-6 * np.linalg.norm(ep.pad.X.max(0) - ep.pad.X.min(0))
    for g in (pad, other):
        assert np.abs(g.read("positions") - xr).max() <= max(tol, 1e-3 * np.abs(xr - ep.pad.X).max())
    pad.set_params(tc.make_params(precision="mixed", **kw))                  # friction off again
    assert pad.step([ep.pose(6)]).status == 0
    for g in (ref, pad, other):
        g.close()
    ref_ctx.close()
    ctx.close()


def test_mesh_contact_mode_leaves_analytic_shapes_alone():
    """mesh_contact changes the barrier of rigid meshes only: a pad under an
    analytic sphere steps bitwise the same in either mode."""
    ep = scenes.config1()
    ctx = context()
    a = gpu_pad(ctx, ep.pad, "mixed", mesh_contact=0)
    b = gpu_pad(ctx, ep.pad, "mixed", mesh_contact=1)
    for s in range(1, 5):
        sa, sb = a.step([ep.pose(s)]), b.step([ep.pose(s)])
        assert sa.newton_iters == sb.newton_iters and sa.cg_iters == sb.cg_iters
    for f in ("positions", "sigma", "contact_force", "reaction"):
        assert np.array_equal(a.read(f), b.read(f)), f
    a.close()
    b.close()
