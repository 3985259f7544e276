"""Staged and lockstep batch schedules (tc_set_schedule).  In the staged
schedule every pad goes through the stages of its Newton iterations at its
own pace, so one launch carries pads at different stages; each pad's
positions, velocities, stress, contact output and its Newton, CG and
line-search counts are bitwise those of the lockstep schedule.  Covered:
pads of the 60-pad batch with analytic indenters, with friction, two-layer
pads, and rigid meshes with vertex-face and edge-edge pairs; small CG chunks
and one trial energy per round (more rounds, more interleaving of stages);
the staged schedule on two streams."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import log, tc
from workloads import scenes

pytestmark = pytest.mark.gpu

FIELDS = ("positions", "velocities", "sigma", "pressure", "contact_force", "reaction")


def _run(envs, steps, staged, ls_evals=0, cg_chunk=0, streams=1, cg_warm=0):
    ctx = tc.Context(0)
    ctx.set_schedule(staged, ls_evals)
    if cg_chunk:
        ctx.set_launch(cg_per_replay=cg_chunk)
    ctx.set_streams(streams)
    ids, pads = {}, []
    try:
        for e in envs:
            m = e.pad.material
            mats, idx = [dict(E=m.E, nu=m.nu, density=m.density)], None
            if e.layers is not None:
                idx = e.layers[0]
                mats = [dict(E=q.E, nu=q.nu, density=q.density) for q in e.layers[1]]
            if e.indenter.mesh is not None and id(e.indenter.mesh) not in ids:
                ids[id(e.indenter.mesh)] = ctx.add_mesh(*e.indenter.mesh)
            pads.append(tc.Pad(ctx, e.pad.X, e.pad.tets, mats,
                               tc.make_params(precision="mixed", dt=e.params.dt, dhat=e.params.dhat,
                                              kappa=e.params.kappa, newton_tol=e.params.newton_tol,
                                              friction=e.friction, mesh_contact=e.mesh_contact,
                                              cg_rel_tol=0.2, cg_eta_max=0.2, cg_forcing=2, hess_proj=4,
                                              ls_expand=4, init_guess=1, cg_warm=cg_warm),
                               tet_material=idx))

        def poses(e, s):
            ind = e.pose(s)
            if ind.mesh is None:
                return [ind]
            return [dict(shape=tc.MESH, prm=ind.prm, R=ind.R, c=ind.c, mesh_id=ids[id(ind.mesh)])]

        stats = []
        for s in range(1, steps + 1):
            st = tc.step_batch(ctx, pads, [poses(e, s) for e in envs])
            stats.append([(x.status, x.newton_iters, x.cg_iters, x.ls_halvings) for x in st])
        out = [[p.read(f) for f in FIELDS] for p in pads]
        return stats, out
    finally:
        for p in pads:
            p.close()
        for i in ids.values():
            ctx.remove_mesh(i)
        ctx.close()


def _same(a, b, label):
    sa, oa = a
    sb, ob = b
    assert sa == sb, label
    for k, (pa, pb) in enumerate(zip(oa, ob)):
        for f, u, v in zip(FIELDS, pa, pb):
            assert np.array_equal(u, v), (label, k, f)


# pads of the 60-pad batch: all three pad shapes, each indenter kind
# (pads 10 and 43 are the slow texture plates)
PICK = (0, 3, 5, 10, 11, 17, 23, 29, 43, 47)


@pytest.mark.parametrize("variant", ["plain", "friction", "layers", "mesh2"])
def test_staged_bitwise_equal_to_lockstep(variant):
    envs = scenes.config3() if variant == "plain" else scenes.config3_variant(variant)
    envs = [envs[k] for k in PICK]
    if variant == "mesh2":
        # mesh indenters with vertex-face / edge-edge pairs among the picks
        assert any(e.mesh_contact == 2 and e.indenter.mesh is not None for e in envs)
    steps = 6
    lock = _run(envs, steps, staged=False)
    staged = _run(envs, steps, staged=True)
    log(f"{variant}: newton per pad at step {steps} {[x[1] for x in lock[0][-1]]}")
    _same(lock, staged, variant)


def test_staged_small_rounds_and_streams():
    """CG chunks of 2 iterations and one trial energy per round (a pad's
    iteration spreads over many rounds), and the staged schedule split over
    two streams: all bitwise equal to lockstep."""
    envs = [scenes.config3()[k] for k in PICK]
    steps = 4
    lock = _run(envs, steps, staged=False)
    _same(lock, _run(envs, steps, staged=True, ls_evals=1, cg_chunk=2), "chunk 2, one trial energy")
    _same(lock, _run(envs, steps, staged=True, streams=2), "two streams")


def test_staged_warm_start_bitwise_equal_to_lockstep():
    """The warm-started CG (iteration -1 along the previous direction) under
    both schedules, including chunks of 2 (the warm product and the first
    iteration in different rounds)."""
    envs = [scenes.config3()[k] for k in PICK]
    steps = 5
    lock = _run(envs, steps, staged=False, cg_warm=1)
    _same(lock, _run(envs, steps, staged=True, cg_warm=1), "warm start")
    _same(lock, _run(envs, steps, staged=True, cg_chunk=2, cg_warm=1), "warm start, chunk 2")
    cold = _run(envs, steps, staged=False)
    log(f"CG iterations per pad at step {steps}: cold {[x[2] for x in cold[0][-1]]}, "
        f"warm {[x[2] for x in lock[0][-1]]}")


def test_set_schedule_rejects_bad_values():
    ctx = tc.Context(0)
    try:
        for staged, evals in ((2, 0), (-1, 0), (1, 9), (1, -1)):
            with pytest.raises(tc.TcError):
                tc.check(ctx.lib.tc_set_schedule(ctx.h, staged, evals))
    finally:
        ctx.close()


def test_failing_pads_leave_the_others_untouched():
    """One batch, staged: a pad capped at one Newton iteration (not
    converged) and a pad whose feasible start fails, beside two pads that
    step normally.  The failing pads keep their state (the step is
    transactional); the others' results are bitwise those of stepping them
    alone."""
    from gpu_util import gpu_pad
    MM = scenes.MM
    ep = scenes.config1()
    ctx = tc.Context(0)
    pads, alone = [], []
    try:
        cube = scenes.one_cube_pad(1 * MM)
        fixed = np.where(cube.X[:, 2] == 0, 7, 3).astype(np.uint8)
        cyl = dict(shape=tc.CYLINDER, prm=(0.8 * MM, 5 * MM), R=np.eye(3), c=(0.5e-3, 0.5e-3, 0.5e-3))
        pads = [gpu_pad(ctx, ep.pad, "fp64"),
                gpu_pad(ctx, ep.pad, "fp64", max_newton=1, newton_tol=1e-12),
                gpu_pad(ctx, cube, "fp64", fixed=fixed),
                gpu_pad(ctx, ep.pad, "fp64", newton_tol=1e-8)]
        alone = [gpu_pad(ctx, ep.pad, "fp64"), gpu_pad(ctx, ep.pad, "fp64", newton_tol=1e-8)]
        poses = [[ep.pose(2)], [ep.pose(1)], [cyl], [ep.pose(2)]]
        for p in (pads[0], pads[3], alone[0], alone[1]):
            p.step([ep.pose(1)])
        before = [(p.read("positions"), p.read("velocities")) for p in pads]
        st = tc.step_batch(ctx, pads, poses, raise_on_error=False)
        assert [x.status for x in st] == [0, tc._abi.E_NOT_CONVERGED, tc._abi.E_INFEASIBLE, 0], st
        for k in (1, 2):
            assert np.array_equal(pads[k].read("positions"), before[k][0])
            assert np.array_equal(pads[k].read("velocities"), before[k][1])
        for p, a in ((pads[0], alone[0]), (pads[3], alone[1])):
            a.step([ep.pose(2)])
            for f in FIELDS:
                assert np.array_equal(p.read(f), a.read(f)), f
        log(f"batch with failures: {[(x.status, x.newton_iters) for x in st]}")
    finally:
        for p in pads + alone:
            p.close()
        ctx.close()
