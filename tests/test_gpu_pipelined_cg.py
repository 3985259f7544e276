"""Pipelined preconditioned CG (one fused launch per iteration) against the
oracle: the Newton direction against the exact sparse solve, an indentation
episode step by step, and a batch against the classic solver's minimiser."""
from __future__ import annotations

import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_util import errors, gpu_pad, log, oracle_episode, oracle_pad, tc
from oracle import stepper
from workloads import scenes

pytestmark = pytest.mark.gpu
MM = 1e-3


@functools.lru_cache(maxsize=1)
def pipe_context():
    ctx = tc.Context(0)
    ctx.set_cg_variant(1)
    return ctx


@pytest.mark.parametrize("prec,tol_d", [("fp64", 1e-7), ("mixed", 2e-3)])
def test_pipelined_newton_direction_matches_exact_solve(prec, tol_d):
    ep = scenes.config1()
    prm = stepper.StepParams(newton_tol=1e-10, quasi_static=True)
    op = oracle_pad(ep.pad)
    for s in range(1, 6):
        stepper.commit(op, stepper.step(op, [ep.pose(s)], prm))
    pose = ep.pose(6)
    x0 = stepper.feasible_start(op, op.x, [pose], prm)
    g = stepper.gradient(op, x0, x0, [pose], prm)
    H = stepper.hessian(op, x0, [pose], prm)
    free = op.free.ravel()
    p_ref = np.zeros(g.size)
    p_ref[free] = spla.spsolve(H[free][:, free].tocsc(), -g.ravel()[free])
    p_ref = p_ref.reshape(-1, 3)
    gp = gpu_pad(pipe_context(), ep.pad, prec, quasi_static=1, cg_rel_tol=1e-12 if prec == "fp64" else 1e-6,
                 cg_forcing=0)
    gp.write("positions", x0)
    gp.write("velocities", np.zeros_like(x0))
    d, _ = gp.newton_direction([pose])
    ed = np.abs(d - p_ref).max() / np.abs(p_ref).max()
    log(f"pipelined {prec}: direction err {ed:.2e}")
    assert ed < tol_d
    gp.close()


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,pos_tol,sig_tol",
                         [("fp64", 1e-9, 1e-9, 1e-6, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4, 1e-4)])
def test_pipelined_episode_matches_oracle(prec, newton_tol, cg_rel_tol, pos_tol, sig_tol):
    ep = scenes.config1()
    op, refs = oracle_episode(ep, ep.n_steps)
    gp = gpu_pad(pipe_context(), ep.pad, prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol)
    top = op.is_top.astype(bool)
    worst = np.zeros(3)
    for s, ref in enumerate(refs, start=1):
        st = gp.step([ep.pose(s)])
        e = np.array(errors(gp, ref, ep.pad.X, top))
        log(f"pipelined {prec} step {s}: {st} err pos {e[0]:.2e} sigma {e[1]:.2e} p_n {e[2]:.2e}")
        worst = np.maximum(worst, e)
    assert worst[0] < pos_tol and worst[1] < sig_tol and worst[2] < sig_tol, worst
    gp.close()


def test_pipelined_batch_matches_classic():
    """Uneven pads (three shapes, five indenters) in one batch: both solvers
    reach the same minimiser within the Newton tolerance."""
    envs = scenes.config3(n_envs=6)
    ctxs = [tc.Context(0), pipe_context()]
    out = []
    for ctx in ctxs:
        pads = [gpu_pad(ctx, e.pad, "mixed", newton_tol=1e-6, cg_rel_tol=1e-4) for e in envs]
        for s in range(1, 4):
            st = tc.step_batch(ctx, pads, [[e.pose(s)] for e in envs])
            assert all(x.status == 0 for x in st)
        out.append([p.read("positions") for p in pads])
        log(f"cg sum {sum(x.cg_iters for x in st)} newton max {max(x.newton_iters for x in st)}")
        for p in pads:
            p.close()
    ctxs[0].close()
    for e, xa, xb in zip(envs, *out):
        disp = np.abs(xa - e.pad.X).max()
        # both stop within the Newton tolerance (1e-6 of the bounding-box diagonal)
        tol = max(1e-3 * disp, 2e-6 * np.linalg.norm(e.pad.X.max(0) - e.pad.X.min(0)))
        assert np.abs(xa - xb).max() <= tol, (np.abs(xa - xb).max(), disp)
