"""Lagged smoothed friction (friction ratio 0.5, eps_v = 0.01 m/s of
Sec. III-B): a sphere pressed into the pad, then slid and twisted across it,
GPU against the FP64 oracle step by step (the oracle lags each step under
the previous step's pose, as the pad does)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import context, errors, log, outputs, tc
from oracle import extract, stepper
from workloads import scenes

pytestmark = pytest.mark.gpu

MU, EPS_V = 0.5, 0.01


def _pad(prec, newton_tol, cg_rel_tol, pad):
    m = pad.material
    return tc.Pad(context(), pad.X, pad.tets, [dict(E=m.E, nu=m.nu, density=m.density)],
                  tc.make_params(precision=prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol,
                                 friction=MU, eps_v=EPS_V),
                  fixed=pad.fixed)


@pytest.fixture(scope="module")
def episode():
    """The oracle's press-slide episode, step by step (computed once)."""
    pad, params, poses = scenes.press_slide_episode()
    m = pad.material
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density, fixed=pad.fixed)
    prm = stepper.StepParams(dt=params.dt, dhat=params.dhat, kappa=params.kappa, newton_tol=1e-10,
                             mu_f=MU, eps_v=EPS_V)
    refs = []
    for s, ind in enumerate(poses, start=1):
        prev = [poses[s - 2]] if s > 1 else None
        res = stepper.step(op, [ind], prm, inds_prev=prev)
        stepper.commit(op, res)
        ref = outputs(op, op.x, [ind], prm)
        ref["cf"] = extract.contact_forces(op, op.x, [ind], prm, fric=res.fric)
        ref["cf0"] = extract.contact_forces(op, op.x, [ind], prm)
        ref["newton"] = res.newton_iters
        refs.append(ref)
    return pad, poses, op, refs


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,pos_tol,sig_tol,f_tol",
                         [("fp64", 1e-9, 1e-9, 1e-6, 1e-6, 1e-5), ("mixed", 1e-6, 1e-4, 1e-4, 1e-4, 1e-3)])
def test_press_slide_matches_oracle(episode, prec, newton_tol, cg_rel_tol, pos_tol, sig_tol, f_tol):
    pad, poses, op, refs = episode
    gp = _pad(prec, newton_tol, cg_rel_tol, pad)
    X = pad.X
    top = op.is_top.astype(bool)
    worst = np.zeros(4)
    drag = 0.0
    for s, (ind, ref) in enumerate(zip(poses, refs), start=1):
        st = gp.step([ind])
        e = np.array(errors(gp, ref, X, top))
        f, fref = gp.read("contact_force"), ref["cf"]["f"]
        ef = np.abs(f - fref).max() / max(np.abs(fref).max(), 1e-12)
        R, Rref = gp.read("reaction"), ref["cf"]["reaction"]
        # friction's share of the reaction (the barrier's tilted normals give
        # a tangential part of their own)
        drag = max(drag, abs(Rref[0] - ref["cf0"]["reaction"][0]) / abs(Rref[2]))
        log(f"{prec} step {s}: {st} oracle newton {ref['newton']} err pos {e[0]:.2e} "
            f"sigma {e[1]:.2e} p_n {e[2]:.2e} f {ef:.2e} reaction {R} ref {Rref}")
        worst = np.maximum(worst, np.append(e, ef))
    assert worst[0] < pos_tol and worst[1] < sig_tol and worst[2] < sig_tol and worst[3] < f_tol, worst
    assert drag > 0.3
    gp.close()


def test_friction_state_round_trip_and_reset():
    """The previous pose travels with the saved state: a step after a load
    reproduces the step after the save bitwise; after a reset (no previous
    pose: w = 0) the same positions and velocities step elsewhere."""
    pad, params, poses = scenes.press_slide_episode()
    gp = _pad("mixed", 1e-6, 1e-4, pad)
    for ind in poses[:6]:
        gp.step([ind])
    buf = gp.save_state()
    x6, v6 = gp.read("positions"), gp.read("velocities")
    gp.step([poses[6]])
    xa = gp.read("positions")
    gp.load_state(buf)
    gp.step([poses[6]])
    assert np.array_equal(gp.read("positions"), xa)
    gp.reset()
    gp.write("positions", x6)
    gp.write("velocities", v6)
    gp.step([poses[6]])
    assert not np.array_equal(gp.read("positions"), xa)
    gp.close()
