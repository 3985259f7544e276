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


def _punch_pads(friction):
    """A 18 x 14 x 4 mm pad (48,384 tets) under the flat cylinder punch
    (r = 2.5 mm), pressed 0.3 mm over 6 steps."""
    pad = scenes.box_pad(18e-3, 14e-3, 4e-3, 36, 28, 8, scenes.Material(0.3e6, 0.45, 1000.0))
    start = scenes.place_indenter(pad, scenes.CYLINDER, (9e-3, 7e-3), 1e-4)
    m = pad.material
    gp = tc.Pad(context(), pad.X, pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                tc.make_params(precision="mixed", friction=friction, eps_v=EPS_V))
    for s in range(1, 7):
        assert gp.step([start.at_depth(0.05e-3 * s)]).status == 0
    return gp, start.at_depth(0.3e-3)


def _forces(gp, axis_xy):
    cand = gp.read("candidates")
    p = gp.read("positions")[cand]
    f = gp.read("contact_force")
    r = p[:, :2] - axis_xy[None]
    rn = np.linalg.norm(r, axis=1)
    er = r / np.maximum(rn, 1e-12)[:, None]
    et = np.stack([-er[:, 1], er[:, 0]], axis=1)
    ft = f[:, :2]
    return f, ft, np.einsum("ki,ki->k", ft, et), np.einsum("ki,ki->k", ft, er), r


def test_contact_modes_translation_and_torsion():
    """The two frictional contact modes of Sec. IV-C under a flat punch.
    Lateral translation: the pad is dragged along the motion, with no
    sideways force.  Axial rotation: the tangential contact forces circulate
    with the rotation (a vortex: azimuthal, no net force, positive torque);
    without friction the same twist leaves no torque."""
    # translation: +x, 0.05 mm per step
    gp, pose = _punch_pads(MU)
    for s in range(1, 6):
        pose = scenes.Indenter(pose.shape, pose.prm, pose.R, pose.c + np.array([0.05e-3, 0.0, 0.0]))
        assert gp.step([pose]).status == 0
    f, ft, _, _, _ = _forces(gp, pose.c[:2])
    F = f.sum(axis=0)
    log(f"translation: net contact force on the pad {F}, |F_t| / F_z {np.hypot(F[0], F[1]) / abs(F[2]):.3f}")
    assert F[0] > 0 and abs(F[1]) < 0.02 * F[0]
    assert np.hypot(F[0], F[1]) <= 1.05 * MU * abs(F[2])
    gp.close()
    # torsion: 2 degrees per step about the punch axis
    torque = {}
    for mu in (MU, 0.0):
        gp, pose = _punch_pads(mu)
        for s in range(1, 6):
            pose = scenes.Indenter(pose.shape, pose.prm, scenes._rot_z(np.radians(2.0 * s)), pose.c)
            assert gp.step([pose]).status == 0
        f, ft, f_theta, f_r, r = _forces(gp, pose.c[:2])
        mag = np.linalg.norm(ft, axis=1)
        torque[mu] = float(np.sum(r[:, 0] * ft[:, 1] - r[:, 1] * ft[:, 0]))
        net = np.linalg.norm(ft.sum(axis=0))
        log(f"torsion mu {mu}: torque {torque[mu]:.4e} N m, azimuthal share {np.abs(f_theta).sum() / max(mag.sum(), 1e-300):.3f}, "
            f"net tangential {net:.3e} of {mag.sum():.3e}")
        if mu > 0:
            big = mag > 0.01 * mag.max()
            assert torque[mu] > 0
            assert np.abs(f_theta).sum() > 0.8 * mag.sum()
            assert (f_theta[big] > 0).mean() > 0.9
            assert net < 0.05 * mag.sum()
        gp.close()
    assert abs(torque[0.0]) < 0.01 * torque[MU]


def test_texture_plate_friction_regression():
    """Friction under the texture plate (phi not a distance): one pad of the
    paper-like 60-environment workload (d_hat = 1 mm, friction 0.5) whose
    steps once stalled at the Newton cap while the lag's normal was not a
    unit vector.  Twelve steps against the oracle, step by step, with few
    Newton iterations each."""
    e = scenes.paper60()[38]
    assert e.indenter.shape == scenes.TEXTURE
    pad = e.pad
    m = pad.material
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density)
    prm = stepper.StepParams(dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa, newton_tol=1e-10,
                             mu_f=MU, eps_v=EPS_V)
    gp = tc.Pad(context(), pad.X, pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                tc.make_params(precision="mixed", dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa,
                               newton_tol=1e-7, cg_rel_tol=1e-4, friction=MU, eps_v=EPS_V))
    worst = 0.0
    for s in range(1, 13):
        prev = [e.pose(s - 1)] if s > 1 else None
        res = stepper.step(op, [e.pose(s)], prm, inds_prev=prev)
        stepper.commit(op, res)
        st = gp.step([e.pose(s)])
        x = gp.read("positions")
        err = np.abs(x - op.x).max() / max(np.abs(op.x - pad.X).max(), 1e-300)
        log(f"step {s}: {st} oracle newton {res.newton_iters} err pos {err:.2e}")
        assert st.status == 0 and st.newton_iters < 40 and res.newton_iters < 40
        worst = max(worst, err)
    assert worst < 1e-4, worst
    gp.close()
