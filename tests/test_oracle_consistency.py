"""The oracle's step potential against its own gradient, for every indenter
kind with friction on: central differences of E(x) along random directions
equal g . v at a state in contact, with the friction lagged from a real
start state under a moved previous pose.  (A lag whose normal was not a unit
vector once made the friction gradient disagree with its energy under the
texture plate; this pin covers every shape, the two mesh barriers included.)"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import stepper
from workloads import meshes, scenes

MM = 1e-3


def _indenters(pad, dhat):
    out = {}
    for name, shape in (("sphere", scenes.SPHERE), ("cylinder", scenes.CYLINDER), ("cube_edge", scenes.BOX),
                        ("torus", scenes.TORUS), ("texture", scenes.TEXTURE)):
        r = 4 * MM if shape == scenes.SPHERE else None
        # over a grid vertex, so that sharp features come within the layer
        out[name] = (scenes.place_indenter(pad, shape, (9 * MM, 14 * MM * 5 / 9), dhat, sphere_radius=r), False)
    ico = scenes.Indenter(scenes.MESH, (0.0,) * 4, np.eye(3), out["sphere"][0].c.copy(), meshes.icosphere(4 * MM, 2))
    out["icosphere_mesh"] = (ico, False)
    tor = scenes.mesh_indenter(out["torus"][0])
    out["torus_mesh_pairs"] = (tor, True)
    return out


@pytest.mark.parametrize("name", ["sphere", "cylinder", "cube_edge", "torus", "texture", "icosphere_mesh",
                                  "torus_mesh_pairs"])
def test_potential_gradient_matches_central_differences(name):
    ep = scenes.config1()
    pad = ep.pad
    m = pad.material
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density)
    dhat = ep.params.dhat
    ind, pairs = _indenters(pad, dhat)[name]
    prm = stepper.StepParams(dt=ep.params.dt, dhat=dhat, kappa=ep.params.kappa, mu_f=0.5, eps_v=0.01,
                             mesh_pairs=pairs)
    # in contact: the indenter lowered into the barrier layer; the previous
    # pose a little to the side (the lag's w), the start state x_t at rest
    now = ind.at_depth(0.6 * dhat)
    prev = scenes.Indenter(now.shape, now.prm, now.R, now.c + np.array([0.05 * MM, -0.03 * MM, 0.02 * MM]), now.mesh)
    fric = stepper.friction_lag(op, [now], prm, [prev])
    lam = fric[0][0]
    assert (lam > 0).sum() >= 1, "no vertex in the barrier layer"
    rng = np.random.default_rng(11)
    x = op.x + 2e-6 * rng.standard_normal(op.x.shape) * op.free
    xhat = op.x.copy()
    E0 = stepper.energy(op, x, xhat, [now], prm, fric=fric)
    assert np.isfinite(E0)
    g = stepper.gradient(op, x, xhat, [now], prm, fric=fric)
    for _ in range(6):
        v = rng.standard_normal(x.shape) * op.free
        v[op.cand] *= 10.0                      # weight the contact layer
        v /= np.abs(v).max()
        h = 1e-9
        fd = (stepper.energy(op, x + h * v, xhat, [now], prm, fric=fric)
              - stepper.energy(op, x - h * v, xhat, [now], prm, fric=fric)) / (2 * h)
        gv = float(np.sum(g * v))
        assert fd == pytest.approx(gv, rel=2e-5, abs=1e-9 * np.abs(g).sum()), (name, fd, gv)



@pytest.mark.parametrize("name", ["sphere", "cylinder", "cube_edge", "torus", "texture", "icosphere_mesh",
                                  "torus_mesh_pairs"])
def test_exact_hessian_matches_gradient_differences(name):
    """The unprojected Hessian (elastic, barrier, friction, inertia) against
    central differences of the gradient along random directions, same
    states as above."""
    ep = scenes.config1()
    pad = ep.pad
    m = pad.material
    op = stepper.make_pad(pad.X, pad.tets, m.E, m.nu, m.density)
    dhat = ep.params.dhat
    ind, pairs = _indenters(pad, dhat)[name]
    prm = stepper.StepParams(dt=ep.params.dt, dhat=dhat, kappa=ep.params.kappa, mu_f=0.5, eps_v=0.01,
                             mesh_pairs=pairs)
    now = ind.at_depth(0.6 * dhat)
    prev = scenes.Indenter(now.shape, now.prm, now.R, now.c + np.array([0.05 * MM, -0.03 * MM, 0.02 * MM]), now.mesh)
    fric = stepper.friction_lag(op, [now], prm, [prev])
    rng = np.random.default_rng(12)
    x = op.x + 2e-6 * rng.standard_normal(op.x.shape) * op.free
    xhat = op.x.copy()
    H = stepper.hessian(op, x, [now], prm, project=False, fric=fric)
    for _ in range(4):
        v = rng.standard_normal(x.shape) * op.free
        v[op.cand] *= 10.0
        v /= np.abs(v).max()
        h = 1e-10
        gp = stepper.gradient(op, x + h * v, xhat, [now], prm, fric=fric).ravel()
        gm = stepper.gradient(op, x - h * v, xhat, [now], prm, fric=fric).ravel()
        fd = (gp - gm) / (2 * h)
        Hv = H @ v.ravel()
        assert np.abs(fd - Hv).max() <= 2e-4 * np.abs(Hv).max(), (name, np.abs(fd - Hv).max() / np.abs(Hv).max())
