"""The assembled Newton system on the GPU (element Hessians with the analytic
PSD projection, barrier Hessians, gather assembly, block-Jacobi CG) against
the oracle's: same gradient, same Newton direction at deformed states."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_util import context, gpu_pad, log, oracle_pad, tc
from oracle import stepper
from workloads import scenes

pytestmark = pytest.mark.gpu
MM = 1e-3


def _oracle_direction(op, x, inds, prm):
    g = stepper.gradient(op, x, x, inds, prm)
    H = stepper.hessian(op, x, inds, prm)
    free = op.free.ravel()
    gf = g.ravel().copy()
    gf[~free] = 0.0
    p = np.zeros(gf.size)
    p[free] = spla.spsolve(H[free][:, free].tocsc(), -gf[free])
    return p.reshape(-1, 3), gf.reshape(-1, 3)


def _state(ep, steps, prm):
    op = oracle_pad(ep.pad)
    for s in range(1, steps + 1):
        stepper.commit(op, stepper.step(op, [ep.pose(s)], prm))
    return op


@pytest.mark.parametrize("shape", ["sphere", "texture"])
@pytest.mark.parametrize("prec,tol_d,tol_g", [("fp64", 1e-7, 1e-11), ("mixed", 2e-3, 1e-5)])
def test_newton_direction_matches_oracle(shape, prec, tol_d, tol_g):
    ep = scenes.config1()
    if shape == "texture":
        ind = scenes.place_indenter(ep.pad, scenes.TEXTURE, (9 * MM, 7 * MM), 1e-4)
        ep = scenes.Episode(ep.pad, ind, 0.4 * MM, 6, ep.params)
    prm = stepper.StepParams(newton_tol=1e-10, quasi_static=True)
    op = _state(ep, 5, prm)
    pose = ep.pose(6)
    x0 = stepper.feasible_start(op, op.x, [pose], prm)
    p_ref, g_ref = _oracle_direction(op, x0, [pose], prm)
    gp = gpu_pad(context(), ep.pad, prec, quasi_static=1, cg_rel_tol=1e-12 if prec == "fp64" else 1e-6,
                 cg_forcing=0)
    gp.write("positions", x0)
    gp.write("velocities", np.zeros_like(x0))
    d, g = gp.newton_direction([pose])
    eg = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    ed = np.abs(d - p_ref).max() / np.abs(p_ref).max()
    log(f"{shape} {prec}: |p| {np.abs(p_ref).max():.3e} gradient err {eg:.2e} direction err {ed:.2e}")
    assert eg < tol_g
    assert ed < tol_d
