"""Heterogeneous materials (per-tet material index, the dual-layer gel of
Sec. IV-D): a soft top layer on a stiffer base under a sphere, GPU against
the FP64 oracle with per-tet Lame parameters and densities, step by step."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import context, errors, log, outputs, tc
from oracle import stepper
from workloads import scenes

pytestmark = pytest.mark.gpu


def _pads(prec, newton_tol, cg_rel_tol):
    ep, idx, mats = scenes.dual_layer_episode()
    pad = ep.pad
    gp = tc.Pad(context(), pad.X, pad.tets,
                [dict(E=m.E, nu=m.nu, density=m.density) for m in mats],
                tc.make_params(precision=prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol),
                fixed=pad.fixed, tet_material=idx)
    E = np.array([m.E for m in mats])[idx]
    nu = np.array([m.nu for m in mats])[idx]
    rho = np.array([m.density for m in mats])[idx]
    op = stepper.make_pad(pad.X, pad.tets, E, nu, rho, fixed=pad.fixed)
    return ep, gp, op


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,pos_tol,sig_tol",
                         [("fp64", 1e-9, 1e-9, 1e-6, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4, 1e-4)])
def test_dual_layer_episode_matches_oracle(prec, newton_tol, cg_rel_tol, pos_tol, sig_tol):
    ep, gp, op = _pads(prec, newton_tol, cg_rel_tol)
    prm = stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa,
                             newton_tol=1e-10)
    X = ep.pad.X
    top = op.is_top.astype(bool)
    assert np.allclose(gp.read("mass"), op.mass, rtol=1e-12)
    worst = np.zeros(3)
    for s in range(1, ep.n_steps + 1):
        ind = [ep.pose(s)]
        res = stepper.step(op, ind, prm)
        stepper.commit(op, res)
        ref = outputs(op, op.x, ind, prm)
        st = gp.step(ind)
        e = np.array(errors(gp, ref, X, top))
        R, Rref = gp.read("reaction"), ref["cf"]["reaction"]
        eR = np.abs(R - Rref).max() / max(np.abs(Rref).max(), 1e-12)
        log(f"{prec} step {s}: {st} oracle newton {res.newton_iters} err pos {e[0]:.2e} "
            f"sigma {e[1]:.2e} p_n {e[2]:.2e} reaction {eR:.2e}")
        worst = np.maximum(worst, e)
        assert eR < 1e-3
    assert worst[0] < pos_tol and worst[1] < sig_tol and worst[2] < sig_tol, worst
    assert np.abs(gp.read("reaction")).max() > 0
    gp.close()
