"""A pad refined by the library's terminal-edge bisection under the Sec.
III-A sizing field (irregular connectivity, graded sizes) stepped on the GPU
against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import context, errors, log, outputs, tc
from oracle import stepper
from workloads import scenes

pytestmark = pytest.mark.gpu

MM = 1e-3


@pytest.fixture(scope="module")
def episode():
    base = scenes.config1()
    X, T, _ = tc.refine_mesh(base.pad.X, base.pad.tets, l_contact=0.5 * MM, l_global=2.0 * MM)
    m = base.pad.material
    op = stepper.make_pad(X, T, m.E, m.nu, m.density)
    prm = stepper.StepParams(dt=base.params.dt, dhat=base.params.dhat, kappa=base.params.kappa, newton_tol=1e-10)
    poses = [base.pose(s) for s in range(1, 6)]
    refs = []
    for ind in poses:
        res = stepper.step(op, [ind], prm)
        stepper.commit(op, res)
        refs.append(dict(outputs(op, op.x, [ind], prm), newton=res.newton_iters))
    return X, T, m, poses, op, refs


@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4)])
def test_refined_pad_matches_oracle(episode, prec, newton_tol, cg_rel_tol, tol):
    X, T, m, poses, op, refs = episode
    gp = tc.Pad(context(), X, T, dict(E=m.E, nu=m.nu, density=m.density),
                tc.make_params(precision=prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol))
    info = gp.info
    log(f"refined pad: {T.shape[0]} tets, {X.shape[0]} verts, ELL width {info['ell_width']}")
    assert np.array_equal(gp.read("candidates"), op.cand)
    top = op.is_top.astype(bool)
    worst = np.zeros(3)
    for s, (ind, ref) in enumerate(zip(poses, refs), start=1):
        st = gp.step([ind])
        e = np.array(errors(gp, ref, X, top))
        log(f"{prec} step {s}: {st} oracle newton {ref['newton']} err pos {e[0]:.2e} sigma {e[1]:.2e} p_n {e[2]:.2e}")
        worst = np.maximum(worst, e)
    assert (worst < tol).all(), worst
    gp.close()
