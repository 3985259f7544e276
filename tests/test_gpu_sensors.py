"""Sensor pad stand-ins beyond the three benchmark shapes (Sec. IV-D runs
GelSight Mini, DIGIT and 9DTact; their CAD is not available): a gel whose
top is a cylindrical cap, and a dual-layer gel whose thin surface layer is
stiffer than its base (9DTact's order).  Each is pressed by a sphere and
stepped on the GPU against the FP64 oracle with the same geometry and
per-tet materials, step by step, in both precisions; the no-penetration
invariant holds at every free surface vertex."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import context, errors, log, min_surface_gap, outputs, tc
from oracle import stepper
from workloads import scenes

pytestmark = pytest.mark.gpu


_REF = {}


def _oracle_refs(kind, ep, op):
    """Oracle outputs after every step of the episode (computed once per
    pad kind, shared by both precisions)."""
    if kind not in _REF:
        prm = stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa, newton_tol=1e-10)
        refs = []
        for s in range(1, ep.n_steps + 1):
            ind = [ep.pose(s)]
            res = stepper.step(op, ind, prm)
            stepper.commit(op, res)
            refs.append((res.newton_iters, outputs(op, op.x, ind, prm)))
        _REF[kind] = refs
    return _REF[kind]


def _setup(kind, prec, newton_tol, cg_rel_tol):
    if kind == "curved":
        ep = scenes.curved_gel_episode()
        mats, idx = [ep.pad.material], None
    else:
        ep, idx, mats = scenes.stiff_skin_episode()
    pad = ep.pad
    gp = tc.Pad(context(), pad.X, pad.tets, [dict(E=m.E, nu=m.nu, density=m.density) for m in mats],
                tc.make_params(precision=prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol),
                tet_material=idx)
    if idx is None:
        op = stepper.make_pad(pad.X, pad.tets, mats[0].E, mats[0].nu, mats[0].density)
    else:
        op = stepper.make_pad(pad.X, pad.tets, np.array([m.E for m in mats])[idx],
                              np.array([m.nu for m in mats])[idx], np.array([m.density for m in mats])[idx])
    return ep, gp, op


@pytest.mark.parametrize("kind", ["curved", "stiff_skin"])
@pytest.mark.parametrize("prec,newton_tol,cg_rel_tol,tol", [("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-6, 1e-4, 1e-4)])
def test_sensor_pad_episode_matches_oracle(kind, prec, newton_tol, cg_rel_tol, tol):
    ep, gp, op = _setup(kind, prec, newton_tol, cg_rel_tol)
    assert np.array_equal(gp.read("candidates"), op.cand)
    assert np.allclose(gp.read("cand_rest_area"), op.area, rtol=1e-13, atol=0)
    top = op.is_top.astype(bool)
    refs = _oracle_refs(kind, ep, op)
    worst = np.zeros(3)
    for s in range(1, ep.n_steps + 1):
        ind = [ep.pose(s)]
        newton, ref = refs[s - 1]
        st = gp.step(ind)
        if np.abs(ref["x"] - ep.pad.X).max() < 1e-12:
            # no contact yet: both sides at rest (the relative norms are 0/0)
            assert np.abs(gp.read("positions") - ref["x"]).max() < 1e-15 and st.status == 0
            continue
        e = np.array(errors(gp, ref, ep.pad.X, top))
        R, Rref = gp.read("reaction"), ref["cf"]["reaction"]
        eR = np.abs(R - Rref).max() / max(np.abs(Rref).max(), 1e-12)
        cp = gp.read("contact_pressure")
        eP = np.abs(cp - ref["cf"]["p"]).max() / max(np.abs(ref["cf"]["p"]).max(), 1e-300)
        gap = min_surface_gap(op, gp.read("positions"), ind)
        log(f"{kind} {prec} step {s}: {st} oracle newton {newton} err pos {e[0]:.2e} sigma {e[1]:.2e} "
            f"p_n {e[2]:.2e} reaction {eR:.2e} p_k {eP:.2e} gap {gap:.2e}")
        worst = np.maximum(worst, e)
        assert eR < 1e-3 and eP < 1e-3 and gap > 0
    assert (worst < tol).all(), worst
    assert np.abs(gp.read("reaction")).max() > 0
    gp.close()
