"""GPU parity against the FP64 oracle through the C ABI (config-1 sizes:
1,944 tets = 7.6 element tiles, 520 vertices = 2+ vertex tiles, ragged)."""
import numpy as np
import pytest

from gpu_util import (context, errors, gpu_pad, log, min_surface_gap, oracle_episode, oracle_pad, outputs, tc,
                      voigt_to_mat)
from oracle import contact, extract, material, stepper, surface
from workloads import scenes

pytestmark = pytest.mark.gpu
MM = 1e-3


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_setup_matches_oracle(prec):
    ep = scenes.config1()
    gp = gpu_pad(context(), ep.pad, prec)
    op = oracle_pad(ep.pad)
    assert np.array_equal(gp.read("tets"), ep.pad.tets)
    assert np.array_equal(gp.read("surface_tris"), op.tris)
    assert np.array_equal(gp.read("surface_parent"), op.parent)
    assert np.array_equal(gp.read("surface_is_top"), op.is_top)
    assert np.array_equal(gp.read("candidates"), op.cand)
    assert np.array_equal(gp.read("fixed"), op.fixed)
    assert np.allclose(gp.read("mass"), op.mass, rtol=1e-13, atol=0)
    assert np.allclose(gp.read("cand_rest_area"), op.area, rtol=1e-13, atol=0)
    assert np.array_equal(gp.read("positions"), ep.pad.X)
    assert gp.info["n_surface_tris"] == 684 and gp.info["n_candidates"] == 214


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 2e-5)])
def test_extraction_on_prescribed_positions(prec, tol):
    ep = scenes.config1()
    ctx = context()
    gp = gpu_pad(ctx, ep.pad, prec)
    op = oracle_pad(ep.pad)
    rng = np.random.default_rng(7)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = q * np.sign(np.linalg.det(q))
    Fbar = np.array([[1.03, 0.02, 0.0], [-0.01, 0.98, 0.015], [0.0, 0.01, 0.95]])
    cases = {
        "patch": ep.pad.X @ Fbar.T,
        "rotated_patch": ep.pad.X @ (Q @ Fbar).T,
        "random": ep.pad.X + 2e-5 * rng.standard_normal(ep.pad.X.shape),
    }
    ind = ep.pose(6)
    prm = stepper.StepParams()
    for name, x in cases.items():
        gp.write("positions", x)
        gp.extract([ind])
        ref = outputs(op, x, [ind], prm)
        sig = voigt_to_mat(gp.read("sigma"))
        scale = np.linalg.norm(ref["sigma"], axis=(1, 2)).max()
        e = np.linalg.norm(sig - ref["sigma"], axis=(1, 2)).max() / scale
        log(f"{prec} {name}: sigma rel err {e:.2e}")
        assert e < tol
        for f, key in (("traction", "t"), ("tangential", "tt"), ("tri_normal", "n")):
            g = gp.read(f).astype(np.float64)
            s = max(np.abs(ref[key]).max(), 1e-300)
            assert np.abs(g - ref[key]).max() / s < 10 * tol, f
        pn = gp.read("pressure").astype(np.float64)
        assert np.abs(pn - ref["pn"]).max() / np.abs(ref["pn"]).max() < 10 * tol
        assert np.allclose(gp.read("tri_area"), ref["area"], rtol=10 * tol)
        if name == "rotated_patch":
            s_bar = material.cauchy((Q @ Fbar)[None], op.mu[0], op.lam[0], op.alpha[0])[0]
            assert np.abs(sig - s_bar).max() / np.abs(s_bar).max() < tol
        # contact path (float64 on both sides)
        cf = ref["cf"]
        for f, key in (("contact_force", "f"), ("contact_normal", "n"), ("contact_area", "area"),
                       ("contact_fn", "f_n"), ("contact_ft", "f_tau"), ("contact_pressure", "p")):
            g = gp.read(f)
            s = max(np.abs(cf[key]).max(), 1e-300)
            assert np.abs(g - cf[key]).max() / s < 1e-9, f
        if np.abs(cf["f"]).max() > 0:
            assert np.allclose(gp.read("reaction"), cf["reaction"], rtol=1e-9, atol=1e-15)


def _episode(prec, steps, newton_tol, cg_rel_tol, **kw):
    ep = scenes.config1()
    ctx = context()
    gp = gpu_pad(ctx, ep.pad, prec, newton_tol=newton_tol, cg_rel_tol=cg_rel_tol, **kw)
    op, refs = oracle_episode(ep, steps, tol=1e-10)
    X = ep.pad.X
    top = op.is_top.astype(bool)
    worst = np.zeros(3)
    for s in range(1, steps + 1):
        st = gp.step([ep.pose(s)])
        e = np.array(errors(gp, refs[s - 1], X, top))
        R = gp.read("reaction")
        Rref = refs[s - 1]["cf"]["reaction"]
        eR = np.abs(R - Rref).max() / max(np.abs(Rref).max(), 1e-12)
        ts = gp.read("traction_sum")
        eT = np.abs(ts - refs[s - 1]["tsum"]).max() / max(np.abs(refs[s - 1]["tsum"]).max(), 1e-12)
        cf = refs[s - 1]["cf"]
        eP = np.abs(gp.read("contact_pressure") - cf["p"]).max() / max(np.abs(cf["p"]).max(), 1e-300)
        gap = min_surface_gap(op, gp.read("positions"), [ep.pose(s)])
        log(f"{prec} step {s}: {st} oracle newton {refs[s - 1]['newton']} "
            f"err pos {e[0]:.2e} sigma {e[1]:.2e} p_n {e[2]:.2e} reaction {eR:.2e} tsum {eT:.2e} "
            f"p_k {eP:.2e} min gap {gap:.3e}")
        worst = np.maximum(worst, e)
        assert eR < 1e-3 and eT < 1e-3 and eP < 1e-3
        assert gap > 0
    return worst


def test_config1_episode_fp64():
    worst = _episode("fp64", 10, 1e-9, 1e-9)
    assert (worst < 1e-4).all(), worst


def test_config1_episode_mixed():
    worst = _episode("mixed", 10, 1e-6, 1e-4)
    assert (worst < 1e-4).all(), worst


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_config1_episode_warm_start(prec):
    """CG started from the best multiple of the previous Newton direction
    (cg_warm): the same minimiser as the oracle's exact Newton."""
    worst = _episode(prec, 10, 1e-9 if prec == "fp64" else 1e-6, 1e-9 if prec == "fp64" else 1e-4, cg_warm=1)
    assert (worst < 1e-4).all(), worst


def test_no_contact_keeps_rest_state():
    ep = scenes.config1()
    for prec in ("fp64", "mixed"):
        gp = gpu_pad(context(), ep.pad, prec)
        far = ep.indenter.at_depth(-5 * MM)      # 5 mm above the start pose
        for _ in range(3):
            st = gp.step([far])
            assert st.status == 0
        assert np.array_equal(gp.read("positions"), ep.pad.X)
        assert np.abs(gp.read("sigma")).max() < 1e-6
        assert np.abs(gp.read("reaction")).max() == 0.0


def test_batch_equals_alone_bitwise():
    ctx = context()
    pads = [scenes.config1().pad, scenes.box_pad(0.012, 0.010, 0.003, 7, 5, 3),
            scenes.dome_pad(0.019, 0.016, 0.003, 9, 8, 3)]
    eps = [scenes.config1()]
    for p in pads[1:]:
        ind = scenes.place_indenter(p, scenes.SPHERE, (0.5 * p.dims[0], 0.45 * p.dims[1]), 1e-4,
                                    sphere_radius=3 * MM)
        eps.append(scenes.Episode(p, ind, 0.4 * MM, 4, scenes.Params()))
    for prec in ("mixed", "fp64"):
        alone = [gpu_pad(ctx, e.pad, prec) for e in eps]
        mixed = [gpu_pad(ctx, e.pad, prec) for e in eps]
        for s in (1, 2, 3):
            inds = [[e.pose(s)] for e in eps]
            sa = [g.step(i) for g, i in zip(alone, inds)]
            sb = tc.step_batch(ctx, mixed, inds)
            for a, b, x, y in zip(alone, mixed, sa, sb):
                assert x.newton_iters == y.newton_iters and x.cg_iters == y.cg_iters
                for f in ("positions", "sigma", "pressure", "contact_force"):
                    assert np.array_equal(a.read(f), b.read(f)), (prec, s, f)
        log(prec, [str(x) for x in sb])


def test_rerun_is_bitwise_reproducible():
    """The same steps from the same state give bitwise equal results: after a
    reset, and on a fresh context (no scheduling-dependent arithmetic)."""
    pads = [scenes.box_pad(0.018, 0.014, 0.004, 30, 24, 6), scenes.config1().pad]
    eps = []
    for p in pads:
        ind = scenes.place_indenter(p, scenes.TEXTURE if len(eps) == 0 else scenes.SPHERE,
                                    (0.5 * p.dims[0], 0.45 * p.dims[1]), 1e-4, sphere_radius=4 * MM)
        eps.append(scenes.Episode(p, ind, 0.5 * MM, 6, scenes.Params()))
    runs = []
    for fresh in (True, False, True):
        if fresh or not runs:
            ctx = tc.Context(0)
            gp = [gpu_pad(ctx, e.pad, "mixed") for e in eps]
        else:
            for g in gp:
                g.reset()
        for s in range(1, 5):
            tc.step_batch(ctx, gp, [[e.pose(s)] for e in eps])
        runs.append([(g.read("positions"), g.read("sigma")) for g in gp])
    for r in runs[1:]:
        for (xa, sa), (xb, sb) in zip(runs[0], r):
            assert np.array_equal(xa, xb) and np.array_equal(sa, sb)


def test_failures_are_transactional():
    ep = scenes.config1()
    ctx = context()
    gp = gpu_pad(ctx, ep.pad, "mixed")
    gp.step([ep.pose(1)])
    gp.step([ep.pose(2)])
    x0, v0 = gp.read("positions"), gp.read("velocities")
    # Newton capped at one iteration with a tight tolerance
    p = tc.make_params(precision="mixed", max_newton=1, newton_tol=1e-12)
    gp.set_params(p)
    st = gp.step([ep.pose(3)], raise_on_error=False)
    assert st.status == tc._abi.E_NOT_CONVERGED
    assert np.array_equal(gp.read("positions"), x0) and np.array_equal(gp.read("velocities"), v0)
    # a pose whose escape direction is blocked: top vertices may only move
    # along z inside a vertical cylinder
    cube = scenes.one_cube_pad(1 * MM)
    fixed = np.where(cube.X[:, 2] == 0, 7, 3).astype(np.uint8)
    gc = gpu_pad(ctx, cube, "fp64", fixed=fixed)
    cyl = dict(shape=tc.CYLINDER, prm=(0.8 * MM, 5 * MM), R=np.eye(3), c=(0.5e-3, 0.5e-3, 0.5e-3))
    st = gc.step([cyl], raise_on_error=False)
    assert st.status == tc._abi.E_INFEASIBLE
    assert np.array_equal(gc.read("positions"), cube.X)


def test_save_load_resume_bitwise():
    ep = scenes.config1()
    ctx = context()
    a = gpu_pad(ctx, ep.pad, "mixed")
    b = gpu_pad(ctx, ep.pad, "mixed")
    for s in (1, 2, 3):
        a.step([ep.pose(s)])
    blob = a.save_state()
    b.load_state(blob)
    for s in (4, 5):
        a.step([ep.pose(s)])
        b.step([ep.pose(s)])
    assert np.array_equal(a.read("positions"), b.read("positions"))
    assert np.array_equal(a.read("velocities"), b.read("velocities"))


def test_tiny_meshes_match_oracle():
    ctx = context()
    for which in ("tet", "cube"):
        if which == "tet":
            p = scenes.one_tet_pad()
            ind = scenes.Indenter(contact.SPHERE, (2 * MM, 0, 0, 0), np.eye(3),
                                  np.array([0.1 * MM, 0.1 * MM, 3 * MM - 0.05 * MM]))
        else:
            p = scenes.one_cube_pad(1 * MM)
            ind = scenes.Indenter(contact.SPHERE, (2 * MM, 0, 0, 0), np.eye(3),
                                  np.array([0.6 * MM, 0.45 * MM, 3 * MM - 0.08 * MM]))
        fixed = np.where(p.X[:, 2] == 0, 7, 0).astype(np.uint8)
        op = oracle_pad(p, fixed=fixed)
        res = stepper.step(op, [ind], stepper.StepParams(newton_tol=1e-12))
        gp = gpu_pad(ctx, p, "fp64", fixed=fixed, newton_tol=1e-10, cg_rel_tol=1e-12)
        st = gp.step([ind])
        x = gp.read("positions")
        disp = np.abs(res.x - p.X).max()
        log(which, st, np.abs(x - res.x).max() / disp)
        assert np.abs(x - res.x).max() <= 1e-6 * disp


@pytest.mark.parametrize("n", [24, 40])
def test_high_valence_fan_matches_oracle(n):
    """A disc pad of n prism sectors: its axis vertices hold about 2n
    Hessian blocks per row, so the SpMV takes several slots per lane (n =
    24) or one thread per row (n = 40, more than 64 slots).  A sphere
    pressed on the axis, FP64 and mixed, against the oracle."""
    from workloads import meshes
    X, T = meshes.fan_prisms(n, 6e-3, 2e-3, 2)
    mat = scenes.Material(0.3e6, 0.45, 1000.0)
    pad = scenes.Pad("fan", X, T, mat, (12e-3, 12e-3, 2e-3))
    params = scenes.Params()
    start = scenes.place_indenter(pad, scenes.SPHERE, (0.0, 0.0), params.dhat, sphere_radius=5e-3)
    op = stepper.make_pad(X, T, mat.E, mat.nu, mat.density)
    prm = stepper.StepParams(dt=params.dt, dhat=params.dhat, kappa=params.kappa, newton_tol=1e-10)
    refs = []
    for s in range(1, 5):
        res = stepper.step(op, [start.at_depth(0.08e-3 * s)], prm)
        stepper.commit(op, res)
        refs.append(op.x.copy())
    for prec, ntol, ctol, tol in (("fp64", 1e-9, 1e-9, 1e-6), ("mixed", 1e-7, 1e-4, 1e-4)):
        gp = gpu_pad(context(), pad, prec, newton_tol=ntol, cg_rel_tol=ctol)
        assert gp.info["ell_width"] > (64 if n == 40 else 32)
        worst = 0.0
        for s, ref in enumerate(refs, start=1):
            st = gp.step([start.at_depth(0.08e-3 * s)])
            x = gp.read("positions")
            worst = max(worst, np.abs(x - ref).max() / max(np.abs(ref - X).max(), 1e-300))
        log(f"fan n={n} {prec}: ELL width {gp.info['ell_width']}, last {st}, worst pos err {worst:.2e}")
        assert worst < tol
        gp.close()
