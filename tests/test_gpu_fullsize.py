"""GPU checks at the workloads' full sizes, where the oracle cannot replay
whole episodes: the graded 122,850-tet pad under its five indenters, and the
60-pad batch in the launch configuration the benchmark times.

After the GPU has run the steps, the oracle (FP64) checks the GPU's final
state of a step from the outside:
  * stationarity: the oracle's own Newton direction of the incremental
    potential at the GPU's positions (x_hat from the GPU's state before the
    step) is within the convergence tolerance, i.e. the GPU stopped at the
    minimiser the oracle defines (Sec. III-B, Alg. 2 Physics);
  * extraction: sigma (Eq. 4), traction, pressure and tangential traction
    (Alg. 1, Eq. 6-9) and contact forces (Alg. 2 Contact) recomputed by the
    oracle from the GPU's positions, element by element;
  * identities: t_tau . n = 0 and reaction = -sum f_k.
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gpu_util import (context, free_surface_vertices, gpu_pad, log, oracle_pad, surface_gap, tc,
                      voigt_to_mat)
from oracle import extract, mesh_pairs, stepper
from workloads import scenes

pytestmark = pytest.mark.gpu

# mixed precision: FP32 element arithmetic, FP64 positions and reductions
SIGMA_TOL = 1e-4
FORCE_TOL = 1e-8
KKT_FACTOR = 3.0        # oracle direction <= KKT_FACTOR * newton_tol * L


def oracle_direction(op, x_prev, v_prev, x, inds, prm, fric=None):
    """The oracle's Newton direction at x for the step that started at
    (x_prev, v_prev): PSD-projected Hessian, Jacobi-preconditioned CG."""
    xhat = x_prev + prm.dt * v_prev
    g = stepper.gradient(op, x, xhat, inds, prm, fric=fric).ravel()
    H = stepper.hessian(op, x, inds, prm, fric=fric)
    free = op.free.ravel()
    Hff = H[free][:, free]
    pf, info = spla.cg(Hff, -g[free], rtol=1e-7, maxiter=200000, M=sp.diags(1.0 / Hff.diagonal()))
    assert info == 0
    return float(np.abs(pf).max())


FIELDS = ("positions", "sigma", "traction", "pressure", "tangential", "tri_normal", "contact_force",
          "contact_pressure", "reaction")


def snapshot(gp):
    return {f: gp.read(f) for f in FIELDS}


def check_state(out, op, x_prev, v_prev, inds, prm, label, inds_prev=None):
    """out: the GPU's outputs after the step (snapshot); inds_prev: the
    indenter poses of the step before (the friction lag)."""
    x = out["positions"]
    fric = None
    if prm.mu_f > 0:
        op.x = x_prev.copy()
        fric = stepper.friction_lag(op, inds, prm, inds_prev)
    p_inf = oracle_direction(op, x_prev, v_prev, x, inds, prm, fric)
    tol = prm.newton_tol * op.L_diag
    # extraction from the GPU's positions
    sig_ref = extract.cauchy_per_tet(op, x)
    sig = voigt_to_mat(out["sigma"])
    # stresses below 1e-6 mu are roundoff (a pad not yet touched is at rest:
    # exactly zero on the GPU, ~1e-11 Pa in the oracle's F = Ds Dm^-1)
    floor = 1e-6 * float(np.max(op.mu))
    smax = max(np.linalg.norm(sig_ref, axis=(1, 2)).max(), floor)
    e_sig = np.linalg.norm(sig - sig_ref, axis=(1, 2)).max() / smax
    t_ref, pn_ref, tt_ref, n_ref, _ = extract.surface_traction(op, x, sig_ref)
    t = out["traction"].astype(np.float64)
    pn = out["pressure"].astype(np.float64)
    tt = out["tangential"].astype(np.float64)
    e_t = np.abs(t - t_ref).max() / max(np.abs(t_ref).max(), floor)
    e_pn = np.abs(pn - pn_ref).max() / max(np.abs(pn_ref).max(), floor)
    cf_ref = extract.contact_forces(op, x, inds, prm, fric=fric)
    f = out["contact_force"]
    fscale = max(np.abs(cf_ref["f"]).max(), 1e-300)
    e_f = np.abs(f - cf_ref["f"]).max() / fscale
    e_p = np.abs(out["contact_pressure"] - cf_ref["p"]).max() / max(np.abs(cf_ref["p"]).max(), 1e-300)
    reaction = out["reaction"]
    e_r = np.abs(reaction + f.sum(axis=0)).max() / max(np.abs(reaction).max(), 1e-300)
    gap = surface_gap(free_surface_vertices(op.tets, op.fixed), x, inds)
    n = out["tri_normal"].astype(np.float64)
    orth = np.abs(np.einsum("si,si->s", tt, n)).max() / max(np.abs(t).max(), floor)
    log(f"{label}: oracle |p|inf / tol {p_inf / tol:.3f}, sigma {e_sig:.2e}, traction {e_t:.2e}, "
        f"pressure {e_pn:.2e}, contact force {e_f:.2e}, contact pressure {e_p:.2e}, reaction {e_r:.1e}, "
        f"t_tau.n {orth:.1e}, |reaction| {np.linalg.norm(reaction):.4e} N, min surface gap {gap:.3e} m")
    assert p_inf <= KKT_FACTOR * tol, label
    assert e_sig <= SIGMA_TOL and e_t <= SIGMA_TOL and e_pn <= SIGMA_TOL, label
    assert e_f <= FORCE_TOL and e_p <= FORCE_TOL and e_r <= 1e-12 and orth <= 1e-5, label
    assert gap > 0, label


@pytest.mark.parametrize("i", range(5), ids=["sphere", "cylinder", "cube_edge", "torus", "texture"])
def test_graded_pad_episode(i):
    pad = _graded_pad()
    ep = scenes.config2(i, pad)
    ctx = context()
    gp = gpu_pad(ctx, pad, "mixed")
    op = oracle_pad(pad)
    prm = stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa,
                             newton_tol=ep.params.newton_tol)
    free_v = free_surface_vertices(pad.tets, op.fixed)
    t0 = time.perf_counter()
    newton = []
    for s in range(1, ep.n_steps + 1):
        if s in (15, ep.n_steps):
            x_prev, v_prev = gp.read("positions"), gp.read("velocities")
        st = gp.step([ep.pose(s)])
        newton.append(st.newton_iters)
        gap = surface_gap(free_v, gp.read("positions"), [ep.pose(s)])
        assert gap > 0, (s, gap)
        if s in (15, ep.n_steps):
            check_state(snapshot(gp), op, x_prev, v_prev, [ep.pose(s)], prm,
                        f"graded {ep.indenter.shape} step {s}")
    log(f"graded pad, indenter {i}: {ep.n_steps} steps in {time.perf_counter() - t0:.2f} s, newton {newton}")
    gp.close()


_PAD = {}


def _graded_pad():
    if "p" not in _PAD:
        _PAD["p"] = scenes.config2_pad()
    return _PAD["p"]


# (step, pads) checked after the batch run; four groups keep each test short
BATCH_CHECKS = [(33, (0, 4, 8, 12, 16)), (33, (20, 24, 28, 32, 36)), (33, (40, 44, 48, 52, 56)),
                (12, (2, 13, 27, 41, 58))]


@pytest.fixture(scope="module")
def batch60_run():
    """The 60-pad batch with the benchmark's solver settings and launch
    shape, steps 1-33; keeps the GPU states the checks need."""
    envs = scenes.config3()
    ctx = tc.Context(0)
    kw = dict(precision="mixed", cg_rel_tol=0.2, cg_eta_max=0.2, cg_forcing=2, hess_proj=4, ls_expand=4,
              init_guess=1)
    pads = []
    for e in envs:
        m = e.pad.material
        pads.append(tc.Pad(ctx, e.pad.X, e.pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                           tc.make_params(dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa,
                                          newton_tol=e.params.newton_tol, **kw)))
    want = {}
    for s, ks in BATCH_CHECKS:
        want.setdefault(s, set()).update(ks)
    saved = {}
    free_v = [free_surface_vertices(e.pad.tets, pads[k].read("fixed")) for k, e in enumerate(envs)]
    t0 = time.perf_counter()
    newton, gaps = [], []
    for s in range(1, 34):
        prev = {k: (pads[k].read("positions"), pads[k].read("velocities")) for k in want.get(s, ())}
        st = tc.step_batch(ctx, pads, [[e.pose(s)] for e in envs])
        assert all(x.status == 0 for x in st)
        newton.append(max(x.newton_iters for x in st))
        gaps.append(min(surface_gap(free_v[k], pads[k].read("positions"), [e.pose(s)])
                        for k, e in enumerate(envs)))
        assert gaps[-1] > 0, (s, gaps[-1])
        if s % 5 == 0:
            log(f"  step {s}: newton max {newton[-1]}, smallest free-surface gap {gaps[-1]:.3e} m")
        for k in want.get(s, ()):
            saved[(s, k)] = (prev[k][0], prev[k][1], snapshot(pads[k]))
    log(f"batch60: 33 steps in {time.perf_counter() - t0:.1f} s, newton max per step {newton}, "
        f"smallest free-surface gap {min(gaps):.3e} m")
    for p in pads:
        p.close()
    ctx.close()
    return envs, saved


@pytest.mark.parametrize("step,ks", BATCH_CHECKS, ids=["last_a", "last_b", "last_c", "mid"])
def test_batch60_bench_configuration(batch60_run, step, ks):
    envs, saved = batch60_run
    for k in ks:
        e = envs[k]
        x_prev, v_prev, out = saved[(step, k)]
        prm = stepper.StepParams(dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa,
                                 newton_tol=e.params.newton_tol)
        check_state(out, oracle_pad(e.pad), x_prev, v_prev, [e.pose(step)], prm,
                    f"batch pad {k} ({e.pad.name}, {e.pad.tets.shape[0]} tets, indenter "
                    f"{e.indenter.shape}) step {step}")


# pads checked per variant at the last step: every indenter shape the
# variant changes (pads 0-5 carry cube, sphere, sphere, cylinder, torus,
# texture) on all three pad shapes
VARIANT_CHECKS = {"friction": (0, 3, 5), "slide": (0, 3, 5), "layers": (1, 4, 5), "mesh": (0, 1, 3, 4),
                  "mesh2": (0, 1, 3, 13), "paper60": (0, 1, 2, 3, 4)}


@pytest.fixture(scope="module", params=sorted(VARIANT_CHECKS))
def variant_run(request):
    """One variant of the 60-pad batch (friction, two layers, mesh
    indenters) in the benchmark's settings, steps 1-33, as the benchmark
    sets the pads up."""
    kind = request.param
    envs = scenes.paper60() if kind == "paper60" else scenes.config3_variant(kind)
    ctx = tc.Context(0)
    kw = dict(precision="mixed", cg_rel_tol=0.2, cg_eta_max=0.2, cg_forcing=2, hess_proj=4, ls_expand=4,
              init_guess=1)
    ids, pads = {}, []
    try:
        return _run_variant(kind, envs, ctx, kw, ids, pads)
    finally:
        for p in pads:
            p.close()
        for i in ids.values():
            ctx.remove_mesh(i)
        ctx.close()


def _run_variant(kind, envs, ctx, kw, ids, pads):
    for e in envs:
        m = e.pad.material
        mats, idx = [dict(E=m.E, nu=m.nu, density=m.density)], None
        if e.layers is not None:
            idx = e.layers[0]
            mats = [dict(E=q.E, nu=q.nu, density=q.density) for q in e.layers[1]]
        if e.indenter.mesh is not None and id(e.indenter.mesh) not in ids:
            ids[id(e.indenter.mesh)] = ctx.add_mesh(*e.indenter.mesh)
        pads.append(tc.Pad(ctx, e.pad.X, e.pad.tets, mats,
                           tc.make_params(dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa,
                                          newton_tol=e.params.newton_tol, friction=e.friction,
                                          mesh_contact=e.mesh_contact, **kw),
                           tet_material=idx))

    def poses(e, s):
        ind = e.pose(s)
        if ind.mesh is None:
            return [ind]
        return [dict(shape=tc.MESH, prm=ind.prm, R=ind.R, c=ind.c, mesh_id=ids[id(ind.mesh)])]

    last, saved, newton, gaps = 33, {}, [], []
    free_v = [free_surface_vertices(e.pad.tets, pads[k].read("fixed")) for k, e in enumerate(envs)]
    t0 = time.perf_counter()
    for s in range(1, last + 1):
        prev = {k: (pads[k].read("positions"), pads[k].read("velocities")) for k in VARIANT_CHECKS[kind]} \
            if s == last else {}
        st = tc.step_batch(ctx, pads, [poses(e, s) for e in envs], raise_on_error=False)
        assert all(x.status == 0 for x in st), (s, [(k, x) for k, x in enumerate(st) if x.status])
        newton.append(max(x.newton_iters for x in st))
        # brute-force distances to triangle meshes are slow in the oracle:
        # every third step there, every step for the analytic shapes
        if kind not in ("mesh", "mesh2") or s % 3 == 0 or s == last:
            gaps.append(min(surface_gap(free_v[k], pads[k].read("positions"), [e.pose(s)])
                            for k, e in enumerate(envs)))
            assert gaps[-1] > 0, (s, gaps[-1])
        if s % 3 == 0:
            log(f"  step {s}: newton max {newton[-1]}, smallest free-surface gap {gaps[-1]:.3e} m")
        for k in prev:
            saved[k] = (prev[k][0], prev[k][1], snapshot(pads[k]))
    log(f"batch60-{kind}: {last} steps in {time.perf_counter() - t0:.1f} s, newton max per step {newton}, "
        f"smallest free-surface gap {min(gaps):.3e} m")
    return kind, envs, last, saved


def test_batch60_variants(variant_run):
    """The 60-pad batch with friction (press then slide), with two-layer
    pads, or with triangle-mesh indenters, checked at the last step by the
    oracle with the same physics: stationarity of the incremental potential
    (friction lagged from the GPU's previous state and the previous poses),
    extraction and contact forces (friction included)."""
    kind, envs, step, saved = variant_run
    for k, (x_prev, v_prev, out) in saved.items():
        e = envs[k]
        m = e.pad.material
        if e.layers is not None:
            idx, mats = e.layers
            op = stepper.make_pad(e.pad.X, e.pad.tets, np.array([q.E for q in mats])[idx],
                                  np.array([q.nu for q in mats])[idx],
                                  np.array([q.density for q in mats])[idx], fixed=e.pad.fixed)
        else:
            op = stepper.make_pad(e.pad.X, e.pad.tets, m.E, m.nu, m.density, fixed=e.pad.fixed)
        prm = stepper.StepParams(dt=e.params.dt, dhat=e.params.dhat, kappa=e.params.kappa,
                                 newton_tol=e.params.newton_tol, mu_f=e.friction, eps_v=0.01,
                                 mesh_pairs=int(e.mesh_contact))
        check_state(out, op, x_prev, v_prev, [e.pose(step)], prm,
                    f"batch60-{kind} pad {k} ({e.pad.name}, {e.pad.tets.shape[0]} tets, indenter "
                    f"{e.indenter.shape}) step {step}", inds_prev=[e.pose(step - 1)])
        if e.mesh_contact == 2:
            # no mesh vertex or edge through the pad surface
            through = [q for q in mesh_pairs.signed_pairs(e.pose(step), out["positions"], op.tris, op.pedges,
                                                           e.params.dhat) if q[2] < 0]
            assert not through, through[:3]
        if kind == "friction":
            r = out["reaction"].ravel()
            log(f"  tangential / normal reaction {np.hypot(r[0], r[1]) / max(abs(r[2]), 1e-300):.3f}")


@pytest.mark.parametrize("kind", ["graded", "refined"])
def test_large_pad_final_state(kind):
    """The 1.2 M-tet pad (the largest workload; graded grid, or the 1.35 M
    tets of the library's adaptive refinement) through its whole episode,
    60 steps to 1.0 mm, in mixed precision with the benchmark's solver
    settings; the oracle then checks the final step from the outside:
    stationarity with its own Newton direction, extraction element by
    element, contact forces and the identities."""
    if kind == "graded":
        ep = scenes.config5()
    else:
        base, kw = scenes.config5_refine_base()
        X, T, _ = tc.refine_mesh(base.X, base.tets, max_tets=4_000_000, **kw)
        ep = scenes.config5_refined(X, T)
    ctx = tc.Context(0)
    m = ep.pad.material
    gp = tc.Pad(ctx, ep.pad.X, ep.pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                tc.make_params(precision="mixed", dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa,
                               newton_tol=ep.params.newton_tol, cg_rel_tol=0.2, cg_eta_max=0.2, cg_forcing=2,
                               hess_proj=4, ls_expand=4, init_guess=1))
    gp_width = gp.info["ell_width"]
    try:
        newton = []
        for s in range(1, ep.n_steps + 1):
            if s == ep.n_steps:
                x_prev, v_prev = gp.read("positions"), gp.read("velocities")
            newton.append(gp.step([ep.pose(s)]).newton_iters)
        out = snapshot(gp)
    finally:
        gp.close()
        ctx.close()
    log(f"large pad, {kind} ({ep.pad.tets.shape[0]} tets, ELL width {gp_width}): newton per step {newton}")
    prm = stepper.StepParams(dt=ep.params.dt, dhat=ep.params.dhat, kappa=ep.params.kappa,
                             newton_tol=ep.params.newton_tol)
    t0 = time.perf_counter()
    check_state(out, oracle_pad(ep.pad), x_prev, v_prev, [ep.pose(ep.n_steps)], prm,
                f"large pad, {kind}, step {ep.n_steps}")
    log(f"oracle check {time.perf_counter() - t0:.0f} s")
    assert np.abs(out["reaction"]).max() > 0


def _hertz_run(ep, steps=(12, 18, 24)):
    m = ep.pad.material
    mu = m.E / (2 * (1 + m.nu))
    lam = m.E * m.nu / ((1 + m.nu) * (1 - 2 * m.nu)) - mu
    E_eff = mu * (3 * lam + 2 * mu) / (lam + mu)
    nu_eff = lam / (2 * (lam + mu))
    E_star = E_eff / (1 - nu_eff ** 2)
    R = ep.indenter.prm[0]
    ctx = tc.Context(0)
    pad = tc.Pad(ctx, ep.pad.X, ep.pad.tets, dict(E=m.E, nu=m.nu, density=m.density),
                 tc.make_params(precision="mixed", dt=ep.params.dt, dhat=ep.params.dhat,
                                kappa=ep.params.kappa, newton_tol=ep.params.newton_tol))
    z_top = ep.pad.X[:, 2].max()
    cand = pad.read("candidates")
    out = []
    for s in range(1, max(steps) + 1):
        pose = ep.pose(s)
        assert pad.step([pose]).status == 0
        if s in steps:
            x = pad.read("positions")[cand]
            gap = np.linalg.norm(x - pose.c[None], axis=1).min() - R
            delta = (z_top - (pose.c[2] - R)) - gap
            F = pad.read("reaction").ravel()[2]
            F_h = 4.0 / 3.0 * E_star * np.sqrt(R) * delta ** 1.5
            log(f"{ep.pad.tets.shape[0]} tets step {s}: delta {delta * 1e3:.4f} mm (gap {gap * 1e6:.2f} um), "
                f"contact radius {np.sqrt(R * delta) * 1e3:.3f} mm, F {F:.5f} N, Hertz {F_h:.5f} N, ratio {F / F_h:.3f}")
            out.append((delta, F, F / F_h))
    pad.close()
    ctx.close()
    return out


def test_large_pad_hertz_sanity():
    """Loose physical check (not a parity pin): a 3 mm sphere pressed into the
    5 mm thick pad against Hertz, F = (4/3) E* sqrt(R) delta^1.5, while the
    contact radius stays small against the thickness.  The rest-stable shift
    makes the small-strain Lame pair (mu, lambda - mu), hence E*; delta is the
    sphere's overlap with the undeformed surface less the barrier gap left at
    the contact.  Linear tets at nu_eff = 0.44 are too stiff (volumetric
    locking, few elements across the contact), so the check is the power law
    on the 1.2 M-tet pad and a force excess that shrinks under refinement."""
    coarse = _hertz_run(scenes.config5(target=0.15e6))
    fine = _hertz_run(scenes.config5())
    (d1, F1, _), (d2, F2, _) = fine[1], fine[2]
    exponent = np.log(F2 / F1) / np.log(d2 / d1)
    log(f"exponent (delta {d1 * 1e3:.3f} -> {d2 * 1e3:.3f} mm): {exponent:.3f}")
    assert abs(exponent - 1.5) < 0.1
    for (_, _, rc), (_, _, rf) in zip(coarse, fine):
        assert 1.0 <= rf < rc, (rf, rc)
    assert fine[-1][2] < 1.4
