"""Pins of the oracle's implicit step (incremental potential + Newton) and of
the extraction outputs (Eq. 4, Alg. 1, Alg. 2 contact path)."""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import contact, extract, material, stepper, surface
from workloads import scenes

MM = 1e-3


def _free_min(op, inds, prm, x0):
    """Generic quasi-Newton minimiser (BFGS) of the same E over the free
    components, started from x0."""
    xhat = op.x + prm.dt * op.v
    free = op.free.ravel()
    scale = 1.0 / max(abs(stepper.energy(op, x0, xhat, inds, prm)), 1e-30)
    L = 1e-3

    def unpack(z):
        x = x0.ravel().copy()
        x[free] = x0.ravel()[free] + L * z
        return x.reshape(-1, 3)

    def f(z):
        return scale * stepper.energy(op, unpack(z), xhat, inds, prm)

    def g(z):
        return scale * L * stepper.gradient(op, unpack(z), xhat, inds, prm).ravel()[free]

    r = so.minimize(f, np.zeros(free.sum()), jac=g, method="BFGS",
                    options=dict(gtol=1e-13, maxiter=20000))
    return unpack(r.x)


@pytest.mark.parametrize("which", ["tet", "cube"])
def test_newton_matches_generic_minimiser(which):
    if which == "tet":
        p = scenes.one_tet_pad()
        ind = scenes.Indenter(contact.SPHERE, (2 * MM, 0, 0, 0), np.eye(3),
                              np.array([0.1 * MM, 0.1 * MM, 1 * MM + 2 * MM - 0.05 * MM]))
    else:
        p = scenes.one_cube_pad(1 * MM)
        ind = scenes.Indenter(contact.SPHERE, (2 * MM, 0, 0, 0), np.eye(3),
                              np.array([0.6 * MM, 0.45 * MM, 1 * MM + 2 * MM - 0.08 * MM]))
    base = np.where(p.X[:, 2] == 0, 7, 0).astype(np.uint8)
    op = stepper.make_pad(p.X, p.tets, 0.3e6, 0.45, 1000.0, fixed=base)
    prm = stepper.StepParams(newton_tol=1e-12)
    res = stepper.step(op, [ind], prm)
    x0 = stepper.feasible_start(op, op.x, [ind], prm)
    xb = _free_min(op, [ind], prm, x0)
    disp = np.abs(res.x - op.X).max()
    assert disp > 1e-6
    assert np.abs(xb - res.x).max() <= 1e-7 * disp
    # energy decreases monotonically along the Newton iterates
    assert np.all(np.diff(res.energies) <= 1e-12 * abs(res.energies[0]))


def test_dirichlet_patch_test():
    # all boundary vertices held at Fbar X: Newton puts the interior on Fbar X
    pad = scenes.box_pad(6 * MM, 5 * MM, 4 * MM, 4, 3, 3)
    tris, _ = surface.surface_triangles(pad.tets)
    bnd = np.zeros(pad.X.shape[0], bool)
    bnd[np.unique(tris)] = True
    op = stepper.make_pad(pad.X, pad.tets, 0.3e6, 0.45, 1000.0,
                          fixed=np.where(bnd, 7, 0).astype(np.uint8))
    Fbar = np.array([[1.04, 0.02, 0.0], [0.01, 0.97, 0.03], [0.0, -0.02, 0.95]])
    target = pad.X @ Fbar.T
    op.x = np.where(bnd[:, None], target, pad.X)
    prm = stepper.StepParams(newton_tol=1e-12, quasi_static=True)
    res = stepper.step(op, [], prm)
    assert np.abs(res.x - target).max() < 1e-12
    assert (~bnd).sum() == 3 * 2 * 2


def _uniform_compression(depth):
    Lx, Ly, H = 18 * MM, 14 * MM, 4 * MM
    pad = scenes.box_pad(Lx, Ly, H, 6, 5, 2)
    X = pad.X
    fixed = np.zeros(X.shape[0], np.uint8)
    fixed[X[:, 2] == 0] = 4                                         # rollers: z fixed
    fixed[np.nonzero((X == 0).all(axis=1))[0]] = 7                  # pin origin
    fixed[np.nonzero((X[:, 0] == Lx) & (X[:, 1] == 0) & (X[:, 2] == 0))[0]] = 6
    op = stepper.make_pad(X, pad.tets, 0.3e6, 0.45, 1000.0, fixed=fixed)
    dhat = 0.1 * MM
    plate = scenes.Indenter(contact.BOX, (60 * MM, 60 * MM, 5 * MM, 0), np.eye(3),
                            np.array([Lx / 2, Ly / 2, H + dhat + 5 * MM - depth]))
    prm = stepper.StepParams(newton_tol=1e-12, quasi_static=True, dhat=dhat)
    res = stepper.step(op, [plate], prm)
    return op, plate, prm, res


def test_uniform_compression_closed_form_and_traction_balance():
    op, plate, prm, res = _uniform_compression(0.2 * MM)
    x = res.x
    H = 4 * MM
    top = op.X[:, 2] == H
    s_z = x[top, 2].mean() / H
    assert np.ptp(x[top, 2]) < 1e-12                                   # homogeneous
    sig = extract.cauchy_per_tet(op, x)
    mu, lam, a = op.mu[0], op.lam[0], op.alpha[0]
    # lateral stretch from sigma_xx = 0: mu s_x^2 / J + lam (J - a) = 0, J = s_x^2 s_z
    s_x = so.brentq(lambda s: mu * s * s / (s * s * s_z) + lam * (s * s * s_z - a), 0.5, 1.5)
    J = s_x ** 2 * s_z
    szz = mu * s_z ** 2 / J + lam * (J - a)
    scale = abs(szz)
    assert np.abs(sig[:, 2, 2] - szz).max() < 1e-8 * scale
    assert np.abs(sig[:, 0, 0]).max() < 1e-8 * scale
    assert np.abs(sig[:, 1, 1]).max() < 1e-8 * scale
    assert np.allclose(x[:, 0], s_x * op.X[:, 0], atol=1e-12)
    # summed Alg. 1 traction over the contact face balances the reaction
    cf = extract.contact_forces(op, x, [plate], prm)
    ts = extract.top_traction_sum(op, x, sig)
    R = cf["reaction"]
    assert np.linalg.norm(ts + R) <= 1e-3 * np.linalg.norm(R)
    assert np.allclose(cf["f"].sum(axis=0), -R)
    # compression gives negative normal pressure on the contact face (Eq. 8 sign)
    _, pn, _, _, _ = extract.surface_traction(op, x, sig)
    assert (pn[op.is_top.astype(bool)] < 0).all()


def test_two_layer_confined_compression_closed_form():
    """Per-tet materials: a soft layer on a stiff one, lateral motion blocked,
    pressed by a flat plate (quasi-static).  Each layer is in uniaxial strain
    F = diag(1, 1, s_i), J = s_i; equilibrium makes sigma_zz the same in both,
    and with Eq. 2 (rest-stable shift) sigma_zz = (mu_i + lam_i) s_i -
    lam_i alpha_i, so the layer stretches follow from the top height alone."""
    Lx, Ly, H = 18 * MM, 14 * MM, 4 * MM
    pad = scenes.box_pad(Lx, Ly, H, 5, 4, 4)
    X, T = pad.X, pad.tets
    zc = X[T, 2].mean(axis=1)
    soft = zc > 2 * MM
    E = np.where(soft, 0.15e6, 1.2e6)
    nu = np.where(soft, 0.47, 0.42)
    rho = np.where(soft, 1050.0, 1200.0)
    fixed = np.full(X.shape[0], 3, np.uint8)                         # x, y blocked
    fixed[X[:, 2] == 0] = 7
    op = stepper.make_pad(X, T, E, nu, rho, fixed=fixed)
    dhat = 0.1 * MM
    depth = 0.3 * MM
    plate = scenes.Indenter(contact.BOX, (60 * MM, 60 * MM, 5 * MM, 0), np.eye(3),
                            np.array([Lx / 2, Ly / 2, H + dhat + 5 * MM - depth]))
    prm = stepper.StepParams(newton_tol=1e-12, quasi_static=True, dhat=dhat)
    x = stepper.step(op, [plate], prm).x
    top = X[:, 2] == H
    assert np.ptp(x[top, 2]) < 1e-12
    h_top = x[top, 2].mean()
    mu, lam, a = op.mu, op.lam, op.alpha
    k = np.array([np.argmax(soft), np.argmax(~soft)])                 # one tet per layer
    # h_top = 2 mm (s_soft + s_stiff), s_i = (sz + lam_i a_i) / (mu_i + lam_i)
    c = (mu[k] + lam[k])
    sz = (h_top / (2 * MM) - np.sum(lam[k] * a[k] / c)) / np.sum(1.0 / c)
    s_i = (sz + lam[k] * a[k]) / c
    F = np.stack([x[T[:, j]] - x[T[:, 0]] for j in (1, 2, 3)], axis=2) @ op.Dminv
    for layer, sel in enumerate((soft, ~soft)):
        expect = np.diag([1.0, 1.0, s_i[layer]])
        assert np.abs(F[sel] - expect).max() < 1e-9
    sig = extract.cauchy_per_tet(op, x)
    scale = abs(sz)
    assert np.abs(sig[:, 2, 2] - sz).max() < 1e-8 * scale
    sxx = mu[k] / s_i + lam[k] * (s_i - a[k])                         # lateral stress per layer
    for layer, sel in enumerate((soft, ~soft)):
        assert np.abs(sig[sel, 0, 0] - sxx[layer]).max() < 1e-8 * scale
        assert np.abs(sig[sel, 1, 1] - sxx[layer]).max() < 1e-8 * scale
    assert s_i[0] < s_i[1] < 1.0                                      # the soft layer yields more
    # per-tet density enters the lumped mass
    assert np.isclose(op.mass.sum(), np.sum(rho * op.vol))


def test_extraction_identities_on_config1_step():
    ep = scenes.config1()
    op = stepper.make_pad(ep.pad.X, ep.pad.tets, 0.3e6, 0.45, 1000.0)
    prm = stepper.StepParams()
    ind = ep.pose(3)
    res = stepper.step(op, [ind], prm)
    x = res.x
    sig = extract.cauchy_per_tet(op, x)
    t, pn, tt, n, area = extract.surface_traction(op, x, sig)
    scale = np.abs(t).max()
    assert np.abs(np.einsum("si,si->s", tt, n)).max() < 1e-12 * scale          # Eq. 9
    assert np.allclose((t * t).sum(1), pn ** 2 + (tt * tt).sum(1), rtol=1e-10, atol=1e-12 * scale ** 2)
    assert np.allclose(pn, np.einsum("si,sij,sj->s", n, sig[op.parent], n), rtol=1e-12,
                       atol=1e-14 * scale)                                        # Eq. 8
    cf = extract.contact_forces(op, x, [ind], prm)
    assert np.allclose(cf["f_n"] + cf["f_tau"], cf["f"])
    assert np.abs(np.einsum("ki,ki->k", cf["f_tau"], cf["n"])).max() < 1e-12 * np.abs(cf["f"]).max()
    assert np.allclose(cf["p"] * cf["area"], np.linalg.norm(cf["f"], axis=1))
    assert cf["reaction"][2] > 0                     # indenter is pushed back up
    # patch test of Alg. 1: uniform stretch -> t_j = sigma_bar n_j on every face
    Fbar = np.diag([1.03, 0.98, 0.96])
    xs = op.X @ Fbar.T
    s_bar = material.cauchy(Fbar[None], op.mu[0], op.lam[0], op.alpha[0])[0]
    sig_s = extract.cauchy_per_tet(op, xs)
    t2, _, _, n2, _ = extract.surface_traction(op, xs, sig_s)
    assert np.abs(t2 - n2 @ s_bar.T).max() < 1e-9 * np.abs(s_bar).max()


def test_infeasible_pose_is_reported():
    # top vertices may only move along z while a vertical cylinder encloses
    # them: the escape direction (radial) is blocked, so no feasible start
    p = scenes.one_cube_pad(1 * MM)
    fixed = np.where(p.X[:, 2] == 0, 7, 3).astype(np.uint8)
    op = stepper.make_pad(p.X, p.tets, 0.3e6, 0.45, 1000.0, fixed=fixed)
    ind = scenes.Indenter(contact.CYLINDER, (0.8 * MM, 5 * MM, 0, 0), np.eye(3),
                          np.array([0.5e-3, 0.5e-3, 0.5e-3]))
    with pytest.raises(stepper.Infeasible):
        stepper.step(op, [ind], stepper.StepParams())
