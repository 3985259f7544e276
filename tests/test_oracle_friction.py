"""Pins of the oracle's lagged smoothed friction (Sec. III-B: friction ratio
and velocity threshold of the contact solver)."""
import numpy as np
import pytest
import scipy.optimize as so

from oracle import contact, extract, friction, stepper
from workloads import scenes

MM = 1e-3


def test_mollifier_closed_forms():
    eps = 0.3
    y = np.linspace(0, 2 * eps, 2001)
    f0, f1, f1p = friction.f0(y, eps), friction.f1(y, eps), friction.f1_prime(y, eps)
    assert np.isclose(friction.f0(0.0, eps), eps / 3)
    assert friction.f1(0.0, eps) == 0.0
    # C1 at eps: value and slope match the linear branch
    assert np.isclose(friction.f0(eps * (1 - 1e-12), eps), eps)
    assert np.isclose(friction.f1(eps * (1 - 1e-12), eps), 1.0)
    # f1 = f0', f1' = f1'' by central differences, f1 in [0, 1] and monotone
    h = 1e-7
    inner = (y > h) & (np.abs(y - eps) > 2 * h)
    d0 = (friction.f0(y + h, eps) - friction.f0(y - h, eps)) / (2 * h)
    d1 = (friction.f1(y + h, eps) - friction.f1(y - h, eps)) / (2 * h)
    assert np.allclose(d0[inner], f1[inner], atol=1e-7)
    assert np.allclose(d1[inner], f1p[inner], atol=1e-6)
    assert (f1 >= 0).all() and (f1 <= 1).all() and (np.diff(f1) >= -1e-15).all()
    assert (f1p >= 0).all()
    assert np.allclose(friction.f1_over_y(y[1:], eps), f1[1:] / y[1:])
    assert np.isclose(friction.f1_over_y(0.0, eps), 2 / eps)


def _random_lag(rng, C, M=2):
    lam = rng.uniform(0.1, 2.0, (M, C))
    n = rng.normal(size=(M, C, 3))
    n /= np.linalg.norm(n, axis=2, keepdims=True)
    w = rng.normal(scale=1e-4, size=(M, C, 3))
    return lam, n, w


@pytest.mark.parametrize("scale", [2e-5, 3e-4])      # slip below and above eps
def test_friction_derivatives_fd(scale):
    rng = np.random.default_rng(3)
    C, eps, mu, h2 = 6, 1e-4, 0.5, 1.0 / 3600
    lagged = _random_lag(rng, C)
    x_t = rng.normal(scale=1e-3, size=(C, 3))
    x = x_t + rng.normal(scale=scale, size=(C, 3))
    E, g, H = friction.terms(lagged, x, x_t, mu, eps, h2)
    d = 1e-9
    for k in range(C):
        for i in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, i] += d
            xm[k, i] -= d
            Ep = friction.terms(lagged, xp, x_t, mu, eps, h2)
            Em = friction.terms(lagged, xm, x_t, mu, eps, h2)
            assert abs((Ep[0] - Em[0]) / (2 * d) - g[k, i]) <= 1e-6 * np.abs(g).max()
            col = (Ep[1][k] - Em[1][k]) / (2 * d)
            assert np.abs(col - H[k, :, i]).max() <= 1e-5 * np.abs(H).max()
    # PSD, and no stiffness along the lagged normals' common complement
    assert np.linalg.eigvalsh(H).min() >= -1e-12 * np.abs(H).max()


def test_indenter_motion_is_rigid():
    rng = np.random.default_rng(4)
    p = rng.normal(size=(5, 3))
    old = scenes.Indenter(contact.SPHERE, (1.0, 0, 0, 0), np.eye(3), np.array([0.1, 0.2, 0.3]))
    shifted = scenes.Indenter(contact.SPHERE, (1.0, 0, 0, 0), np.eye(3), np.array([0.4, 0.2, 0.1]))
    assert np.allclose(friction.indenter_motion(old, shifted, p), [0.3, 0.0, -0.2])
    t = 0.3
    Rz = np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1.0]])
    turned = scenes.Indenter(contact.SPHERE, (1.0, 0, 0, 0), Rz, old.c)
    expect = (p - old.c) @ Rz.T + old.c - p
    assert np.allclose(friction.indenter_motion(old, turned, p), expect)
    # distances to the moving body are preserved by the motion
    moved = p + friction.indenter_motion(old, turned, p)
    assert np.allclose(contact.sdf(turned, moved)[0], contact.sdf(old, p)[0])


def _pressed_cube(mu_f):
    pad = scenes.one_cube_pad(1 * MM)
    X = pad.X
    fixed = np.where(X[:, 2] == 0, 7, 0).astype(np.uint8)
    op = stepper.make_pad(X, pad.tets, 0.3e6, 0.45, 1000.0, fixed=fixed)
    dhat = 0.1 * MM
    plate0 = scenes.Indenter(contact.BOX, (5 * MM, 5 * MM, 1 * MM, 0), np.eye(3),
                             np.array([0.5 * MM, 0.5 * MM, 1 * MM + 1 * MM + 0.5 * dhat]))
    prm = stepper.StepParams(newton_tol=1e-12, dhat=dhat, mu_f=mu_f, eps_v=0.01)
    res = stepper.step(op, [plate0], prm)
    stepper.commit(op, res)
    return op, plate0, prm


def test_sliding_force_is_mu_lambda_and_sticking_below():
    op, plate0, prm = _pressed_cube(0.5)
    for shift, sliding in ((2.0 * MM, True), (1e-3 * MM, False)):
        plate1 = scenes.Indenter(plate0.shape, plate0.prm, plate0.R, plate0.c + np.array([shift, 0, 0]))
        res = stepper.step(op, [plate1], prm, inds_prev=[plate0])
        lam, nrm, _ = res.fric[0]
        assert (lam > 0).any()
        cf = extract.contact_forces(op, res.x, [plate1], prm, fric=res.fric)
        cf0 = extract.contact_forces(op, res.x, [plate1], prm)       # barrier part only
        ff = cf["f"] - cf0["f"]                                       # friction part
        act = lam[0] > 0
        mag = np.linalg.norm(ff, axis=1)
        # tangential to the lagged normal, bounded by Coulomb's mu lambda
        assert np.abs(np.einsum("ki,ki->k", ff, nrm[0])).max() < 1e-12 * max(mag.max(), 1e-30)
        assert (mag <= prm.mu_f * lam[0] * (1 + 1e-12)).all()
        if sliding:
            # the plate drags the top along +x; the pad slides (slip >> eps)
            assert np.allclose(mag[act], prm.mu_f * lam[0][act], rtol=1e-9)
            assert (ff[act, 0] > 0).all()
        else:
            assert (mag[act] < 0.5 * prm.mu_f * lam[0][act]).all()


def test_friction_step_matches_generic_minimiser():
    op, plate0, prm = _pressed_cube(0.5)
    plate1 = scenes.Indenter(plate0.shape, plate0.prm, plate0.R, plate0.c + np.array([0.05 * MM, 0, 0]))
    res = stepper.step(op, [plate1], prm, inds_prev=[plate0])
    xhat = op.x + prm.dt * op.v
    free = op.free.ravel()
    x0 = res.x
    fric = res.fric
    scale = 1.0 / abs(stepper.energy(op, x0, xhat, [plate1], prm, fric))
    L = 1e-3

    def unpack(z):
        x = x0.ravel().copy()
        x[free] += L * z
        return x.reshape(-1, 3)

    r = so.minimize(lambda z: scale * stepper.energy(op, unpack(z), xhat, [plate1], prm, fric),
                    np.zeros(free.sum()),
                    jac=lambda z: scale * L * stepper.gradient(op, unpack(z), xhat, [plate1], prm, fric).ravel()[free],
                    method="BFGS", options=dict(gtol=1e-14, maxiter=20000))
    x_ref = unpack(r.x)
    disp = np.abs(res.x - op.X).max()
    assert np.abs(x_ref - res.x).max() <= 1e-7 * disp


def test_sliding_impulse_closed_form():
    """A near-massless-stiffness heavy cube under a plate sweeping past it:
    each contact vertex's tangential momentum change over the step is the
    Coulomb impulse h mu lambda (so m dx = h^2 mu lambda), pinning the h^2
    weight of the friction potential against inertia."""
    pad = scenes.one_cube_pad(1 * MM)
    X = pad.X
    fixed = np.where(X[:, 2] == 0, 7, 0).astype(np.uint8)
    op = stepper.make_pad(X, pad.tets, 1e-3, 0.45, 1e8, fixed=fixed)
    dhat = 0.1 * MM
    plate0 = scenes.Indenter(contact.BOX, (5 * MM, 5 * MM, 1 * MM, 0), np.eye(3),
                             np.array([0.5 * MM, 0.5 * MM, 2 * MM + 0.5 * dhat]))
    plate1 = scenes.Indenter(plate0.shape, plate0.prm, plate0.R, plate0.c + np.array([2 * MM, 0, 0]))
    prm = stepper.StepParams(newton_tol=1e-13, dhat=dhat, mu_f=0.5, eps_v=0.01)
    res = stepper.step(op, [plate1], prm, inds_prev=[plate0])
    lam = res.fric[0][0][0]
    k = op.cand
    assert (lam > 0).all() and len(k) >= 2
    dx = res.x[k] - X[k]
    h2 = prm.dt ** 2
    assert np.allclose(op.mass[k] * dx[:, 0], h2 * prm.mu_f * lam, rtol=1e-6)
    assert np.abs(dx[:, 1]).max() < 1e-6 * np.abs(dx[:, 0]).max()
    assert (2 * MM - np.abs(dx[:, 0]) > 10 * prm.eps_v * prm.dt).all()     # slip >> eps: sliding


def test_lag_normal_is_unit_and_lambda_the_force_for_a_non_distance_phi():
    """The texture plate's phi is a scaled height function, |grad phi| < 1
    off its extrema.  The lag must hold the unit contact normal and the
    barrier force's magnitude, lambda = -kappa A b'(phi / d_hat) |grad phi|,
    so that lambda n is the contact force and the slip projector I - n n^T
    is a projector; then the friction gradient is the derivative of the
    friction energy (central differences) for vertices under the plate."""
    dhat, kappa, mu, eps, h2 = 1e-3, 1e3, 0.5, 1e-4, 1.0 / 3600
    A, lam_t = 0.2e-3, 2e-3
    plate = scenes.Indenter(contact.TEXTURE, (A, lam_t, 0, 0), np.eye(3), np.zeros(3))
    rng = np.random.default_rng(9)
    x_t = np.column_stack([rng.uniform(0, 4e-3, 8), rng.uniform(0, 4e-3, 8), np.full(8, -0.5e-3)])
    area = rng.uniform(0.5e-6, 1.5e-6, 8)
    lam, nrm, w = friction.lag([plate], [plate], x_t, area, dhat, kappa)
    phi, g, _ = contact.sdf(plate, x_t)
    assert np.allclose(np.linalg.norm(nrm[0], axis=1), 1.0, atol=1e-12)
    assert (np.linalg.norm(g, axis=1) < 1 - 1e-3).any()             # not a distance
    _, gb, _ = contact.barrier_terms([plate], x_t, area, dhat, kappa)
    assert np.allclose(lam[0][:, None] * nrm[0], -gb, rtol=1e-12, atol=0)
    x = x_t + rng.normal(scale=3e-5, size=x_t.shape)
    E, gf, _ = friction.terms((lam, nrm, w), x, x_t, mu, eps, h2)
    d = 1e-10
    for k in range(8):
        for i in range(3):
            xp, xm = x.copy(), x.copy()
            xp[k, i] += d
            xm[k, i] -= d
            fd = (friction.terms((lam, nrm, w), xp, x_t, mu, eps, h2)[0]
                  - friction.terms((lam, nrm, w), xm, x_t, mu, eps, h2)[0]) / (2 * d)
            assert abs(fd - gf[k, i]) <= 1e-6 * np.abs(gf).max()
