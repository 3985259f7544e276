"""Pins of the oracle's constitutive law (Eq. 1-4) against closed forms,
finite differences and invariants."""
import numpy as np
import pytest

from oracle import fem, material
from workloads import scenes

E0, NU0 = 0.3e6, 0.45


def rand_F(rng, n, spread=0.25):
    F = np.eye(3)[None] + spread * rng.standard_normal((n, 3, 3))
    J = np.linalg.det(F)
    F[J < 0.2] = np.eye(3)           # keep the samples well away from inversion
    return F


def test_lame_inverts_to_E_nu():
    # Eq. 1 and the textbook inverse relations E = mu(3 lam + 2 mu)/(lam + mu),
    # nu = lam / (2 (lam + mu)) recover the inputs.
    for E, nu in ((0.3e6, 0.45), (1e6, 0.40), (0.1e6, 0.48), (2e5, 0.0)):
        mu, lam = material.lame(E, nu)
        assert np.isclose(mu * (3 * lam + 2 * mu) / (lam + mu), E, rtol=1e-13)
        if nu > 0:
            assert np.isclose(lam / (2 * (lam + mu)), nu, rtol=1e-13)
    mu, lam = material.lame(E0, NU0)
    assert np.isclose(mu, 103448.27586206897, rtol=1e-12)
    assert np.isclose(lam, 931034.4827586207, rtol=1e-12)


def test_rest_state_is_stress_free():
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    I = np.eye(3)[None]
    assert np.abs(material.first_piola(I, mu, lam, a)).max() < 1e-9 * mu
    assert np.abs(material.cauchy(I, mu, lam, a)).max() < 1e-9 * mu
    # the literal shift alpha = 1 of Eq. 2 as printed leaves P(I) = mu I
    P1 = material.first_piola(I, mu, lam, material.rest_shift(mu, lam, literal=True))
    assert np.allclose(P1[0], mu * np.eye(3), rtol=1e-14)


def test_eq3_equals_eq4():
    rng = np.random.default_rng(0)
    F = rand_F(rng, 200)
    mu, lam = material.lame(E0, NU0)
    for a in (material.rest_shift(mu, lam), 1.0):
        s3 = material.cauchy_from_piola(F, mu, lam, a)
        s4 = material.cauchy(F, mu, lam, a)
        assert np.abs(s3 - s4).max() <= 1e-12 * np.abs(s4).max()
        assert np.allclose(s4, np.swapaxes(s4, 1, 2), atol=1e-9)


def test_piola_is_energy_derivative_fd():
    rng = np.random.default_rng(1)
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    F = rand_F(rng, 20)
    P = material.first_piola(F, mu, lam, a)
    h = 1e-6
    fd = np.zeros_like(F)
    for i in range(3):
        for j in range(3):
            d = np.zeros((3, 3)); d[i, j] = h
            fd[:, i, j] = (material.energy_density(F + d, mu, lam, a)
                           - material.energy_density(F - d, mu, lam, a)) / (2 * h)
    assert np.abs(fd - P).max() / np.abs(P).max() < 1e-6


def test_hessian_is_piola_derivative_fd():
    rng = np.random.default_rng(2)
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    F = rand_F(rng, 20)
    H = material.energy_hessian(F, mu, lam, a)
    h = 1e-6
    fd = np.zeros_like(H)
    for k in range(9):
        d = np.zeros(9); d[k] = h
        d = d.reshape(3, 3)
        fd[:, :, k] = ((material.first_piola(F + d, mu, lam, a)
                        - material.first_piola(F - d, mu, lam, a)) / (2 * h)).reshape(-1, 9)
    assert np.abs(fd - H).max() / np.abs(H).max() < 1e-6


def test_det_hessian_is_cofactor_derivative():
    rng = np.random.default_rng(3)
    F = rand_F(rng, 10)
    HJ = material.det_hessian(F)
    h = 1e-6
    for k in range(9):
        d = np.zeros(9); d[k] = h
        d = d.reshape(3, 3)
        col = ((material.cofactor(F + d) - material.cofactor(F - d)) / (2 * h)).reshape(-1, 9)
        assert np.abs(col - HJ[:, :, k]).max() < 1e-8
    # cof F = J F^-T
    assert np.allclose(material.cofactor(F),
                       np.linalg.det(F)[:, None, None] * np.linalg.inv(F).transpose(0, 2, 1))


def test_rest_hessian_eigenvalues_closed_form():
    # At F = I: rotations are null (0 x3), deviatoric modes 2 mu (x5), the
    # volumetric mode 3 lam - mu (effective first Lame parameter lam - mu).
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    w = np.linalg.eigvalsh(material.energy_hessian(np.eye(3)[None], mu, lam, a)[0])
    expect = np.sort([0, 0, 0] + [2 * mu] * 5 + [3 * lam - mu])
    assert np.allclose(w, expect, atol=1e-8 * lam)


def test_small_strain_effective_lame():
    # uniaxial strain eps_xx: sigma_xx ~ (2 mu + lam') eps, sigma_yy ~ lam' eps,
    # lam' = lam - mu with the rest-stable shift.
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    eps = 1e-7
    F = np.diag([1 + eps, 1, 1])[None]
    s = material.cauchy(F, mu, lam, a)[0]
    assert np.isclose(s[1, 1] / eps, lam - mu, rtol=1e-5)
    assert np.isclose(s[0, 0] / eps, 2 * mu + lam - mu, rtol=1e-5)


def test_projection_psd_and_idempotent():
    rng = np.random.default_rng(4)
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    F = rand_F(rng, 100, spread=0.4)
    F[:10] = np.diag([0.7, 0.8, 0.9])       # compression: indefinite Hessian
    H = material.energy_hessian(F, mu, lam, a)
    assert np.linalg.eigvalsh(H).min() < 0          # some samples are indefinite
    Hp = material.project_psd(H)
    scale = np.abs(H).max(axis=(1, 2))
    assert (np.linalg.eigvalsh(Hp).min(axis=1) >= -1e-12 * scale).all()
    assert np.abs(material.project_psd(Hp) - Hp).max() < 1e-9 * scale.max()
    # already-PSD matrices are left unchanged
    spd = np.linalg.eigvalsh(H).min(axis=1) > 0
    assert np.abs(Hp[spd] - H[spd]).max() < 1e-9 * scale.max()


def test_patch_test_uniform_stretch():
    # x = Fbar X on a Kuhn grid: every tet sees F = Fbar (linear completeness)
    # and Eq. 4 gives sigma_ii = mu s_i^2 / J + lam (J - alpha) for a diagonal Fbar.
    pad = scenes.box_pad(0.018, 0.014, 0.004, 6, 5, 3)
    Dminv, vol = fem.rest_data(pad.X, pad.tets)
    s = np.array([1.05, 0.97, 0.9])
    Fbar = np.diag(s)
    x = pad.X @ Fbar.T
    F = fem.deformation_gradient(x, pad.tets, Dminv)
    assert np.abs(F - Fbar).max() < 1e-12
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    sig = material.cauchy(F, mu, lam, a)
    J = s.prod()
    expect = np.diag(mu * s ** 2 / J + lam * (J - a))
    assert np.abs(sig - expect).max() < 1e-10 * np.abs(expect).max()


def test_rotation_covariance():
    rng = np.random.default_rng(5)
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = q * np.sign(np.linalg.det(q))
    F = rand_F(rng, 30)
    s = material.cauchy(F, mu, lam, a)
    sQ = material.cauchy(Q[None] @ F, mu, lam, a)
    assert np.abs(sQ - Q[None] @ s @ Q.T[None]).max() < 1e-9 * np.abs(s).max()
    # pure rotation is stress free
    assert np.abs(material.cauchy(Q[None], mu, lam, a)).max() < 1e-9 * mu


def test_element_gradient_hessian_fd():
    rng = np.random.default_rng(6)
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 1e-3
    tets = np.array([[0, 1, 2, 3]], np.int32)
    Dminv, vol = fem.rest_data(X, tets)
    mu, lam = material.lame(E0, NU0)
    a = material.rest_shift(mu, lam)
    for trial in range(5):
        x = X + 1.5e-4 * rng.standard_normal(X.shape)
        g = fem.elastic_gradient(x, tets, Dminv, vol, mu, lam, a)[0]
        K = fem.elastic_hessian(x, tets, Dminv, vol, mu, lam, a, project=False)[0]
        h = 1e-9
        fd_g = np.zeros(12)
        fd_K = np.zeros((12, 12))
        for k in range(12):
            d = np.zeros(12); d[k] = h
            d = d.reshape(4, 3)
            ep = fem.elastic_energy(x + d, tets, Dminv, vol, mu, lam, a)[0]
            em = fem.elastic_energy(x - d, tets, Dminv, vol, mu, lam, a)[0]
            fd_g[k] = (ep - em) / (2 * h)
            fd_K[:, k] = (fem.elastic_gradient(x + d, tets, Dminv, vol, mu, lam, a)[0]
                          - fem.elastic_gradient(x - d, tets, Dminv, vol, mu, lam, a)[0]) / (2 * h)
        assert np.abs(fd_g - g).max() / np.abs(g).max() < 1e-6
        assert np.abs(fd_K - K).max() / np.abs(K).max() < 1e-6
        # rigid translations are in the null space of the element Hessian
        t = np.tile(rng.standard_normal(3), 4)
        assert np.abs(K @ t).max() < 1e-9 * np.abs(K).max()
