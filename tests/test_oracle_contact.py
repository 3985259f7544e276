"""Pins of the oracle's barrier and indenter distance functions."""
import numpy as np
import pytest

from oracle import contact
from workloads import scenes

MM = 1e-3


def test_barrier_limits_and_smoothness():
    s = np.array([1e-12, 1e-8, 1e-4])
    b = contact.barrier(s)
    assert np.all(np.diff(b) < 0) and b[0] > 27          # grows without bound
    assert np.allclose(b / -np.log(s), 1.0, rtol=1e-3)   # ~ -ln s as s -> 0+
    assert contact.barrier(np.array([0.0]))[0] == np.inf
    assert contact.barrier(np.array([-1e-3]))[0] == np.inf
    one = np.array([1.0, 1.5])
    for f in (contact.barrier, contact.barrier_d1, contact.barrier_d2):
        assert np.all(f(one) == 0)
    # C2 at s = 1: values, first and second derivatives vanish from the left
    e = np.array([1 - 1e-6])
    assert abs(contact.barrier(e)[0]) < 1e-17
    assert abs(contact.barrier_d1(e)[0]) < 1e-11
    assert abs(contact.barrier_d2(e)[0]) < 1e-5
    grid = np.linspace(1e-4, 1 - 1e-4, 1001)
    assert np.all(contact.barrier_d2(grid) > 0)         # convex on (0, 1)
    assert np.all(contact.barrier_d1(grid) < 0)         # repulsive


def test_barrier_derivatives_fd():
    s = np.linspace(0.05, 0.95, 19)
    h = 1e-7
    d1 = (contact.barrier(s + h) - contact.barrier(s - h)) / (2 * h)
    d2 = (contact.barrier_d1(s + h) - contact.barrier_d1(s - h)) / (2 * h)
    assert np.abs(d1 - contact.barrier_d1(s)).max() / np.abs(d1).max() < 1e-6
    assert np.abs(d2 - contact.barrier_d2(s)).max() / np.abs(d2).max() < 1e-6


def _shapes():
    I = np.eye(3)
    return [
        scenes.Indenter(contact.SPHERE, (2 * MM, 0, 0, 0), I, np.zeros(3)),
        scenes.Indenter(contact.CYLINDER, (2.5 * MM, 5 * MM, 0, 0), I, np.zeros(3)),
        scenes.Indenter(contact.BOX, (3 * MM, 2 * MM, 1 * MM, 0), I, np.zeros(3)),
        scenes.Indenter(contact.TORUS, (4 * MM, 1 * MM, 0, 0), I, np.zeros(3)),
    ]


def _surface_samples(ind, n=200000, seed=0):
    """Dense samples of the indenter's boundary, written independently of
    the distance formulas (parametrisations of each surface)."""
    rng = np.random.default_rng(seed)
    p = ind.prm
    if ind.shape == contact.SPHERE:
        v = rng.standard_normal((n, 3))
        return p[0] * v / np.linalg.norm(v, axis=1)[:, None]
    if ind.shape == contact.CYLINDER:
        r, a = p[0], p[1]
        th = rng.uniform(0, 2 * np.pi, n)
        side = np.stack([r * np.cos(th), r * np.sin(th), rng.uniform(-a, a, n)], 1)
        rr = r * np.sqrt(rng.uniform(0, 1, n))
        cap = np.stack([rr * np.cos(th), rr * np.sin(th), np.where(rng.uniform(size=n) < .5, a, -a)], 1)
        return np.concatenate([side, cap])
    if ind.shape == contact.BOX:
        a = np.array(p[:3])
        pts = rng.uniform(-1, 1, (n, 3)) * a
        ax = rng.integers(0, 3, n)
        pts[np.arange(n), ax] = np.where(rng.uniform(size=n) < .5, -1, 1) * a[ax]
        return pts
    if ind.shape == contact.TORUS:
        Rt, rt = p[0], p[1]
        u, v = rng.uniform(0, 2 * np.pi, (2, n))
        return np.stack([(Rt + rt * np.cos(v)) * np.cos(u), (Rt + rt * np.cos(v)) * np.sin(u), rt * np.sin(v)], 1)
    raise ValueError


def _inside(ind, y):
    p = ind.prm
    if ind.shape == contact.SPHERE:
        return np.linalg.norm(y, axis=1) < p[0]
    if ind.shape == contact.CYLINDER:
        return (np.hypot(y[:, 0], y[:, 1]) < p[0]) & (np.abs(y[:, 2]) < p[1])
    if ind.shape == contact.BOX:
        return np.all(np.abs(y) < np.array(p[:3]), axis=1)
    if ind.shape == contact.TORUS:
        return np.hypot(np.hypot(y[:, 0], y[:, 1]) - p[0], y[:, 2]) < p[1]


@pytest.mark.parametrize("k", range(4))
def test_sdf_matches_brute_force_distance(k):
    ind = _shapes()[k]
    surf = _surface_samples(ind)
    rng = np.random.default_rng(10 + k)
    q = rng.uniform(-7 * MM, 7 * MM, (300, 3))
    phi, _, _ = contact.sdf_local(ind.shape, ind.prm, q)
    d = np.sqrt(((q[:, None, :] - surf[None, ::4, :]) ** 2).sum(-1)).min(1)
    d = np.where(_inside(ind, q), -d, d)
    # sampling error of the brute force is a small fraction of a millimetre
    assert np.abs(phi - d).max() < 0.1 * MM


@pytest.mark.parametrize("k", range(4))
def test_sdf_derivatives_fd(k):
    ind = _shapes()[k]
    rng = np.random.default_rng(20 + k)
    q = rng.uniform(-7 * MM, 7 * MM, (400, 3))
    phi, g, H = contact.sdf_local(ind.shape, ind.prm, q)
    keep = phi > 0.05 * MM          # outside, away from kinks of the distance
    q, phi, g, H = q[keep], phi[keep], g[keep], H[keep]
    assert np.allclose(np.linalg.norm(g, axis=1), 1.0, atol=1e-12)  # exact distance
    h = 1e-9
    for i in range(3):
        d = np.zeros(3); d[i] = h
        pp, gp, _ = contact.sdf_local(ind.shape, ind.prm, q + d)
        pm, gm, _ = contact.sdf_local(ind.shape, ind.prm, q - d)
        ok = np.abs(pp - pm) < 3 * h     # exclude samples straddling a region switch
        assert np.abs((pp - pm)[ok] / (2 * h) - g[ok, i]).max() < 1e-5
        fdH = (gp - gm) / (2 * h)
        scale = np.abs(H).max() + 1 / MM
        assert np.abs(fdH[ok] - H[ok, :, i]).max() / scale < 1e-4


def test_texture_is_lipschitz_lower_bound():
    ind = scenes.Indenter(contact.TEXTURE, (0.2 * MM, 2 * MM, 0, 0), np.eye(3), np.zeros(3))
    rng = np.random.default_rng(3)
    q = np.concatenate([rng.uniform(-3 * MM, 3 * MM, (400, 2)),
                        rng.uniform(-1.5 * MM, -0.2 * MM, (400, 1))], axis=1)
    phi, g, H = contact.sdf_local(ind.shape, ind.prm, q)
    assert (np.linalg.norm(g, axis=1) <= 1 + 1e-12).all()
    A, lam = ind.prm[0], ind.prm[1]
    u = np.linspace(-6 * MM, 6 * MM, 601)
    U, W = np.meshgrid(u, u, indexing="ij")
    surf = np.stack([U.ravel(), W.ravel(),
                     A * np.sin(2 * np.pi * U.ravel() / lam) * np.sin(2 * np.pi * W.ravel() / lam)], 1)
    d = np.array([np.sqrt(((surf - p) ** 2).sum(1)).min() for p in q[:60]])
    assert (phi[:60] <= d + 0.02 * MM).all() and (phi[:60] > 0).all()
    h = 1e-9
    for i in range(3):
        e = np.zeros(3); e[i] = h
        fd = (contact.sdf_local(4, ind.prm, q + e)[0] - contact.sdf_local(4, ind.prm, q - e)[0]) / (2 * h)
        assert np.abs(fd - g[:, i]).max() < 1e-6


def test_world_frame_and_barrier_fd():
    rng = np.random.default_rng(7)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    R = q * np.sign(np.linalg.det(q))
    dhat, kappa = 0.1 * MM, 1e3
    for shape, prm in ((contact.SPHERE, (3 * MM, 0, 0, 0)), (contact.TORUS, (4 * MM, 1 * MM, 0, 0)),
                       (contact.CYLINDER, (2.5 * MM, 5 * MM, 0, 0)), (contact.BOX, (3 * MM, 3 * MM, 3 * MM, 0))):
        ind = scenes.Indenter(shape, prm, R, np.array([1e-3, 2e-3, 3e-3]))
        # points at s in [0.05, 0.95] along random outward directions
        pts = []
        while len(pts) < 40:
            x = ind.c + rng.uniform(-9 * MM, 9 * MM, 3)
            phi, n, _ = contact.sdf(ind, x[None])
            if phi[0] <= 0:
                continue
            target = rng.uniform(0.05, 0.95) * dhat
            y = x[None] - (phi[0] - target) * n
            p2, _, _ = contact.sdf(ind, y)
            if abs(p2[0] - target) < 1e-3 * dhat:
                pts.append(y[0])
        xc = np.array(pts)
        area = rng.uniform(0.5, 2.0, len(xc)) * 1e-6
        E, g, H = contact.barrier_terms([ind], xc, area, dhat, kappa, project=False)
        h = 1e-11
        for i in range(3):
            d = np.zeros(3); d[i] = h
            fd = np.array([(contact.barrier_terms([ind], xc[k:k + 1] + d, area[k:k + 1], dhat, kappa)[0]
                            - contact.barrier_terms([ind], xc[k:k + 1] - d, area[k:k + 1], dhat, kappa)[0]) / (2 * h)
                           for k in range(len(xc))])
            assert np.abs(fd - g[:, i]).max() / np.abs(g).max() < 1e-5
            _, gp, _ = contact.barrier_terms([ind], xc + d, area, dhat, kappa)
            _, gm, _ = contact.barrier_terms([ind], xc - d, area, dhat, kappa)
            assert np.abs((gp - gm) / (2 * h) - H[:, :, i]).max() / np.abs(H).max() < 1e-5
        # Newton's third law: moving the indenter by dc changes E_b by -sum_k g_k . dc
        for i in range(3):
            d = np.zeros(3); d[i] = 1e-11
            ip = scenes.Indenter(shape, prm, R, ind.c + d)
            im = scenes.Indenter(shape, prm, R, ind.c - d)
            dE = (contact.barrier_terms([ip], xc, area, dhat, kappa)[0]
                  - contact.barrier_terms([im], xc, area, dhat, kappa)[0]) / 2e-11
            assert abs(dE + g[:, i].sum()) <= 1e-5 * np.abs(g).sum()


def test_projected_barrier_hessian_psd():
    rng = np.random.default_rng(8)
    ind = scenes.Indenter(contact.TORUS, (4 * MM, 1 * MM, 0, 0), np.eye(3), np.zeros(3))
    xc = np.stack([4 * MM + rng.uniform(-1.08, -1.01, 50) * MM * 1.0,
                   np.zeros(50), np.zeros(50)], 1)        # inner side: concave region
    _, _, H = contact.barrier_terms([ind], xc, np.full(50, 1e-6), 0.1 * MM, 1e3)
    assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()
