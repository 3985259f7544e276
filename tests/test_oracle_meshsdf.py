"""Pins of the oracle's signed distance to a rigid triangle mesh."""
import numpy as np
import pytest

from oracle import contact, meshsdf, stepper
from workloads import meshes, scenes

MM = 1e-3


def test_box_mesh_equals_analytic_box():
    """Outside a convex polytope and inside it, the distance to its surface is
    the box SDF: values, gradients and Hessians agree."""
    a = (1.0, 2.0, 0.5)
    mesh = meshsdf.MeshData(*meshes.box_surface(*a))
    rng = np.random.default_rng(0)
    y = rng.uniform(-3, 3, (4000, 3))
    phi, g, H = meshsdf.sdf_local(mesh, y)
    phi0, g0, H0 = contact.sdf_local(contact.BOX, (*a, 0.0), y)
    assert (phi < 0).sum() > 50 and (phi > 0).sum() > 50
    assert np.abs(phi - phi0).max() < 1e-12
    assert np.abs(g - g0).max() < 1e-9
    assert np.abs(H - H0).max() < 1e-9 * np.abs(H0).max()


def test_icosphere_within_chord_error():
    r = 1.0
    V, F = meshes.icosphere(r, 3)
    mesh = meshsdf.MeshData(V, F)
    # the mesh is inscribed: its surface lies between r - delta and r
    delta = r - np.min(np.einsum("ki,ki->k", mesh.fn, V[F[:, 0]]))
    rng = np.random.default_rng(1)
    y = rng.normal(size=(3000, 3)) * rng.uniform(0.2, 2.0, (3000, 1))
    phi, _, _ = meshsdf.sdf_local(mesh, y)
    diff = phi - (np.linalg.norm(y, axis=1) - r)
    assert diff.min() >= -1e-12 and diff.max() <= delta * (1 + 1e-9)
    assert delta < 0.01


def test_torus_distance_brute_force_samples_and_sign():
    V, F = meshes.torus_surface(4.0, 1.0, 24, 12)
    mesh = meshsdf.MeshData(V, F)
    rng = np.random.default_rng(2)
    y = rng.uniform(-6, 6, (300, 3)) * np.array([1, 1, 0.4])
    phi, _, _ = meshsdf.sdf_local(mesh, y)
    # dense surface samples: their nearest is never closer than the
    # distance, and approaches it within the sampling resolution
    n = 400
    u, w = rng.random((2, len(F), n))
    flip = u + w > 1
    u, w = np.where(flip, 1 - u, u), np.where(flip, 1 - w, w)
    P = (V[F[:, 0]][:, None] + u[..., None] * (V[F[:, 1]] - V[F[:, 0]])[:, None]
         + w[..., None] * (V[F[:, 2]] - V[F[:, 0]])[:, None]).reshape(-1, 3)
    dmin = np.array([np.sqrt(((P - q) ** 2).sum(1)).min() for q in y])
    assert (dmin >= np.abs(phi) - 1e-12).all()
    assert (dmin - np.abs(phi)).max() < 0.1
    # sign: the hole and far points are outside, the tube core inside
    core = np.array([[4.0 * np.cos(t), 4.0 * np.sin(t), 0.0] for t in np.linspace(0, 6, 7)])
    assert (meshsdf.sdf_local(mesh, core)[0] < -0.9).all()
    assert meshsdf.sdf_local(mesh, [[0.0, 0.0, 0.0]])[0][0] > 2.9
    # inside/outside agrees with the analytic torus wherever it is clear
    ana = contact.sdf_local(contact.TORUS, (4.0, 1.0, 0, 0), y)[0]
    clear = np.abs(ana) > 0.1
    assert (np.sign(phi[clear]) == np.sign(ana[clear])).all()


def test_mesh_sdf_derivatives_fd():
    V, F = meshes.torus_surface(4.0, 1.0, 16, 8)
    mesh = meshsdf.MeshData(V, F)
    rng = np.random.default_rng(3)
    y = rng.uniform(-6, 6, (200, 3)) * np.array([1, 1, 0.4])
    d, _, kind, fid, _ = meshsdf.closest(mesh, y)
    h = 1e-6
    checked = 0
    for k in range(len(y)):
        # skip points near a change of closest feature (the Hessian jumps)
        probes = y[k] + h * np.vstack([np.eye(3), -np.eye(3)])
        _, _, kp, fp, _ = meshsdf.closest(mesh, probes)
        if not ((kp == kind[k]) & (fp == fid[k])).all():
            continue
        phi, g, H = meshsdf.sdf_local(mesh, y[k:k + 1])
        pp = meshsdf.sdf_local(mesh, probes)
        fd_g = (pp[0][:3] - pp[0][3:]) / (2 * h)
        fd_H = (pp[1][:3] - pp[1][3:]) / (2 * h)
        assert np.abs(fd_g - g[0]).max() < 1e-6
        assert np.abs(fd_H - H[0]).max() < 1e-4 * max(1.0, np.abs(H[0]).max())
        assert abs(np.linalg.norm(g[0]) - 1) < 1e-12
        checked += 1
    assert checked > 150
    assert set(kind.tolist()) >= {meshsdf.FACE, meshsdf.EDGE, meshsdf.VERTEX}


def test_step_with_box_mesh_equals_analytic_box():
    """A pad step pressed by a cube given as 12 triangles equals the step
    pressed by the analytic box at the same pose."""
    pad = scenes.box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2)
    op_a = stepper.make_pad(pad.X, pad.tets, 0.3e6, 0.45, 1000.0)
    op_m = stepper.make_pad(pad.X, pad.tets, 0.3e6, 0.45, 1000.0)
    a = 3 * MM
    prm = stepper.StepParams(newton_tol=1e-10)
    R = scenes._rot_z(0.3) @ scenes._rot_x(0.05)       # face down, slightly tilted
    low = a * (np.cos(0.05) + np.sin(0.05))
    c = np.array([9 * MM, 7 * MM, 4 * MM + low + prm.dhat])
    for s in range(1, 4):
        cc = c - np.array([0, 0, 0.15 * MM * s])
        box = scenes.Indenter(contact.BOX, (a, a, a, 0.0), R, cc)
        msh = scenes.Indenter(contact.MESH, (0.0, 0.0, 0.0, 0.0), R, cc, meshes.box_surface(a, a, a))
        ra = stepper.step(op_a, [box], prm)
        rm = stepper.step(op_m, [msh], prm)
        stepper.commit(op_a, ra)
        stepper.commit(op_m, rm)
        assert ra.newton_iters == rm.newton_iters
        assert np.abs(ra.x - rm.x).max() <= 1e-12 * np.abs(ra.x - pad.X).max()
    assert np.abs(op_m.x - pad.X).max() > 0.1 * MM


# ---------------------------------------------------------------- pair barrier

class _Ind:
    def __init__(self, mesh, R=None, c=None):
        self.shape, self.prm, self.mesh = contact.MESH, (0.0,), mesh
        self.R = np.eye(3) if R is None else R
        self.c = np.zeros(3) if c is None else c


def test_pair_barrier_closed_forms_on_a_split_face():
    """Above a box face made of two triangles (split along a diagonal): a
    point over the diagonal is at height h from both triangles, a point off
    it is at h from its own triangle and at sqrt(h^2 + delta^2) from the
    diagonal edge of the other.  The pair barrier is the sum of the two
    barriers; the distance barrier takes the nearer only."""
    dhat, kappa, area = 0.3, 2.0, np.array([0.7])
    V, F = meshes.box_surface(5.0, 5.0, 5.0)
    ind = _Ind((V, F))
    top = F[np.all(V[F][:, :, 2] > 4.9, axis=1)]
    assert len(top) == 2
    shared = sorted(set(top[0]) & set(top[1]))
    p0, p1 = V[shared[0]], V[shared[1]]
    e = (p1 - p0) / np.linalg.norm(p1 - p0)
    m = np.cross(e, [0, 0, 1.0])                       # in-plane normal of the diagonal
    B = lambda s: kappa * area[0] * dhat * contact.barrier(np.array([s]))[0]
    for h, delta in [(0.1, 0.0), (0.05, 0.2), (0.2, 0.25), (0.1, 0.4)]:
        y = 0.5 * (p0 + p1) + 0.3 * e + delta * m + np.array([0, 0, h])
        Ep, _, _ = contact.barrier_terms([ind], y[None], area, dhat, kappa, mesh_pairs=True)
        Ed, _, _ = contact.barrier_terms([ind], y[None], area, dhat, kappa)
        other = np.hypot(h, delta)
        want = B(h / dhat) + (B(other / dhat) if other < dhat else 0.0)
        assert Ep == pytest.approx(want, rel=1e-12), (h, delta)
        assert Ed == pytest.approx(B(h / dhat), rel=1e-12)


def test_pair_barrier_derivatives_fd():
    """Gradient and (unprojected) Hessian of the pair barrier against central
    differences of the energy and of the gradient, near a rotated, shifted
    torus mesh (faces, edges and vertices all in reach)."""
    V, F = meshes.torus_surface(4.0, 1.5, 16, 8, phase=0.5)
    R = scenes._rot_z(0.4) @ scenes._rot_x(0.3)
    c = np.array([0.3, -0.2, 0.1])
    ind = _Ind((V, F), R, c)
    dhat, kappa = 0.6, 3.0
    rng = np.random.default_rng(5)
    # points just outside the tube: along outward normals of random surface points
    t = rng.integers(len(F), size=60)
    w = rng.dirichlet(np.ones(3), size=60)
    P = np.einsum("kj,kji->ki", w, V[F[t]])
    fn = np.cross(V[F[t, 1]] - V[F[t, 0]], V[F[t, 2]] - V[F[t, 0]])
    fn /= np.linalg.norm(fn, axis=1)[:, None]
    y = P + rng.uniform(0.05, 0.5, (60, 1)) * fn
    x = y @ R.T + c
    area = rng.uniform(0.5, 1.5, 60)
    E0, g, H = contact.barrier_terms([ind], x, area, dhat, kappa, project=False, mesh_pairs=True)
    assert E0 > 0 and np.abs(g).max() > 0
    h = 1e-6
    for k in range(60):
        for i in range(3):
            dx = np.zeros((60, 3))
            dx[k, i] = h
            Ep, gp, _ = contact.barrier_terms([ind], x + dx, area, dhat, kappa, mesh_pairs=True)
            Em, gm, _ = contact.barrier_terms([ind], x - dx, area, dhat, kappa, mesh_pairs=True)
            assert (Ep - Em) / (2 * h) == pytest.approx(g[k, i], rel=1e-5, abs=1e-7 * np.abs(g).max())
            assert np.abs((gp[k] - gm[k]) / (2 * h) - H[k, :, i]).max() <= 1e-4 * np.abs(H[k]).max() + 1e-6


def test_pair_barrier_smooth_across_a_concave_edge():
    """On the torus's inner side the ring-direction edges are concave.  On
    the bisector plane of such an edge the distance to the mesh switches
    between the two faces, so the distance barrier's gradient jumps across
    the plane; the pair barrier's gradient is continuous there."""
    V, F = meshes.torus_surface(4.0, 1.5, 16, 8, phase=0.5)
    mesh = meshsdf.MeshData(V, F)
    ind = _Ind((V, F))
    dhat, kappa, area = 0.5, 1.0, np.array([1.0])
    # a concave edge: shared by two triangles whose normals turn towards each
    # other (the far vertex of one lies on the outer side of the other's plane)
    found = None
    for t1 in range(len(F)):
        for t2 in range(t1 + 1, len(F)):
            sh = set(F[t1]) & set(F[t2])
            if len(sh) != 2:
                continue
            far = (set(F[t2]) - sh).pop()
            side = mesh.fn[t1] @ (V[far] - V[F[t1, 0]])
            angle = np.arccos(np.clip(mesh.fn[t1] @ mesh.fn[t2], -1, 1))
            if side > 1e-9 and angle > 0.2:
                found = (t1, t2, sorted(sh))
                break
        if found:
            break
    assert found is not None
    t1, t2, (a, b) = found
    nA, nB = mesh.fn[t1], mesh.fn[t2]
    mid = 0.5 * (V[a] + V[b])
    bis = (nA + nB) / np.linalg.norm(nA + nB)
    across = (nA - nB) / np.linalg.norm(nA - nB)
    y0 = mid + 0.1 * bis
    eps = 1e-7
    gd = [contact.barrier_terms([ind], (y0 + s * eps * across)[None], area, dhat, kappa)[1][0] for s in (-1, 1)]
    gp = [contact.barrier_terms([ind], (y0 + s * eps * across)[None], area, dhat, kappa, mesh_pairs=True)[1][0]
          for s in (-1, 1)]
    scale = np.linalg.norm(gd[0])
    assert np.linalg.norm(gd[1] - gd[0]) > 0.1 * scale          # the kink
    assert np.linalg.norm(gp[1] - gp[0]) < 1e-4 * scale         # smooth


def test_pair_friction_lag_closed_forms():
    """The friction lag under the pair barrier is the summed pair force:
    over a split face's diagonal both triangles push along the face normal,
    so lambda doubles and n stays the normal; over one triangle's interior,
    away from the others, it equals the distance barrier's lag."""
    from oracle import friction
    dhat, kappa = 0.3, 2.0
    V, F = meshes.box_surface(5.0, 5.0, 5.0)
    ind = _Ind((V, F))
    top = F[np.all(V[F][:, :, 2] > 4.9, axis=1)]
    a, b = sorted(set(top[0]) & set(top[1]))
    mid = 0.5 * (V[a] + V[b])
    e = (V[b] - V[a]) / np.linalg.norm(V[b] - V[a])
    m = np.cross(e, [0, 0, 1.0])
    x = np.array([mid + np.array([0, 0, 0.1]), mid + 0.5 * m + np.array([0, 0, 0.1])])
    area = np.array([0.7, 0.9])
    l0, n0, _ = friction.lag([ind], [ind], x, area, dhat, kappa)
    l1, n1, _ = friction.lag([ind], [ind], x, area, dhat, kappa, mesh_pairs=True)
    assert l1[0, 0] == pytest.approx(2 * l0[0, 0], rel=1e-12) and l0[0, 0] > 0
    assert np.allclose(n1[0, 0], [0, 0, 1], atol=1e-12) and np.allclose(n0[0, 0], [0, 0, 1], atol=1e-12)
    assert l1[0, 1] == pytest.approx(l0[0, 1], rel=1e-12) and np.allclose(n1[0, 1], n0[0, 1], atol=1e-12)
