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
