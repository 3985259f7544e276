"""Pins of the oracle's rigid-mesh vertex/pad-triangle and edge/edge pairs
(oracle/mesh_pairs.py): closest points against dense sampling, closed forms,
central differences of the energy, the mollifier's continuity, the third law
(the indenter's reaction is minus the pad forces) and the step bound."""
import numpy as np
import pytest

from oracle import contact, mesh_pairs as mp
from workloads import meshes, scenes

MM = 1e-3


def test_closest_on_triangles_against_sampling():
    rng = np.random.default_rng(0)
    N = 300
    a, b, c = (rng.normal(size=(N, 3)) for _ in range(3))
    y = rng.normal(size=(N, 3)) * 1.5
    d, lam = mp.closest_on_triangles(y, a, b, c)
    assert np.allclose(lam.sum(axis=1), 1.0) and (lam >= -1e-12).all()
    q = lam[:, :1] * a + lam[:, 1:2] * b + lam[:, 2:] * c
    assert np.allclose(np.linalg.norm(y - q, axis=1), d, rtol=1e-12, atol=1e-14)
    u, v = rng.random((2, 40000))
    flip = u + v > 1
    u, v = np.where(flip, 1 - u, u), np.where(flip, 1 - v, v)
    for k in range(0, N, 7):
        P = a[k] + u[:, None] * (b[k] - a[k]) + v[:, None] * (c[k] - a[k])
        dmin = np.linalg.norm(P - y[k], axis=1).min()
        size = max(np.linalg.norm(b[k] - a[k]), np.linalg.norm(c[k] - a[k]), np.linalg.norm(c[k] - b[k]))
        assert d[k] <= dmin + 1e-12 and dmin - d[k] < 0.02 * size


def test_closest_on_segments_against_sampling_and_parallel_case():
    rng = np.random.default_rng(1)
    N = 300
    p0, p1, q0, q1 = (rng.normal(size=(N, 3)) for _ in range(4))
    d, s, t = mp.closest_on_segments(p0, p1, q0, q1)
    assert ((s >= 0) & (s <= 1) & (t >= 0) & (t <= 1)).all()
    P = p0 + s[:, None] * (p1 - p0)
    Q = q0 + t[:, None] * (q1 - q0)
    assert np.allclose(np.linalg.norm(P - Q, axis=1), d, rtol=1e-12)
    g = np.linspace(0, 1, 801)
    for k in range(0, N, 11):
        A = p0[k] + g[:, None] * (p1[k] - p0[k])
        B = q0[k] + g[:, None] * (q1[k] - q0[k])
        dmin = np.sqrt(((A[:, None, :] - B[None, :, :]) ** 2).sum(-1)).min()
        assert d[k] <= dmin + 1e-12 and dmin - d[k] < 1e-2
    # parallel, overlapping segments one unit apart: distance 1
    d, s, t = mp.closest_on_segments(np.array([[0, 0, 0.]]), np.array([[2, 0, 0.]]),
                                     np.array([[1, 1, 0.]]), np.array([[3, 1, 0.]]))
    assert np.isclose(d[0], 1.0)


class _Mesh:
    def __init__(self, V, F, c, R=np.eye(3)):
        self.shape, self.prm, self.mesh = contact.MESH, (0, 0, 0, 0), (V, F)
        self.R, self.c = R, np.asarray(c, float)


def _flat_pad(n=4, L=4 * MM):
    """A flat square of 2 n^2 triangles at z = 0 (counter-clockwise seen from
    +z) with its edges and rest edge lengths."""
    xs = np.linspace(0, L, n + 1)
    X = np.array([[x, y, 0.0] for y in xs for x in xs])
    tris = []
    for j in range(n):
        for i in range(n):
            v = i + (n + 1) * j
            tris += [[v, v + 1, v + n + 2], [v, v + n + 2, v + n + 1]]
    tris = np.array(tris, np.int64)
    edges = mp.surface_edges(tris)
    return X, tris, edges, np.linalg.norm(X[edges[:, 1]] - X[edges[:, 0]], axis=1)


def test_vertex_face_closed_form():
    # a tetrahedron's apex pointing down at height h over the centroid of a
    # pad triangle: one vertex-face pair, force split 1/3 per triangle vertex
    X, tris, edges, elen = _flat_pad(1, 2 * MM)
    t0 = X[tris[0]].mean(axis=0)
    h, dhat, kappa = 0.03 * MM, 0.1 * MM, 1e3
    V = np.array([[0, 0, 0], [1, 0, 3], [-1, 1, 3], [-1, -1, 3.]]) * MM
    F = np.array([[0, 2, 1], [0, 3, 2], [0, 1, 3], [1, 2, 3]])
    ind = _Mesh(V, F, t0 + np.array([0, 0, h]))
    E, g, _ = mp.pair_terms(ind, X, tris[:1], np.zeros((0, 2), np.int64), np.zeros(0), dhat, kappa)
    va, _ = mp.mesh_tables(V, F)
    s = h / dhat
    assert np.isclose(E, kappa * va[0] * dhat * contact.barrier(np.array([s]))[0], rtol=1e-12)
    fz = kappa * va[0] * contact.barrier_d1(np.array([s]))[0]       # dE/dh < 0
    for a in tris[0]:                                                  # raising a vertex lowers h by 1/3
        assert np.allclose(g[a], [0, 0, -fz / 3.0], rtol=1e-10, atol=1e-12 * abs(fz))


def test_edge_edge_closed_form_crossing():
    # a mesh edge along y crossing a pad edge along x at height h (the pad
    # edge's midpoint under the mesh edge's midpoint): d = h, weight |e||f|/4
    X = np.array([[0, 0, 0], [2, 0, 0.]]) * MM
    pedges = np.array([[0, 1]])
    plen = np.array([2 * MM])
    h, dhat, kappa = 0.04 * MM, 0.1 * MM, 1e3
    V = np.array([[1, -1, 0], [1, 1, 0], [1, 0, 5], [0, 0, 5]]) * MM     # a thin tetrahedron, edge 0-1 down
    F = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]])
    ind = _Mesh(V, F, [0, 0, h])
    _, medges = mp.mesh_tables(V, F)
    E, g, _ = mp.pair_terms(ind, X, np.zeros((0, 3), np.int64), pedges, plen, dhat, kappa)
    s = h / dhat
    w = kappa * 0.25 * 2 * MM * 2 * MM
    assert np.isclose(E, w * dhat * contact.barrier(np.array([s]))[0], rtol=1e-12)   # perpendicular: m = 1
    fz = w * contact.barrier_d1(np.array([s]))[0]                      # dE/dh < 0
    assert np.allclose(g[0], [0, 0, -fz / 2], rtol=1e-10, atol=1e-12 * abs(fz))
    assert np.allclose(g[1], [0, 0, -fz / 2], rtol=1e-10, atol=1e-12 * abs(fz))


def test_mollifier_is_c1_and_vanishes_parallel():
    c0 = 2.0
    c = np.array([0.0, 1.0, 2.0 - 1e-9, 2.0 + 1e-9, 3.0])
    m, dm = mp.mollifier(c, c0)
    assert m[0] == 0 and np.isclose(m[1], 0.75) and abs(m[2] - 1) < 1e-9 and m[3] == 1 and m[4] == 1
    assert abs(dm[2]) < 1e-8 and dm[3] == 0
    eps = 1e-6
    for x in (0.3, 1.1, 1.7):
        assert np.isclose((mp.mollifier(x + eps, c0)[0] - mp.mollifier(x - eps, c0)[0]) / (2 * eps),
                          mp.mollifier(x, c0)[1], rtol=1e-6)


def _scene(seed):
    X, tris, edges, elen = _flat_pad(4)
    rng = np.random.default_rng(seed)
    X = X + rng.normal(scale=0.03 * MM, size=X.shape) * np.array([1, 1, 0.5])
    V, F = meshes.icosphere(1.2 * MM, 1)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    R = q * np.sign(np.linalg.det(q))
    Vw = V @ R.T
    c = np.array([2.0 * MM, 2.0 * MM, 0.0]) - np.array([0, 0, Vw[:, 2].min()]) + np.array([0, 0, 0.04 * MM])
    return X, tris, edges, elen, _Mesh(V, F, c, R)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pair_energy_gradient_fd(seed):
    X, tris, edges, elen, ind = _scene(seed)
    dhat, kappa = 0.1 * MM, 1e3
    E, g, _ = mp.pair_terms(ind, X, tris, edges, elen, dhat, kappa)
    iv, *_ = mp.vf_pairs(mp._world(ind)[0], X, tris, dhat)
    ie, *_ = mp.ee_pairs(mp._world(ind)[0], mp.mesh_tables(*ind.mesh)[1], X, edges, dhat)
    assert E > 0 and len(iv) + len(ie) > 0
    rng = np.random.default_rng(10 + seed)
    h = 1e-9
    for _ in range(6):
        v = rng.normal(size=X.shape)
        Ep = mp.pair_terms(ind, X + h * v, tris, edges, elen, dhat, kappa)[0]
        Em = mp.pair_terms(ind, X - h * v, tris, edges, elen, dhat, kappa)[0]
        fd = (Ep - Em) / (2 * h)
        assert np.isclose(fd, np.sum(g * v), rtol=1e-5, atol=1e-6 * np.abs(g).sum() * 1e-3)


def test_third_law_reaction_on_the_indenter():
    # translating the indenter by dc changes E as -sum_a g_a . dc
    X, tris, edges, elen, ind = _scene(3)
    dhat, kappa = 0.1 * MM, 1e3
    _, g, _ = mp.pair_terms(ind, X, tris, edges, elen, dhat, kappa)
    h = 1e-9
    for k in range(3):
        dc = np.zeros(3)
        dc[k] = h
        ip = _Mesh(ind.mesh[0], ind.mesh[1], ind.c + dc, ind.R)
        im = _Mesh(ind.mesh[0], ind.mesh[1], ind.c - dc, ind.R)
        fd = (mp.pair_terms(ip, X, tris, edges, elen, dhat, kappa)[0]
              - mp.pair_terms(im, X, tris, edges, elen, dhat, kappa)[0]) / (2 * h)
        assert np.isclose(fd, -g[:, k].sum(), rtol=1e-5, atol=1e-12)


def test_gauss_newton_blocks_are_psd_and_rank_one_per_pair():
    X, tris, edges, elen, ind = _scene(4)
    _, _, (r, c, v) = mp.pair_terms(ind, X, tris, edges, elen, 0.1 * MM, 1e3)
    n = X.shape[0]
    H = np.zeros((3 * n, 3 * n))
    for i, j, b in zip(r, c, v):
        H[3 * i:3 * i + 3, 3 * j:3 * j + 3] += b
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(H).min() >= -1e-9 * np.abs(H).max()


def test_step_bound_keeps_pairs_apart():
    X, tris, edges, elen, ind = _scene(5)
    rng = np.random.default_rng(6)
    p = rng.normal(size=X.shape) * 0.1 * MM - np.array([0, 0, 0.3 * MM])    # towards the sphere? away
    p[:, 2] = np.abs(p[:, 2])                                                # up, into the indenter
    a = mp.step_bound(ind, X, p, tris, edges)
    assert 0 < a <= 1
    Yw, _ = mp._world(ind)
    _, medges = mp.mesh_tables(*ind.mesh)
    for f in np.linspace(0, 1, 11):
        Xa = X + f * a * p
        d0 = mp.vf_pairs(Yw, Xa, tris, np.inf)[2].min()
        d1 = mp.ee_pairs(Yw, medges, Xa, edges, np.inf)[2].min()
        assert min(d0, d1) > 0


def test_signed_pairs_find_a_tunnelled_corner():
    # a tetrahedron's apex 0.05 mm below a pad triangle's interior (through
    # the surface) is reported with its negative signed distance; 0.05 mm
    # above, nothing is
    X, tris, edges, elen = _flat_pad(1, 2 * MM)
    t0 = X[tris[0]].mean(axis=0)
    V = np.array([[0, 0, 0], [1, 0, 3], [-1, 1, 3], [-1, -1, 3.]]) * MM
    F = np.array([[0, 2, 1], [0, 3, 2], [0, 1, 3], [1, 2, 3]])
    below = mp.signed_pairs(_Mesh(V, F, t0 - [0, 0, 0.05 * MM]), X, tris, edges, 0.2 * MM)
    vf = [b for b in below if len(b[0]) == 3]
    assert len(vf) == 1 and np.isclose(vf[0][2], -0.05 * MM) and np.allclose(vf[0][1], [0, 0, 1])
    above = mp.signed_pairs(_Mesh(V, F, t0 + [0, 0, 0.05 * MM]), X, tris, edges, 0.2 * MM)
    assert not above


def test_corner_between_pad_vertices_needs_the_triangle_pairs():
    """A cube corner pressed into a coarse pad between its vertices: with
    pad-vertex pairs only (mesh_contact 1) it passes through the surface
    unseen (no force, the pad at rest, the corner behind a top triangle);
    with the vertex-face and edge-edge pairs (mesh_contact 2) the triangle
    under it is held outside, the pad deforms and the reaction grows."""
    ep = scenes.corner_press_episode()
    X = ep.pad.X
    from oracle import extract, stepper
    out = {}
    for mode in (1, 2):
        op = stepper.make_pad(X, ep.pad.tets, 0.3e6, 0.45, 1000.0)
        prm = stepper.StepParams(newton_tol=1e-10, mesh_pairs=mode)
        for s in (1, 2, 3):
            ind = ep.pose(s)
            res = stepper.step(op, [ind], prm, inds_prev=[ep.pose(s - 1)])
            stepper.commit(op, res)
        cf = extract.contact_forces(op, op.x, [ind], prm)
        tunnelled = [p for p in mp.signed_pairs(ind, op.x, op.tris, op.pedges, 1e-3) if p[2] < 0]
        out[mode] = (cf["reaction"], tunnelled, np.abs(op.x - X).max())
    r1, t1, m1 = out[1]
    r2, t2, m2 = out[2]
    assert np.abs(r1).max() == 0 and m1 < 1e-15 and t1            # through the surface, unseen
    assert min(p[2] for p in t1) < -0.15 * MM
    assert r2[2] > 0.5 and not t2 and m2 > 0.1 * MM              # held: force, deformation, no crossing


def test_step_bound_lets_tangential_motion_through():
    """A pad sliding sideways under a mesh vertex held just above a triangle:
    the separation along the pair direction does not change, so the bound
    allows the full step where the displacement bound 0.9 d / |p| would cut
    it to a fraction; every pair stays apart along the step."""
    X, tris, edges, elen = _flat_pad(2, 2 * MM)
    t0 = X[tris[3]].mean(axis=0)
    V = np.array([[0, 0, 0], [1, 0, 3], [-1, 1, 3], [-1, -1, 3.]]) * MM
    F = np.array([[0, 2, 1], [0, 3, 2], [0, 1, 3], [1, 2, 3]])
    h = 0.01 * MM
    ind = _Mesh(V, F, t0 + [0, 0, h])
    p = np.zeros_like(X)
    p[:, 0] = 0.2 * MM                               # sideways, 20 h
    a = mp.step_bound(ind, X, p, tris, edges)
    assert a == 1.0
    p[:, 2] = -0.5 * h                               # and half the gap away from the apex
    assert mp.step_bound(ind, X, p, tris, edges) == 1.0
    p[:, 2] = 2.0 * h                                # towards it: 0.9 h / 2 h
    a = mp.step_bound(ind, X, p, tris, edges)
    assert np.isclose(a, 0.45)
    Yw, _ = mp._world(ind)
    _, medges = mp.mesh_tables(*ind.mesh)
    for f in np.linspace(0, 1, 21):
        Xa = X + f * a * p
        d0 = mp.vf_pairs(Yw, Xa, tris, np.inf)[2].min()
        d1 = mp.ee_pairs(Yw, medges, Xa, edges, np.inf)[2].min()
        assert min(d0, d1) > 0


def test_step_bound_advances_past_a_tilt():
    """A pad triangle tilting about the point under a mesh vertex: its
    vertices rise and sink by far more than the gap, so both the
    displacement and the separation bounds stop the step at a small
    fraction, while conservative advancement along the actual distance goes
    on until the tilted triangle nears the vertex; every pair stays apart
    along the step."""
    X, tris, edges, elen = _flat_pad(2, 2 * MM)
    t = 3
    c = X[tris[t]].mean(axis=0)
    V = np.array([[0, 0, 0], [1, 0, 3], [-1, 1, 3], [-1, -1, 3.]]) * MM
    F = np.array([[0, 2, 1], [0, 3, 2], [0, 1, 3], [1, 2, 3]])
    h = 0.01 * MM
    ind = _Mesh(V, F, c + [0, 0, h])
    p = np.zeros_like(X)
    w = np.array([0.0, 20 * h / MM, 0.0])                 # rotation about y through the centroid
    p = np.cross(w[None], X - c[None])
    a = mp.step_bound(ind, X, p, tris, edges)
    Yw, _ = mp._world(ind)
    iv, it, d, lam, u = mp.vf_pairs(Yw, X, tris, np.inf)
    k = np.nonzero(it == t)[0][0]
    pu = (p[tris[t]] @ u[k]).max()
    sep_only = 0.9 * d[k] / pu
    assert a > 2 * sep_only, (a, sep_only)
    _, medges = mp.mesh_tables(*ind.mesh)
    for f in np.linspace(0, 1, 41):
        Xa = X + f * a * p
        assert mp.vf_pairs(Yw, Xa, tris, np.inf)[2].min() > 0
        assert mp.ee_pairs(Yw, medges, Xa, edges, np.inf)[2].min() > 0
