"""Pins of the Alg. 2 contact-vertex normal and area (oracle/surface.py).

The normal at a contact vertex is the normalised sum of e1 x e2 over its
triangles, i.e. the area-weighted average of their unit normals; the area is
a third of their summed areas.  A vertex on the contact face takes its
incident contact-face triangles, a vertex of the side faces only all its
incident surface triangles.  The pins are closed forms that an unweighted
sum, a flipped winding, or the wrong set of triangles would fail."""
import numpy as np

from oracle import stepper, surface
from workloads import scenes

MM = 1e-3


def test_fan_of_unequal_triangles_closed_form():
    # vertex 0 shared by a triangle of area 2 facing +z and one of area 0.5
    # facing +x; the area-weighted normal is (0.5, 0, 2) / |.|, the
    # unweighted one would be (1, 0, 1) / sqrt(2)
    P = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 1, 0], [0, 0, 1]], float)
    tris = np.array([[0, 1, 2], [0, 3, 4]], np.int32)
    n = surface.vertex_normals(P, tris, np.array([0, 1, 3]))
    assert np.allclose(n[0], np.array([0.5, 0.0, 2.0]) / np.sqrt(4.25), rtol=0, atol=1e-15)
    assert np.allclose(n[1], [0, 0, 1], atol=1e-15)
    assert np.allclose(n[2], [1, 0, 0], atol=1e-15)
    A = surface.vertex_areas(P, tris, np.array([0, 1, 3]))
    assert np.allclose(A, [2.5 / 3, 2.0 / 3, 0.5 / 3], rtol=1e-15)


def test_fan_normal_is_invariant_under_splitting_a_triangle():
    # splitting the +z triangle into two halves keeps the area-weighted normal
    # (an unweighted average would tilt further towards +z)
    P = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]], float)
    one = np.array([[0, 1, 2], [0, 3, 4]], np.int32)
    two = np.array([[0, 1, 5], [0, 5, 2], [0, 3, 4]], np.int32)
    a = surface.vertex_normals(P, one, np.array([0]))
    b = surface.vertex_normals(P, two, np.array([0]))
    assert np.allclose(a, b, atol=1e-15)


def test_box_edge_vertex_normal_and_area_closed_form():
    # config-1 pad, uniform Kuhn grid hx = 1.5, hy = 14/9, hz = 4/3 mm.  A
    # vertex inside the top edge at x = 0 touches 1.5 quads of the top face
    # and 1.5 quads of the side face whatever the diagonals.  All its
    # incident triangles would give the normal (-hz, 0, hx) / |.| and the area
    # (hx hy + hy hz) / 2; as a contact-face vertex it takes the contact-face
    # triangles only: normal +z, area hx hy / 2.  A vertex inside the side
    # face (x = 0, one layer down) takes its six side triangles: normal -x,
    # area hy hz.
    ep = scenes.config1()
    X, T = ep.pad.X, ep.pad.tets
    hx, hy, hz = 18 / 12 * MM, 14 / 9 * MM, 4 / 3 * MM
    op = stepper.make_pad(X, T, 0.3e6, 0.45, 1000.0)
    inside_y = (X[:, 1] > 1e-9) & (X[:, 1] < 14 * MM - 1e-9)
    edge = np.nonzero((np.abs(X[:, 0]) < 1e-12) & (np.abs(X[:, 2] - 4 * MM) < 1e-12) & inside_y)[0]
    side = np.nonzero((np.abs(X[:, 0]) < 1e-12) & (np.abs(X[:, 2] - (4 * MM - hz)) < 1e-12) & inside_y)[0]
    assert edge.size == 8 and side.size == 8
    assert np.allclose(surface.vertex_normals(X, op.tris, edge), np.array([-hz, 0, hx]) / np.hypot(hx, hz),
                       atol=1e-14)
    assert np.allclose(surface.vertex_areas(X, op.tris, edge), 0.5 * (hx * hy + hy * hz), rtol=1e-13)
    for verts, n_ref, a_ref in ((edge, [0, 0, 1], 0.5 * hx * hy), (side, [-1, 0, 0], hy * hz)):
        n, A = surface.contact_vertex_geometry(X, op.tris, op.is_top, verts)
        assert np.allclose(n, n_ref, atol=1e-14)
        assert np.allclose(A, a_ref, rtol=1e-13)
        # the barrier weight of the pad is the same rest area
        k = np.searchsorted(op.cand, verts)
        assert np.array_equal(op.cand[k], verts)
        assert np.allclose(op.area[k], a_ref, rtol=1e-13)
    # interior vertices of the top face: the face normal, 6 half-quads
    top_in = np.nonzero((np.abs(X[:, 2] - 4 * MM) < 1e-12) & (X[:, 0] > 1e-9) & (X[:, 0] < 18 * MM - 1e-9)
                        & inside_y)[0]
    n, A = surface.contact_vertex_geometry(X, op.tris, op.is_top, top_in)
    assert np.allclose(n, [0, 0, 1], atol=1e-14)
    assert np.allclose(A, hx * hy, rtol=1e-13)


def test_contact_area_partitions_the_surface():
    # contact-face vertices share out exactly the contact face, side-only
    # vertices the rest of the free surface: with the base fixed, the
    # candidates' areas sum to the top plus the side faces less the third
    # of each side triangle that lies at a base or contact-face vertex
    ep = scenes.config1()
    op = stepper.make_pad(ep.pad.X, ep.pad.tets, 0.3e6, 0.45, 1000.0)
    on_top = surface.contact_vertex_tris(op.tris, op.is_top, op.cand, ep.pad.X.shape[0])
    assert np.isclose(op.area[on_top].sum(), 18 * 14 * MM ** 2, rtol=1e-12)
    # side faces: 2 (18 + 14) mm x 4 mm; a side triangle gives a third of its
    # area to each corner that is neither on the base nor on the top edge
    _, a = surface.tri_normals_areas(ep.pad.X, op.tris)
    z = ep.pad.X[op.tris, 2]
    side = op.is_top == 0
    side &= ~np.all(np.abs(z) < 1e-12, axis=1)            # not the base face
    mid = (np.abs(z) > 1e-12) & (np.abs(z - 4 * MM) > 1e-12)
    expect = (a[side, None] / 3.0 * mid[side]).sum()
    assert np.isclose(op.area[~on_top].sum(), expect, rtol=1e-12)


def test_dome_cap_normals_converge_to_the_sphere_normal():
    # the dome pad's top is a sphere of radius 30 mm centred below the pad;
    # on the regular triangulation the area-weighted vertex normal converges
    # to the sphere's normal at O(h^2)
    R = 30 * MM
    rmax = np.hypot(9.5 * MM, 8 * MM)
    c = np.array([9.5 * MM, 8 * MM, 3 * MM - np.sqrt(R ** 2 - rmax ** 2)])
    errs = []
    for n in (2, 4):
        pad = scenes.dome_pad(19 * MM, 16 * MM, 3 * MM, 8 * n, 6 * n, 3)
        X = pad.X
        tris, _ = surface.surface_triangles(pad.tets)
        top = surface.contact_face_labels(X, tris).astype(bool)
        vt = np.unique(tris[top])
        inner = vt[(X[vt, 0] > 1e-9) & (X[vt, 0] < 19 * MM - 1e-9) & (X[vt, 1] > 1e-9) & (X[vt, 1] < 16 * MM - 1e-9)]
        exact = (X[inner] - c) / R
        assert np.allclose(np.linalg.norm(X[inner] - c, axis=1), R, rtol=1e-12)
        nv = surface.vertex_normals(X, tris, inner)
        errs.append(np.linalg.norm(nv - exact, axis=1).max())
    assert errs[0] < 1e-3
    assert errs[1] < errs[0] / 3.0, errs


def test_closed_surface_vector_area_vanishes_and_areas_sum_to_the_box():
    ep = scenes.config1()
    tris, _ = surface.surface_triangles(ep.pad.tets)
    v0, v1, v2 = (ep.pad.X[tris[:, k]] for k in range(3))
    c = np.cross(v1 - v0, v2 - v0)
    assert np.abs(c.sum(axis=0)).max() < 1e-18
    allv = np.unique(tris)
    A = surface.vertex_areas(ep.pad.X, tris, allv)
    assert np.isclose(A.sum(), 2 * (18 * 14 + 18 * 4 + 14 * 4) * MM ** 2, rtol=1e-12)
