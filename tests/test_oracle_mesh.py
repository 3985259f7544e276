"""Pins of the oracle's surface extraction and per-vertex setup (Alg. 1's
surface extraction, contact-surface band rule) against exact integer counts
and geometric identities."""
import json
import os

import numpy as np
import pytest

from oracle import fem, surface
from workloads import meshes, scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_numbers.json")


def test_paper_mesh_counts_satisfy_closed_surface_relation():
    # Sec. IV-A prints 358 surface vertices and 712 surface triangles for the
    # refined GelSight Mini pad: a closed genus-0 triangulation has F = 2V - 4
    # (Euler V - E + F = 2 with 3F = 2E).  Our extractor must obey the same law.
    g = json.load(open(GOLDEN))["gelsight_mini_mesh"]
    assert g["surface_tris"] == 2 * g["surface_verts"] - 4
    assert round(g["tets_refined"] / g["tets_baseline"], 2) == g["tet_increase_factor"]


@pytest.mark.parametrize("n", [(12, 9, 3), (5, 4, 2), (1, 1, 1), (7, 3, 5)])
def test_structured_counts(n):
    nx, ny, nz = n
    pad = scenes.box_pad(0.018, 0.014, 0.004, nx, ny, nz)
    assert pad.tets.shape[0] == 6 * nx * ny * nz
    assert pad.X.shape[0] == (nx + 1) * (ny + 1) * (nz + 1)
    tris, parent = surface.surface_triangles(pad.tets)
    S = tris.shape[0]
    assert S == 4 * (nx * ny + nx * nz + ny * nz)
    Vs = np.unique(tris).size
    assert Vs == pad.X.shape[0] - (nx - 1) * (ny - 1) * (nz - 1)
    assert S == 2 * Vs - 4
    top = surface.contact_face_labels(pad.X, tris)
    if nz >= 2:
        assert top.sum() == 2 * nx * ny
    # ascending (parent, local face) order, parent owns the face
    assert np.all(np.diff(parent) >= 0)
    for j in range(0, S, max(1, S // 50)):
        assert set(tris[j]) <= set(pad.tets[parent[j]])


def test_config_sizes():
    e1 = scenes.config1()
    assert e1.pad.tets.shape[0] == 1944 and e1.pad.X.shape[0] == 520
    tris, _ = surface.surface_triangles(e1.pad.tets)
    assert tris.shape[0] == 684
    assert surface.contact_face_labels(e1.pad.X, tris).sum() == 216
    assert np.unique(tris).size == 344
    fixed = surface.default_fixed(e1.pad.X)
    cand = surface.candidates(tris, fixed, 520)
    assert (fixed == 7).sum() == 13 * 10               # the base
    assert cand.size == 344 - 13 * 10                  # every other surface vertex
    top_v = np.unique(tris[surface.contact_face_labels(e1.pad.X, tris).astype(bool)])
    assert np.isin(top_v, cand).all() and top_v.size == 13 * 10
    p2 = scenes.config2_pad()
    assert p2.tets.shape[0] == 122850 and p2.X.shape[0] == 23184
    zs = np.unique(p2.X[:, 2])
    assert np.isclose(zs[-1] - zs[-2], 0.2e-3, rtol=1e-9)


def test_surface_closed_and_consistently_oriented():
    for pad in (scenes.box_pad(0.018, 0.014, 0.004, 6, 5, 3),
                scenes.dome_pad(0.019, 0.016, 0.003, 7, 6, 3)):
        tris, _ = surface.surface_triangles(pad.tets)
        e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
        fwd = {tuple(r) for r in e}
        assert len(fwd) == e.shape[0]                  # no directed edge twice
        assert all((b, a) in fwd for a, b in fwd)      # each edge once per direction
        # divergence theorem: (1/6) sum X0 . (X1 x X2) = total tet volume
        X = pad.X
        vol_s = np.einsum("ij,ij->i", X[tris[:, 0]], np.cross(X[tris[:, 1]], X[tris[:, 2]])).sum() / 6
        _, vol = fem.rest_data(X, pad.tets)
        assert np.isclose(vol_s, vol.sum(), rtol=1e-12)


def test_outward_normals_on_box():
    pad = scenes.box_pad(0.018, 0.014, 0.004, 6, 5, 3)
    tris, _ = surface.surface_triangles(pad.tets)
    n, area = surface.tri_normals_areas(pad.X, tris)
    cen = pad.X[tris].mean(axis=1)
    mid = pad.X.mean(axis=0)
    assert np.all(np.abs(np.abs(n).max(axis=1) - 1) < 1e-12)   # axis aligned
    assert np.all(np.einsum("ij,ij->i", n, cen - mid) > 0)
    assert np.isclose(area.sum(), 2 * (0.018 * 0.014 + 0.018 * 0.004 + 0.014 * 0.004), rtol=1e-12)


def test_volume_mass_and_areas():
    e = scenes.config1()
    X, T = e.pad.X, e.pad.tets
    _, vol = fem.rest_data(X, T)
    assert (vol > 0).all()
    assert np.isclose(vol.sum(), 0.018 * 0.014 * 0.004, rtol=1e-12)
    m = surface.lumped_mass(X, T, 1000.0)
    assert np.isclose(m.sum(), 1.008e-3, rtol=1e-12)
    tris, _ = surface.surface_triangles(T)
    allv = np.unique(tris)
    A = surface.vertex_areas(X, tris, allv)
    _, area = surface.tri_normals_areas(X, tris)
    assert np.isclose(A.sum(), area.sum(), rtol=1e-12)


def test_graded_and_dome_generators():
    zs = meshes.graded_axis_top(4e-3, 13, 0.2e-3)
    w = np.diff(zs)
    assert np.isclose(w[-1], 0.2e-3) and np.all(np.diff(w) < 0)
    r = w[:-1] / w[1:]
    assert np.allclose(r, r[0], rtol=1e-9) and 1.06 < r[0] < 1.08
    pad = scenes.dome_pad(0.019, 0.016, 0.003, 8, 6, 3)
    ztop = pad.X[:, 2].max()
    assert np.isclose(ztop, 3e-3 + 0.030 - np.sqrt(0.030 ** 2 - (0.0095 ** 2 + 0.008 ** 2)), rtol=1e-9)
    _, vol = fem.rest_data(pad.X, pad.tets)
    assert (vol > 0).all()
