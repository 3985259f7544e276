"""Pins of the oracle's adaptive refinement (Sec. III-A sizing field,
terminal-edge bisection)."""
import math

import numpy as np
import pytest

from oracle import refine
from workloads import meshes, scenes

MM = 1e-3


def _vol(X, T):
    a, b, c, d = (X[T[:, k]] for k in range(4))
    return np.einsum("ki,ki->k", b - a, np.cross(c - a, d - a)) / 6.0


def _faces(T):
    F = np.sort(np.concatenate([T[:, [1, 2, 3]], T[:, [0, 2, 3]], T[:, [0, 1, 3]], T[:, [0, 1, 2]]]), axis=1)
    u, cnt = np.unique(F, axis=0, return_counts=True)
    return u, cnt


def test_sizing_field_closed_forms():
    X = scenes.box_pad(24 * MM, 16 * MM, 5 * MM, 2, 2, 1).X
    s = refine.Sizing(X)
    assert s.k == 2 and (s.u, s.v) == (0, 1)
    top = 5 * MM
    assert s.h((12 * MM, 8 * MM, top)) == 0.8e-3                        # centre of the contact face
    assert s.h((12 * MM, 8 * MM, top - 0.76 * MM)) == 3.2e-3           # below the 15 % band
    assert s.h((12 * MM, 8 * MM, top - 0.74 * MM)) == 0.8e-3
    # mid-transition (rho = 0.5): half way between l_c and l_g
    assert math.isclose(s.h((12 * MM + 0.5 * 12 * MM, 8 * MM, top)), 2.0e-3, rel_tol=1e-12)
    # elliptical normalisation: the same rho along v
    assert math.isclose(s.h((12 * MM, 8 * MM + 0.5 * 8 * MM, top)), 2.0e-3, rel_tol=1e-12)
    assert s.h((0.0, 0.0, top)) == 3.2e-3
    s2 = refine.Sizing(X, side=-1)
    assert s2.h((12 * MM, 8 * MM, 0.0)) == 0.8e-3 and s2.h((12 * MM, 8 * MM, top)) == 3.2e-3


def test_single_cube_body_diagonal_closed_form():
    """Uniform h just below the cube side: only the body diagonal (length^2 3
    > 3 h^2) is too long; it is the longest edge of all six Kuhn tets, so one
    bisection gives 12 tets around the cube centre."""
    pad = scenes.one_cube_pad(1.0)
    s = refine.Sizing(pad.X, band=10.0, inner=10.0, transition=1.0, l_contact=0.999, l_global=0.999)
    X, T, M = refine.refine(pad.X, pad.tets, s)
    assert X.shape == (9, 3) and T.shape == (12, 4)
    assert np.array_equal(X[8], [0.5, 0.5, 0.5])
    v = _vol(X, T)
    assert (v > 0).all() and np.allclose(v, 1.0 / 12)


@pytest.fixture(scope="module")
def refined():
    pad = scenes.box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2)       # 3 x 2.8 x 2 mm cells
    s = refine.Sizing(pad.X, l_contact=0.8 * MM, l_global=3.2 * MM)
    X, T, M = refine.refine(pad.X, pad.tets, s)
    return pad, s, X, T, M


def test_refined_mesh_is_conforming_and_closed(refined):
    pad, s, X, T, M = refined
    assert T.shape[0] > 2 * pad.tets.shape[0]
    v = _vol(X, T)
    assert (v > 0).all()
    assert math.isclose(v.sum(), 18 * 14 * 4 * MM ** 3, rel_tol=1e-12)
    # every face shared by two tets, or on the boundary (one tet)
    F, cnt = _faces(T)
    assert set(cnt.tolist()) == {1, 2}
    B = F[cnt == 1]
    # boundary faces lie on the box planes, and the boundary is a closed
    # genus-0 surface: F = 2 V_b - 4
    Xb = X[B]
    on = [(np.abs(Xb[..., k] - lim) < 1e-15).all(axis=1) for k, lim in
          ((0, 0), (0, 18 * MM), (1, 0), (1, 14 * MM), (2, 0), (2, 4 * MM))]
    assert np.logical_or.reduce(on).all()
    assert len(B) == 2 * len(np.unique(B)) - 4
    # Euler characteristic of a tetrahedralised ball
    E = np.unique(np.sort(np.concatenate([T[:, [i, j]] for i, j in refine._PAIRS]), axis=1), axis=0)
    assert X.shape[0] - len(E) + len(F) - len(T) == 1
    # no vertex hangs in the middle of another edge (conformity)
    assert len(np.unique(T)) == X.shape[0]


def test_refined_mesh_meets_the_sizing_field(refined):
    pad, s, X, T, M = refined
    E = np.unique(np.sort(np.concatenate([T[:, [i, j]] for i, j in refine._PAIRS]), axis=1), axis=0)
    L2 = ((X[E[:, 0]] - X[E[:, 1]]) ** 2).sum(axis=1)
    h = np.array([s.h(0.5 * (X[a] + X[b])) for a, b in E])
    assert (L2 <= 3 * h * h).all()
    # the contact centre reaches the fine size, the far base keeps the coarse one
    centre = (np.abs(X[:, 0] - 9 * MM) < 2 * MM) & (np.abs(X[:, 1] - 7 * MM) < 2 * MM) & (X[:, 2] > 3.5 * MM)
    assert centre.sum() > 20
    base = (X[T].mean(axis=1)[:, 2] < 1.5 * MM)
    assert abs(_vol(X, T)[base]).max() > 0.5 * (3 * 2.8 * 2 * MM ** 3 / 6)


def test_bisection_keeps_shape_quality(refined):
    """Terminal-edge bisection of Kuhn tets stays in a few similarity
    classes: the ratio of longest to shortest edge never exceeds twice the
    input's."""
    pad, s, X, T, M = refined

    def ratio(Xa, Ta):
        L = np.stack([np.linalg.norm(Xa[Ta[:, i]] - Xa[Ta[:, j]], axis=1) for i, j in refine._PAIRS], 1)
        return (L.max(1) / L.min(1)).max()
    assert ratio(X, T) <= 2 * ratio(pad.X, pad.tets)


def test_materials_follow_parents():
    pad = scenes.box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2)
    idx, _ = scenes.layered_materials(pad.X, pad.tets, 2 * MM, None, None)
    s = refine.Sizing(pad.X)
    X, T, M = refine.refine(pad.X, pad.tets, s, mat=idx)
    zc = X[T].mean(axis=1)[:, 2]
    assert (M[zc > 2 * MM] == 0).all() and (M[zc < 2 * MM] == 1).all()
