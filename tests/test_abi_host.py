"""Host-only checks of the C-ABI library: it loads, exports every entry point
declared in include/tacauchy.h, its surface extraction (Alg. 1 (surface extraction))
matches the oracle bit for bit, and argument validation returns the
documented error codes.  No GPU is touched."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import surface as osurf
from workloads import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tacauchy.h")


@pytest.fixture(scope="module")
def tc():
    import paper_2606_20426_amd as tc
    from paper_2606_20426_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2606_20426_amd import build
        build.build()
    tc.load()
    return tc


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tc_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(tc):
    lib = tc.load()
    names = header_functions()
    assert len(names) >= 35
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.tc_version().decode().startswith("tacauchy")
    assert tc._abi.status_name(-6) == "TC_E_NOT_CONVERGED"


def _oracle_surface(X, tets, fixed=None):
    tris, parent = osurf.surface_triangles(tets)
    top = osurf.contact_face_labels(X, tris)
    fixed = osurf.default_fixed(X) if fixed is None else fixed
    cand = osurf.candidates(tris, fixed, X.shape[0])
    return tris, parent, top, cand


@pytest.mark.parametrize("which", ["config1", "dome", "graded", "odd", "one_cube"])
def test_surface_bit_exact_vs_oracle(tc, which):
    fixed = None
    if which == "config1":
        p = scenes.config1().pad
    elif which == "dome":
        p = scenes.dome_pad(0.019, 0.016, 0.003, 9, 7, 4)
    elif which == "graded":
        from workloads import meshes
        p = scenes.box_pad(0.018, 0.014, 0.004, 9, 7, 6, zs=meshes.graded_axis_top(0.004, 6, 0.0002))
    elif which == "odd":
        p = scenes.box_pad(0.005, 0.007, 0.003, 5, 7, 3)
        rng = np.random.default_rng(0)
        fixed = rng.integers(0, 8, p.X.shape[0]).astype(np.uint8)
    else:
        p = scenes.one_cube_pad()
        fixed = np.where(p.X[:, 2] == 0, 7, 0).astype(np.uint8)
    got = tc.mesh_surface(p.X, p.tets, fixed)
    tris, parent, top, cand = _oracle_surface(p.X, p.tets, fixed)
    assert np.array_equal(got["tris"], tris)
    assert np.array_equal(got["parent"], parent)
    assert np.array_equal(got["is_top"], top)
    assert np.array_equal(got["candidates"], cand)


def test_config2_surface_bit_exact(tc):
    p = scenes.config2_pad()
    got = tc.mesh_surface(p.X, p.tets)
    tris, parent, top, cand = _oracle_surface(p.X, p.tets)
    assert got["tris"].shape[0] == 10460 and int(top.sum()) == 3150
    assert np.array_equal(got["tris"], tris) and np.array_equal(got["parent"], parent)
    assert np.array_equal(got["is_top"], top) and np.array_equal(got["candidates"], cand)


def _status(fn):
    from paper_2606_20426_amd import TcError
    try:
        fn()
    except TcError as e:
        return e.status
    return 0


def test_validation_error_codes(tc):
    p = scenes.one_cube_pad()
    X, T = p.X.copy(), p.tets.copy()
    V = tc.validate
    assert _status(lambda: V(mesh=(X, T))) == 0
    bad = T.copy(); bad[0, 1] = 99
    assert _status(lambda: V(mesh=(X, bad))) == -2               # index out of range
    inv = T.copy(); inv[0, [2, 3]] = inv[0, [3, 2]]
    assert _status(lambda: V(mesh=(X, inv))) == -2               # negative volume
    rep = T.copy(); rep[0, 1] = rep[0, 0]
    assert _status(lambda: V(mesh=(X, rep))) == -2               # repeated vertex
    Xn = X.copy(); Xn[3, 1] = np.nan
    assert _status(lambda: V(mesh=(Xn, T))) == -1
    assert _status(lambda: V(mesh=(X, T, np.full(8, 9, np.uint8)))) == -1
    ok = dict(E=3e5, nu=0.45, density=1000.0)
    assert _status(lambda: V(materials=ok)) == 0
    for badm in (dict(ok, E=0.0), dict(ok, E=-1.0), dict(ok, nu=0.5), dict(ok, nu=-1.0),
                 dict(ok, density=0.0), dict(ok, E=float("nan"))):
        assert _status(lambda: V(materials=badm)) == -1
    assert _status(lambda: V(params=tc.make_params())) == 0
    for kw in (dict(dt=0.0), dict(dhat=-1.0), dict(kappa=float("inf")), dict(max_newton=0),
               dict(precision=7), dict(precond=3), dict(cg_rel_tol=0.0), dict(friction=-0.5),
               dict(friction=float("nan")), dict(friction=0.5, eps_v=0.0), dict(ls_expand=17),
               dict(mesh_contact=3), dict(mesh_contact=-1),
               dict(hess_proj=3), dict(cg_forcing=3), dict(cg_eta_max=1.0)):
        assert _status(lambda: V(params=tc.make_params(**kw))) == -1
    # friction off: the threshold is not used
    assert _status(lambda: V(params=tc.make_params(friction=0.0, eps_v=0.0))) == 0
    assert _status(lambda: V(params=tc.make_params(friction=0.5, eps_v=0.01))) == 0
    assert _status(lambda: V(params=tc.make_params(mesh_contact=1))) == 0
    assert _status(lambda: V(params=tc.make_params(mesh_contact=2))) == 0
    assert _status(lambda: V(params=tc.make_params(mesh_contact=1, friction=0.5))) == 0
    d = tc.make_params()
    assert d.friction == 0.0 and d.eps_v == 0.01
    I = np.eye(3)
    good = dict(shape=0, prm=(1e-3,), R=I, c=(0, 0, 0))
    assert _status(lambda: V(indenters=[good])) == 0
    assert _status(lambda: V(indenters=[good] * 6)) == -1
    assert _status(lambda: V(indenters=[dict(good, shape=9)])) == -1
    assert _status(lambda: V(indenters=[dict(good, prm=(0.0,))])) == -1
    assert _status(lambda: V(indenters=[dict(good, R=2 * I)])) == -1
    assert _status(lambda: V(indenters=[dict(good, R=np.diag([1.0, 1.0, -1.0]))])) == -1
    assert _status(lambda: V(indenters=[dict(good, shape=2, prm=(1e-3, 1e-3, 0.0))])) == -1


def test_rigid_mesh_validation(tc):
    from workloads import meshes
    V = tc.validate
    for good in (meshes.box_surface(1e-3, 2e-3, 3e-3), meshes.icosphere(2e-3, 2),
                 meshes.torus_surface(4e-3, 1e-3, 16, 8), meshes.cylinder_surface(2.5e-3, 5e-3, 32)):
        assert _status(lambda: V(rigid_mesh=good)) == 0
    Vb, Fb = meshes.box_surface(1e-3, 1e-3, 1e-3)
    assert _status(lambda: V(rigid_mesh=(Vb, Fb[:, ::-1]))) == -1        # inward normals
    assert _status(lambda: V(rigid_mesh=(Vb, Fb[:-1]))) == -1            # open surface
    flip = Fb.copy(); flip[0] = flip[0, ::-1]
    assert _status(lambda: V(rigid_mesh=(Vb, flip))) == -1               # inconsistent orientation
    bad = Fb.copy(); bad[0, 0] = 99
    assert _status(lambda: V(rigid_mesh=(Vb, bad))) == -1                # index out of range
    dup = Fb.copy(); dup[0, 1] = dup[0, 0]
    assert _status(lambda: V(rigid_mesh=(Vb, dup))) == -1                # repeated vertex
    flat = Vb.copy(); flat[:, 2] = 0.0
    assert _status(lambda: V(rigid_mesh=(flat, Fb))) == -1               # degenerate triangles
    nan = Vb.copy(); nan[3, 0] = np.nan
    assert _status(lambda: V(rigid_mesh=(nan, Fb))) == -1
    # mesh indenters: id range and finite (unused) parameters
    I = np.eye(3)
    m = dict(shape=tc.MESH, prm=(0.0,), R=I, c=(0, 0, 0), mesh_id=0)
    assert _status(lambda: V(indenters=[m])) == 0
    assert _status(lambda: V(indenters=[dict(m, mesh_id=64)])) == -1
    assert _status(lambda: V(indenters=[dict(m, mesh_id=-1)])) == -1
    assert _status(lambda: V(indenters=[dict(m, prm=(np.inf,))])) == -1


def test_context_without_device_fails_loudly(tc):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(tc.TcError) as e:
        tc.Context(0)
    assert e.value.status == -8


@pytest.mark.parametrize("case", ["box", "config1_fine", "dome_offset", "side_minus_layers"])
def test_refine_mesh_bit_exact_vs_oracle(tc, case):
    """Library refinement (host C++) equals the oracle's: integers and
    positions bit for bit."""
    from oracle import refine
    MM = 1e-3
    mat = None
    kw = {}
    if case == "box":
        pad = scenes.box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2)
    elif case == "config1_fine":
        pad = scenes.config1().pad
        kw = dict(l_contact=0.5 * MM, l_global=2.0 * MM)
    elif case == "dome_offset":
        pad = scenes.dome_pad(19 * MM, 16 * MM, 3 * MM, 6, 5, 2)
        kw = dict(centre=(7 * MM, 9 * MM), inner=0.3, transition=0.3)
    else:
        pad = scenes.box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2)
        mat, _ = scenes.layered_materials(pad.X, pad.tets, 2 * MM, None, None)
        kw = dict(side=-1, band=0.3)
    s = refine.Sizing(pad.X, **kw)
    Xo, To, Mo = refine.refine(pad.X, pad.tets, s, mat=mat)
    Xl, Tl, Ml = tc.refine_mesh(pad.X, pad.tets, tet_material=mat, **kw)
    assert Tl.shape == To.shape and Xl.shape == Xo.shape
    assert np.array_equal(Tl, To) and np.array_equal(Ml, Mo)
    assert np.array_equal(Xl.view(np.int64), Xo.view(np.int64))
    assert To.shape[0] > pad.tets.shape[0]


def test_refine_mesh_errors(tc):
    p = scenes.one_cube_pad()
    with pytest.raises(tc.TcError):
        tc.refine_mesh(p.X, p.tets, l_contact=0.0)
    with pytest.raises(tc.TcError):
        tc.refine_mesh(p.X, p.tets, side=0)
    with pytest.raises(tc.TcError):                  # growth beyond max_tets
        tc.refine_mesh(p.X, p.tets, l_contact=1e-5, l_global=1e-5, max_tets=100)
    bad = p.tets.copy(); bad[0, [2, 3]] = bad[0, [3, 2]]
    with pytest.raises(tc.TcError):
        tc.refine_mesh(p.X, bad)


def test_batch_variants_keep_the_batch():
    """The NEXT-row variants of the 60-pad batch keep its pads, materials
    and start poses and change only their own feature; the mesh variant's
    surfaces lie inside their analytic shapes (the start stays feasible)."""
    from oracle import contact
    from workloads import scenes
    base = scenes.config3(8)
    for kind in scenes.VARIANTS:
        envs = scenes.config3_variant(kind, 8)
        for b, e in zip(base, envs):
            assert e.pad is b.pad or np.array_equal(e.pad.X, b.pad.X)
            assert e.depth == b.depth and np.array_equal(e.indenter.c, b.indenter.c)
            if kind in ("slide", "friction"):
                assert e.friction == (0.5 if kind == "friction" else 0.0) and e.n_steps == 15
                step = np.linalg.norm(e.pose(17).c - e.pose(16).c)
                assert np.isclose(step, 0.1e-3)
                assert np.array_equal(e.pose(15).c, b.indenter.at_depth(b.depth).c)
            elif kind == "layers":
                idx, mats = e.layers
                assert set(np.unique(idx)) == {0, 1} and mats[0] == b.pad.material
                assert mats[1].E == 8 * mats[0].E
            else:
                if b.indenter.shape == scenes.TEXTURE:
                    assert e.indenter.shape == scenes.TEXTURE and e.indenter.mesh is None
                    continue
                assert e.indenter.shape == scenes.MESH
                if kind == "mesh2":
                    assert e.mesh_contact == 2
                else:
                    assert e.mesh_contact == (1 if b.indenter.shape == scenes.TORUS else 0)
                V, F = e.indenter.mesh
                assert _status(lambda: __import__("paper_2606_20426_amd").validate(rigid_mesh=(V, F))) == 0
                # every mesh vertex on or inside the analytic surface
                phi, _, _ = contact.sdf_local(b.indenter.shape, b.indenter.prm, V)
                assert phi.max() <= 1e-12 * np.abs(V).max()
