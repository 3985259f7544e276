"""Seeded synthetic scenes: pads, materials, indenter poses, schedules.

The paper measures on its own sensor meshes (GelSight Mini, DIGIT, 9DTact)
which are not available; these scenes stand in with the shapes and sizes of
the five benchmark workloads:

  1. single 18x14x4 mm pad, 12x9x3 cells (1,944 tets), sphere r = 5 mm,
     0.5 mm over 10 steps, FP64;
  2. the same pad as a 45x35x13 graded grid (122,850 tets, top layer
     0.2 mm) with five indenters, 30 steps each;
  3. 60 uneven pads (flat 18x14x4, dome 19x16x3 + R30 cap, flat 24x24x5),
     20k-80k tets each, random material and indenter;
  4. 256 resident pads, 5k-150k tets log-uniform, Poisson step requests;
  5. one 24x24x5 mm pad, ~1.2M tets, four-level refinement around a
     seeded patch, sphere r = 3 mm, 1 mm over 60 steps.

Random draws use numpy's PCG64 seeded by SeedSequence.  Nothing here
evaluates the method: indenter start heights come from vertex heights only
(no signed distances).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from . import meshes

MM = 1e-3

SPHERE, CYLINDER, BOX, TORUS, TEXTURE, MESH = 0, 1, 2, 3, 4, 5
SHAPE_NAMES = {SPHERE: "sphere", CYLINDER: "cylinder", BOX: "cube_edge",
               TORUS: "torus", TEXTURE: "texture", MESH: "mesh"}


@dataclasses.dataclass
class Material:
    E: float = 0.3e6        # Young's modulus [Pa]
    nu: float = 0.45        # Poisson ratio
    density: float = 1000.0  # [kg/m^3]


@dataclasses.dataclass
class Params:
    dt: float = 1.0 / 60.0
    dhat: float = 0.1 * MM
    kappa: float = 1e3       # barrier stiffness [Pa]
    newton_tol: float = 1e-6  # ||p||_inf <= tol * bbox diagonal
    cg_rel_tol: float = 1e-4
    max_newton: int = 1024
    max_cg: int = 4000
    quasi_static: int = 0
    gravity: tuple = (0.0, 0.0, 0.0)
    literal_alpha: int = 0   # 1: rest shift alpha = 1 exactly as printed


@dataclasses.dataclass
class Indenter:
    shape: int
    prm: tuple               # shape parameters [m]
    R: np.ndarray            # 3x3 rotation, local -> world
    c: np.ndarray            # centre at the start of the episode [m]
    mesh: Optional[tuple] = None   # (V [n,3], F [m,3]) local frame, shape MESH only

    def at_depth(self, depth):
        """Pose after travelling `depth` metres along world -z."""
        return Indenter(self.shape, self.prm, self.R.copy(),
                        self.c - np.array([0.0, 0.0, depth]), self.mesh)


@dataclasses.dataclass
class Pad:
    name: str
    X: np.ndarray            # rest positions [V,3] float64
    tets: np.ndarray         # [T,4] int32
    material: Material
    dims: tuple              # (Lx, Ly, H) [m]
    fixed: Optional[np.ndarray] = None   # per-vertex xyz bitmask (uint8)


@dataclasses.dataclass
class Episode:
    pad: Pad
    indenter: Indenter       # start pose (barrier just inactive)
    depth: float             # total travel [m]
    n_steps: int             # steps to reach `depth`
    params: Params
    schedule: str = "press"  # "press": ramp then hold; "triangle": press/release
    slide: Optional[np.ndarray] = None   # world xy travel per step once the ramp is done [m]
    friction: float = 0.0                # friction ratio of the pad
    layers: Optional[tuple] = None       # (per-tet material index [T], [Material, ...])
    mesh_contact: int = 0                # rigid meshes: 1 = barrier summed over triangle pairs

    def depth_at(self, step):
        """Indenter travel after `step` steps (step >= 1)."""
        n = self.n_steps
        if self.schedule == "triangle":
            ph = step % (2 * n)
            frac = ph / n if ph <= n else (2 * n - ph) / n
        else:
            frac = min(step, n) / n
        return self.depth * frac

    def pose(self, step):
        ind = self.indenter.at_depth(self.depth_at(step))
        if self.slide is not None:
            k = max(step - self.n_steps, 0)
            ind.c = ind.c + np.array([self.slide[0] * k, self.slide[1] * k, 0.0])
        return ind


# ----------------------------------------------------------------------------
# pads

def box_pad(Lx, Ly, H, nx, ny, nz, material=None, name="box", zs=None):
    xs = meshes.uniform_axis(Lx, nx)
    ys = meshes.uniform_axis(Ly, ny)
    zs = meshes.uniform_axis(H, nz) if zs is None else zs
    X, T = meshes.kuhn_grid(xs, ys, zs)
    return Pad(name, X, T, material or Material(), (Lx, Ly, H))


def dome_pad(Lx, Ly, H, nx, ny, nz, cap_radius=30 * MM, material=None):
    pad = box_pad(Lx, Ly, H, nx, ny, nz, material, name="dome")
    pad.X = meshes.dome_map(pad.X, H, cap_radius, (0.5 * Lx, 0.5 * Ly))
    return pad


def one_tet_pad():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * MM
    return Pad("one_tet", X, np.array([[0, 1, 2, 3]], np.int32), Material(),
               (1 * MM, 1 * MM, 1 * MM))


def one_cube_pad(size=1 * MM):
    return box_pad(size, size, size, 1, 1, 1, name="one_cube")


SHAPES3 = (("flat18", 18 * MM, 14 * MM, 4 * MM, False),
           ("dome19", 19 * MM, 16 * MM, 3 * MM, True),
           ("flat24", 24 * MM, 24 * MM, 5 * MM, False))


def pad_for_target(shape_idx, target_tets, material):
    name, Lx, Ly, H, dome = SHAPES3[shape_idx]
    nx, ny, nz = meshes.cells_for_target(Lx, Ly, H, target_tets)
    if dome:
        pad = dome_pad(Lx, Ly, H, nx, ny, nz, material=material)
    else:
        pad = box_pad(Lx, Ly, H, nx, ny, nz, material, name=name)
    return pad


# ----------------------------------------------------------------------------
# indenters

def _rot_x(angle):
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], float)


def indenter_geometry(shape, rng=None, sphere_radius=None):
    """(prm, R, footprint radius, lowest-point offset below the centre)."""
    if shape == SPHERE:
        r = sphere_radius if sphere_radius is not None else rng.uniform(2, 8) * MM
        return (r, 0, 0, 0), np.eye(3), r, r
    if shape == CYLINDER:      # 5 mm diameter, 10 mm long, axis vertical
        r, a = 2.5 * MM, 5 * MM
        return (r, a, 0, 0), np.eye(3), r, a
    if shape == BOX:           # cube of half-size 3 mm, edge pointing down
        a = 3 * MM
        return (a, a, a, 0), _rot_x(math.pi / 4), a * math.sqrt(2), a * math.sqrt(2)
    if shape == TORUS:         # ring lying flat
        Rt, rt = 4 * MM, 1 * MM
        return (Rt, rt, 0, 0), np.eye(3), Rt + rt, rt
    if shape == TEXTURE:       # sinusoidal plate, amplitude 0.2 mm, period 2 mm
        A, lam = 0.2 * MM, 2 * MM
        return (A, lam, 0, 0), np.eye(3), np.inf, A
    raise ValueError(shape)


def place_indenter(pad, shape, xy, dhat, rng=None, sphere_radius=None):
    """Start pose: lowest point d_hat above the highest rest vertex under the
    indenter footprint (vertex heights only)."""
    prm, R, foot, low = indenter_geometry(shape, rng, sphere_radius)
    X = pad.X
    near = np.hypot(X[:, 0] - xy[0], X[:, 1] - xy[1]) <= foot + 10 * dhat
    ztop = X[near, 2].max() if near.any() else X[:, 2].max()
    c = np.array([xy[0], xy[1], ztop + dhat + low], float)
    return Indenter(shape, prm, R, c)


def seeded_xy(rng, pad, margin):
    Lx, Ly, _ = pad.dims
    mx = min(margin, 0.45 * Lx)
    my = min(margin, 0.45 * Ly)
    return rng.uniform(mx, Lx - mx), rng.uniform(my, Ly - my)


# ----------------------------------------------------------------------------
# the five workloads

def layered_materials(X, tets, z_split, top, bottom):
    """Per-tet material index of a two-layer pad (the dual-layer gel of
    Sec. IV-D): 0 above z_split (tet centroid), 1 below; returns (index,
    [top, bottom])."""
    zc = X[tets, 2].mean(axis=1)
    return np.where(zc > z_split, 0, 1).astype(np.int32), [top, bottom]


def dual_layer_episode():
    """18x14x4 mm pad, 12x9x4 cells: a soft 2 mm top layer (E = 0.15 MPa,
    nu = 0.47, rho = 1050) on a stiffer 2 mm base (E = 1.2 MPa, nu = 0.42,
    rho = 1200); sphere r = 4 mm pressed 0.6 mm over 8 steps (seed 7)."""
    pad = box_pad(18 * MM, 14 * MM, 4 * MM, 12, 9, 4, Material(0.15e6, 0.47, 1050.0), name="dual")
    idx, mats = layered_materials(pad.X, pad.tets, 2 * MM, Material(0.15e6, 0.47, 1050.0),
                                  Material(1.2e6, 0.42, 1200.0))
    params = Params()
    rng = np.random.default_rng(7)
    r = 4 * MM
    xy = (rng.uniform(r / 2, pad.dims[0] - r / 2), rng.uniform(r / 2, pad.dims[1] - r / 2))
    ind = place_indenter(pad, SPHERE, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, 0.6 * MM, 8, params), idx, mats


def curved_gel_episode(nx=14, ny=10, nz=3):
    """Stand-in for a curved sensor gel (the paper's DIGIT, Sec. IV-D; its
    CAD is not available): a 20x14 mm pad, 2.5 mm thick at its two curved
    edges, whose top is a cylindrical cap of radius 30 mm curved along x
    (1.7 mm higher at the ridge).  E = 0.3 MPa, nu = 0.45; sphere r = 5 mm at
    a seeded point (seed 11) pressed 0.5 mm over 8 steps."""
    Lx, Ly, H = 20 * MM, 14 * MM, 2.5 * MM
    pad = box_pad(Lx, Ly, H, nx, ny, nz, Material(0.3e6, 0.45, 1000.0), name="curved")
    pad.X = meshes.cylinder_map(pad.X, H, 30 * MM, 0.5 * Lx)
    params = Params()
    rng = np.random.default_rng(11)
    r = 5 * MM
    xy = (rng.uniform(0.35 * Lx, 0.65 * Lx), rng.uniform(r / 2, Ly - r / 2))
    ind = place_indenter(pad, SPHERE, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, 0.5 * MM, 8, params)


def stiff_skin_episode(nx=12, ny=12, nz=6):
    """Stand-in for a dual-layer gel whose surface layer is the stiffer one
    (the paper's 9DTact, Sec. IV-D: a soft translucent base under a stiffer
    black surface layer; its CAD and moduli are not given): a 20x20x4 mm
    pad, the top 0.67 mm (one cell layer) with E = 1.2 MPa, nu = 0.45,
    rho = 1100 over a base with E = 0.2 MPa, nu = 0.47, rho = 1050; sphere
    r = 4 mm at a seeded point (seed 12) pressed 0.6 mm over 8 steps.
    Returns (episode, per-tet material index, [skin, base])."""
    Lx, Ly, H = 20 * MM, 20 * MM, 4 * MM
    base = Material(0.2e6, 0.47, 1050.0)
    skin = Material(1.2e6, 0.45, 1100.0)
    pad = box_pad(Lx, Ly, H, nx, ny, nz, base, name="stiff_skin")
    idx, mats = layered_materials(pad.X, pad.tets, H - H / nz, skin, base)
    params = Params()
    rng = np.random.default_rng(12)
    r = 4 * MM
    xy = (rng.uniform(r / 2, Lx - r / 2), rng.uniform(r / 2, Ly - r / 2))
    ind = place_indenter(pad, SPHERE, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, 0.6 * MM, 8, params), idx, mats


def corner_press_episode(mesh_contact=2):
    """A sharp rigid feature between pad vertices: a 2 mm cube as a
    12-triangle mesh with one corner pointing straight down (body diagonal
    vertical) over the centroid of a top triangle of a coarse 18x14x4 mm pad
    (6x5x2 cells, vertices 3 mm apart), its tip d_hat above the surface at
    step 0, pressed 0.3 mm over 3 steps.  Every pad vertex stays more than
    1.5 mm from the corner's axis, where the cube's faces rise about 2 mm, so
    only the corner-against-triangle pair sees the contact."""
    pad = box_pad(18 * MM, 14 * MM, 4 * MM, 6, 5, 2, Material(0.3e6, 0.45, 1000.0), name="coarse")
    V, F = meshes.box_surface(1 * MM, 1 * MM, 1 * MM)
    a = np.ones(3) / math.sqrt(3.0)                    # corner (-1,-1,-1) -> straight down
    b = np.array([0.0, 0.0, 1.0])
    k = np.cross(a, b)
    sk = np.linalg.norm(k)
    k /= sk
    th = math.atan2(sk, a @ b)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    R = np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K
    X = pad.X
    top = np.nonzero(np.isclose(X[:, 2], 4 * MM))[0]
    # the top-face triangle of the cell left of the pad's centre
    cx = X[top, 0][np.argmin(np.abs(X[top, 0] - 9 * MM))]
    cy = X[top, 1][np.argmin(np.abs(X[top, 1] - 7 * MM))]
    tip_xy = np.array([cx - 2.0 * MM, cy + 0.9 * MM])
    params = Params()
    tip = (V @ R.T)[np.argmin((V @ R.T)[:, 2])]
    c = np.array([tip_xy[0], tip_xy[1], 4 * MM + params.dhat]) - tip
    ind = Indenter(MESH, (0.0, 0.0, 0.0, 0.0), R, c, mesh=(V, F))
    return Episode(pad, ind, 0.3 * MM, 3, params, mesh_contact=mesh_contact)


def _rot_z(angle):
    c, s = math.cos(angle), math.sin(angle)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], float)


def press_slide_episode():
    """Friction workload (friction ratio 0.5, eps_v = 0.01 m/s of Sec.
    III-B): config1's 18x14x4 mm pad (12x9x3 cells), sphere r = 5 mm pressed
    0.5 mm over 4 steps at (6, 7) mm, then slid 0.25 mm per step along +x
    while twisting 3 degrees per step about its vertical axis, 6 steps.
    Returns (pad, params, [pose of step 1 .. 10])."""
    pad = box_pad(18 * MM, 14 * MM, 4 * MM, 12, 9, 3, Material(0.3e6, 0.45, 1000.0), name="slide")
    params = Params()
    r = 5 * MM
    start = place_indenter(pad, SPHERE, (6 * MM, 7 * MM), params.dhat, sphere_radius=r)
    poses = []
    for s in range(1, 11):
        depth = 0.5 * MM * min(s, 4) / 4
        k = max(s - 4, 0)
        c = start.c + np.array([0.25 * MM * k, 0.0, -depth])
        poses.append(Indenter(SPHERE, start.prm, _rot_z(math.radians(3.0 * k)), c))
    return pad, params, poses


def mesh_press_episode():
    """Rigid triangle-mesh indenters on config1's pad: a torus surface (ring
    4 mm, tube 1.5 mm, 16 x 8 quads, a facet strip at the bottom) lying flat
    at (9, 7) mm, pressed 0.5 mm over 5 steps.  Returns (pad, params, [pose
    of step 1 .. 5])."""
    pad = box_pad(18 * MM, 14 * MM, 4 * MM, 12, 9, 3, Material(0.3e6, 0.45, 1000.0), name="mesh")
    params = Params()
    mesh = meshes.torus_surface(4 * MM, 1.5 * MM, 16, 8, phase=0.5)
    low = -mesh[0][:, 2].min()
    c = np.array([9 * MM, 7 * MM, pad.X[:, 2].max() + params.dhat + low])
    start = Indenter(MESH, (0.0, 0.0, 0.0, 0.0), np.eye(3), c, mesh)
    return pad, params, [start.at_depth(0.5 * MM * s / 5) for s in range(1, 6)]


def mesh_slide_episode():
    """press_slide_episode with the sphere given as an icosphere surface
    (r = 5 mm, 320 triangles): the facets turn with the twist."""
    pad, params, poses = press_slide_episode()
    mesh = meshes.icosphere(5 * MM, 2)
    return pad, params, [Indenter(MESH, (0.0, 0.0, 0.0, 0.0), p.R, p.c, mesh) for p in poses]


def config1():
    """Single 18x14x4 mm pad, 12x9x3 cells, sphere r = 5 mm at a seeded (x, y)
    on the top face shrunk by r/2 margins (seed 1), 0.5 mm over 10 steps."""
    pad = box_pad(18 * MM, 14 * MM, 4 * MM, 12, 9, 3, Material(0.3e6, 0.45, 1000.0),
                  name="config1")
    params = Params()
    rng = np.random.default_rng(1)
    r = 5 * MM
    xy = (rng.uniform(r / 2, pad.dims[0] - r / 2), rng.uniform(r / 2, pad.dims[1] - r / 2))
    ind = place_indenter(pad, SPHERE, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, 0.5 * MM, 10, params)


def config2_pad():
    zs = meshes.graded_axis_top(4 * MM, 13, 0.2 * MM)
    return box_pad(18 * MM, 14 * MM, 4 * MM, 45, 35, 13, Material(0.3e6, 0.45, 1000.0),
                   name="config2", zs=zs)


def config2(i, pad=None):
    """Graded 45x35x13 pad; episode i in 0..4 = sphere, cylinder, cube edge,
    torus, texture; depth ~ U[0.2, 1.0] mm, 30 steps (SeedSequence(2).spawn(5))."""
    pad = pad or config2_pad()
    params = Params()
    rng = np.random.default_rng(np.random.SeedSequence(2).spawn(5)[i])
    shape = (SPHERE, CYLINDER, BOX, TORUS, TEXTURE)[i]
    depth = rng.uniform(0.2, 1.0) * MM
    r = rng.uniform(2, 8) * MM if shape == SPHERE else None
    _, _, foot, _ = indenter_geometry(shape, rng, r)
    margin = 0.5 * foot if np.isfinite(foot) else 0.0
    xy = seeded_xy(rng, pad, margin)
    ind = place_indenter(pad, shape, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, depth, 30, params)


def _random_env(rng, target_lo, target_hi, log_uniform, n_steps, schedule):
    shape_idx = int(rng.integers(3))
    if log_uniform:
        target = math.exp(rng.uniform(math.log(target_lo), math.log(target_hi)))
    else:
        target = rng.uniform(target_lo, target_hi)
    mat = Material(rng.uniform(0.1, 1.0) * 1e6, rng.uniform(0.40, 0.48), 1000.0)
    pad = pad_for_target(shape_idx, target, mat)
    params = Params()
    shape = int(rng.integers(5))
    r = rng.uniform(2, 8) * MM if shape == SPHERE else None
    _, _, foot, _ = indenter_geometry(shape, rng, r)
    margin = 0.5 * foot if np.isfinite(foot) else 0.0
    xy = seeded_xy(rng, pad, margin)
    depth = rng.uniform(0.2, 1.0) * MM
    ind = place_indenter(pad, shape, xy, params.dhat, sphere_radius=r)
    return Episode(pad, ind, depth, n_steps, params, schedule)


def config3(n_envs=60):
    """60 uneven envs from SeedSequence(3).spawn(60): pad shape uniform over
    three, tets ~ U[20k, 80k], E ~ U[0.1, 1.0] MPa, nu ~ U[0.40, 0.48], random
    indenter type/pose, depth ~ U[0.2, 1.0] mm over 30 steps."""
    seqs = np.random.SeedSequence(3).spawn(60)
    return [_random_env(np.random.default_rng(s), 20e3, 80e3, False, 30, "press")
            for s in seqs[:n_envs]]


def mesh_indenter(ind):
    """The same indenter given as a closed triangle surface (MESH), where
    the shape is bounded: sphere -> icosphere (1,280 triangles, vertices on
    the sphere), cylinder -> 32-gon prism, cube -> its 12 triangles, torus ->
    32 x 12 quads with a facet strip at the bottom.  Every mesh lies inside
    its analytic shape, so a start pose feasible for the shape stays
    feasible.  The texture plate (unbounded) stays analytic."""
    p = ind.prm
    if ind.shape == SPHERE:
        mesh = meshes.icosphere(p[0], 3)
    elif ind.shape == CYLINDER:
        mesh = meshes.cylinder_surface(p[0], p[1], 32)
    elif ind.shape == BOX:
        mesh = meshes.box_surface(p[0], p[1], p[2])
    elif ind.shape == TORUS:
        mesh = meshes.torus_surface(p[0], p[1], 32, 12, phase=0.5)
    else:
        return ind
    return Indenter(MESH, (0.0, 0.0, 0.0, 0.0), ind.R.copy(), ind.c.copy(), mesh)


VARIANTS = ("slide", "friction", "layers", "mesh", "mesh2")


def config3_variant(kind, n_envs=60):
    """config3's pads, materials and start poses with one feature beyond the
    frictionless press switched on for every pad (variant draws from
    SeedSequence(5), one per pad):
      slide    : pressed to depth over 15 steps, then slid 0.1 mm per step
                 (6 mm/s) in a seeded direction (friction off);
      friction : the same press-slide with friction ratio 0.5 (Sec. III-B);
      layers   : two layers split at half thickness, the drawn material on
                 top and a base 8x stiffer (nu = 0.42, rho = 1200), the
                 dual-layer gel of Sec. IV-D;
      mesh     : the bounded indenters given as triangle meshes (mesh_indenter);
                 the torus, whose mesh has concave edges on the inner side
                 of the tube, with the barrier summed over triangle pairs
                 (mesh_contact 1: the distance to the whole mesh has a kink
                 across each concave edge, where Newton can stall);
      mesh2    : the same meshes, every one with mesh_contact 2 (also mesh
                 vertices against pad triangles and edge-edge pairs)."""
    if kind not in VARIANTS:
        raise ValueError(kind)
    rng = np.random.default_rng(np.random.SeedSequence(5))
    out = []
    for e in config3(n_envs):
        ang = rng.uniform(0.0, 2.0 * math.pi)
        if kind in ("slide", "friction"):
            v = 0.1 * MM * np.array([math.cos(ang), math.sin(ang)])
            e = dataclasses.replace(e, n_steps=15, slide=v, friction=0.5 if kind == "friction" else 0.0)
        elif kind == "layers":
            m = e.pad.material
            idx, mats = layered_materials(e.pad.X, e.pad.tets, e.pad.X[:, 2].min() + 0.5 * e.pad.dims[2], m,
                                          Material(8.0 * m.E, 0.42, 1200.0))
            e = dataclasses.replace(e, layers=(idx, mats))
        elif kind == "mesh":
            e = dataclasses.replace(e, indenter=mesh_indenter(e.indenter),
                                    mesh_contact=int(e.indenter.shape == TORUS))
        else:
            mi = mesh_indenter(e.indenter)
            e = dataclasses.replace(e, indenter=mi, mesh_contact=2 if mi.shape == MESH else 0)
        out.append(e)
    return out


def paper60(n_envs=60):
    """A stand-in for the paper's own multi-environment run (Sec. IV-A: 60
    environments of a GelSight Mini pad of about 1,900 tets, d_hat = 1 mm,
    friction ratio 0.5): 60 copies of config1's 18x14x4 mm pad (1,944 tets,
    E = 0.3 MPa, nu = 0.45), each under its own indenter drawn from
    SeedSequence(6) (shape uniform over the five, sphere radius U[2, 8] mm,
    seeded position on the face), d_hat = 1 mm, friction 0.5, pressed
    U[0.2, 1.0] mm over 30 steps."""
    seqs = np.random.SeedSequence(6).spawn(n_envs)
    out = []
    for s in seqs:
        rng = np.random.default_rng(s)
        pad = box_pad(18 * MM, 14 * MM, 4 * MM, 12, 9, 3, Material(0.3e6, 0.45, 1000.0), name="paper60")
        params = Params(dhat=1.0 * MM)
        shape = int(rng.integers(5))
        r = rng.uniform(2, 8) * MM if shape == SPHERE else None
        _, _, foot, _ = indenter_geometry(shape, rng, r)
        margin = 0.5 * foot if np.isfinite(foot) else 0.0
        xy = seeded_xy(rng, pad, margin)
        depth = rng.uniform(0.2, 1.0) * MM
        ind = place_indenter(pad, shape, xy, params.dhat, sphere_radius=r)
        out.append(Episode(pad, ind, depth, 30, params, friction=0.5))
    return out


def config4(n_pads=256):
    """256 resident pads, tets log-uniform in [5k, 150k] (SeedSequence(4));
    each pad presses and releases its indenter over 2 x 30 steps."""
    seqs = np.random.SeedSequence(4).spawn(n_pads + 1)
    return [_random_env(np.random.default_rng(s), 5e3, 150e3, True, 30, "triangle")
            for s in seqs[:n_pads]]


def config4_arrivals(rate_hz, duration_s, n_pads, seed=4):
    """Poisson arrival times and uniformly chosen pad ids."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(n_pads + 1)[-1])
    n = rng.poisson(rate_hz * duration_s)
    t = np.sort(rng.uniform(0.0, duration_s, n))
    env = rng.integers(0, n_pads, n)
    return t, env


def config5_axes(h_f, centre):
    L, H = 24 * MM, 5 * MM
    xs = meshes.sizing_profile_axis(L, centre[0], h_f)
    ys = meshes.sizing_profile_axis(L, centre[1], h_f)
    zs = meshes.graded_axis_top(H, 12, h_f)
    return xs, ys, zs


def config5(target=1.2e6):
    """24x24x5 mm pad, x/y spacing from the cosine sizing profile around a
    seeded patch centre quantised to h_f * {1, 2, 4, 8}, 12 graded layers with
    top layer h_f; h_f chosen so that tets ~ 1.2M; sphere r = 3 mm pressed
    1.0 mm over 60 steps at the patch centre."""
    rng = np.random.default_rng(np.random.SeedSequence(5))
    L = 24 * MM
    centre = (rng.uniform(0.35 * L, 0.65 * L), rng.uniform(0.35 * L, 0.65 * L))
    lo, hi = 0.02 * MM, 0.5 * MM
    best = None
    for _ in range(40):
        h = math.sqrt(lo * hi)
        xs, ys, zs = config5_axes(h, centre)
        n = 6 * (len(xs) - 1) * (len(ys) - 1) * (len(zs) - 1)
        if best is None or abs(n - target) < abs(best[1] - target):
            best = (h, n)
        if n > target:
            lo = h
        else:
            hi = h
    h_f = best[0]
    xs, ys, zs = config5_axes(h_f, centre)
    X, T = meshes.kuhn_grid(xs, ys, zs)
    pad = Pad("config5", X, T, Material(0.3e6, 0.45, 1000.0), (L, L, 5 * MM))
    params = Params()
    ind = place_indenter(pad, SPHERE, centre, params.dhat, sphere_radius=3 * MM)
    return Episode(pad, ind, 1.0 * MM, 60, params)


def config5_refine_base():
    """The large pad built by conforming refinement instead of a graded grid:
    a uniform 28 x 28 x 6-cell Kuhn mesh of the 24 x 24 x 5 mm pad (28,224
    tets) and the Sec. III-A sizing field around config5's seeded patch
    centre (l_c = 0.075 mm, l_g = 1.6 mm, other constants default), which
    refines it to about 1.35 M tets.  Returns (coarse pad, sizing keywords);
    the episode is config5's: sphere r = 3 mm at the centre, 1.0 mm over 60
    steps, placed on the refined pad."""
    rng = np.random.default_rng(np.random.SeedSequence(5))
    L = 24 * MM
    centre = (rng.uniform(0.35 * L, 0.65 * L), rng.uniform(0.35 * L, 0.65 * L))
    pad = box_pad(L, L, 5 * MM, 28, 28, 6, Material(0.3e6, 0.45, 1000.0), name="config5_refined")
    return pad, dict(l_contact=0.075 * MM, l_global=1.6 * MM, centre=centre)


def config5_refined(X, tets):
    """config5's episode on a refined pad (X, tets from refining the
    config5_refine_base mesh)."""
    base, kw = config5_refine_base()
    pad = Pad("config5_refined", np.asarray(X, np.float64), np.asarray(tets, np.int32), base.material, base.dims)
    params = Params()
    ind = place_indenter(pad, SPHERE, kw["centre"], params.dhat, sphere_radius=3 * MM)
    return Episode(pad, ind, 1.0 * MM, 60, params)
