"""MI355X tactile-FEM hot path (TaCauchy) - Python binding of libtacauchy.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI (include/tacauchy.h).  torch is used for device memory and
streams only.  Importing the package does not touch the GPU; creating a
Context does, and fails loudly without a gfx950 device or a built library.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (BOX, CYLINDER, FIELDS, MESH, PREC_FP64, PREC_MIXED, PRECOND_BLOCK_JACOBI,  # noqa: F401
                   PRECOND_JACOBI, SPHERE, TEXTURE, TORUS, TcError, check, load)

# Live library objects, closed in dependency order (servers, pads, contexts)
# before the interpreter and the HIP runtime shut down.
_LIVE = {"server": weakref.WeakSet(), "pad": weakref.WeakSet(), "ctx": weakref.WeakSet()}


@atexit.register
def _close_all():
    for kind in ("server", "pad", "ctx"):
        for obj in list(_LIVE[kind]):
            try:
                obj.close()
            except Exception:
                pass


_DT_NP = {_abi.DT_F64: np.float64, _abi.DT_F32: np.float32, _abi.DT_I32: np.int32, _abi.DT_U8: np.uint8}


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None else None


def make_params(**kw) -> _abi.TcParams:
    """tc_params with library defaults, overridden by keyword arguments
    (dt, dhat, kappa, newton_tol, cg_rel_tol, max_newton, max_cg,
    quasi_static, precision, gravity, literal_alpha, precond, max_halvings,
    cg_forcing, hess_proj, init_guess, cg_conv_tol, cg_eta_max, ls_expand,
    mesh_contact, friction, eps_v, cg_warm)."""
    p = _abi.TcParams()
    check(load().tc_params_default(C.byref(p)))
    for k, v in kw.items():
        if k == "gravity":
            for i in range(3):
                p.gravity[i] = float(v[i])
        elif k == "precision" and isinstance(v, str):
            p.precision = PREC_FP64 if v.lower() in ("fp64", "f64", "double") else PREC_MIXED
        else:
            if not hasattr(p, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(p, k, type(getattr(p, k))(v))
    return p


def to_indenter(ind) -> _abi.TcIndenter:
    """Any object with shape, prm (<= 4), R (3x3), c (3) -> tc_indenter;
    a MESH indenter also carries mesh_id (from Context.add_mesh)."""
    if isinstance(ind, _abi.TcIndenter):
        return ind
    get = (lambda k: ind[k]) if isinstance(ind, dict) else (lambda k: getattr(ind, k))
    t = _abi.TcIndenter()
    t.shape = int(get("shape"))
    if t.shape == MESH:
        t.reserved = int(get("mesh_id"))
    R = np.asarray(get("R"), dtype=np.float64).reshape(9)
    c = np.asarray(get("c"), dtype=np.float64).reshape(3)
    prm = list(get("prm")) + [0.0] * 4
    for i in range(9):
        t.R[i] = R[i]
    for i in range(3):
        t.c[i] = c[i]
    for i in range(4):
        t.prm[i] = float(prm[i])
    return t


def _indenter_array(inds: Sequence):
    arr = (_abi.TcIndenter * max(len(inds), 1))()
    for i, ind in enumerate(inds):
        arr[i] = to_indenter(ind)
    return arr


class StepStats:
    __slots__ = ("status", "newton_iters", "cg_iters", "ls_halvings", "final_step_inf", "energy",
                 "reaction", "ms")

    def __init__(self, s: _abi.TcStepStats):
        self.status = s.status
        self.newton_iters = s.newton_iters
        self.cg_iters = s.cg_iters
        self.ls_halvings = s.ls_halvings
        self.final_step_inf = s.final_step_inf
        self.energy = s.energy
        self.reaction = np.array(list(s.reaction))
        self.ms = s.ms

    def __repr__(self):
        return (f"StepStats(status={self.status}, newton={self.newton_iters}, cg={self.cg_iters}, "
                f"ls={self.ls_halvings}, |p|={self.final_step_inf:.3e}, ms={self.ms:.3f})")


def _mesh(X, tets, fixed=None, tet_material=None):
    X = np.ascontiguousarray(X, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    fixed = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    tm = None if tet_material is None else np.ascontiguousarray(tet_material, dtype=np.int32)
    m = _abi.TcMesh(X.shape[0], tets.shape[0], _ptr(X, C.c_double), _ptr(tets, C.c_int32),
                    _ptr(fixed, C.c_uint8), _ptr(tm, C.c_int32))
    return m, (X, tets, fixed, tm)


def sizing(**kw) -> _abi.TcSizing:
    """tc_sizing with library defaults, overridden by keyword arguments
    (axis, side, band, inner, transition, l_contact, l_global, centre,
    max_tets)."""
    sz = _abi.TcSizing()
    check(load().tc_sizing_default(C.byref(sz)))
    for k, v in kw.items():
        if k == "centre":
            sz.centre[0], sz.centre[1] = float(v[0]), float(v[1])
        elif not hasattr(sz, k):
            raise TypeError(f"unknown sizing field {k}")
        else:
            setattr(sz, k, type(getattr(sz, k))(v))
    return sz


def refine_mesh(X, tets, tet_material=None, max_tets=2_000_000, **kw):
    """Host-only conforming refinement under the contact sizing field:
    returns (X', tets', material') with the input vertices first."""
    lib = load()
    m, keep = _mesh(X, tets, None, tet_material)
    sz = sizing(max_tets=max_tets, **kw)
    cap_t = int(max_tets)
    cap_v = int(np.asarray(X).shape[0]) + cap_t
    xo = np.empty((cap_v, 3))
    to = np.empty((cap_t, 4), np.int32)
    mo = np.empty(cap_t, np.int32)
    nv, nt = C.c_int32(), C.c_int32()
    check(lib.tc_refine_mesh(C.byref(m), C.byref(sz), cap_v, cap_t, _ptr(xo, C.c_double), _ptr(to, C.c_int32),
                             _ptr(mo, C.c_int32), C.byref(nv), C.byref(nt)))
    return xo[:nv.value].copy(), to[:nt.value].copy(), mo[:nt.value].copy()


def mesh_surface(X, tets, fixed=None):
    """Host-only Alg. 1 (surface extraction): dict(tris, parent, is_top, candidates)."""
    lib = load()
    m, keep = _mesh(X, tets, fixed)
    ns, nc = C.c_int32(), C.c_int32()
    check(lib.tc_mesh_surface(C.byref(m), C.byref(ns), C.byref(nc), None, None, None, None, 0, 0))
    tris = np.empty((ns.value, 3), np.int32)
    parent = np.empty(ns.value, np.int32)
    top = np.empty(ns.value, np.uint8)
    cand = np.empty(max(nc.value, 1), np.int32)
    check(lib.tc_mesh_surface(C.byref(m), C.byref(ns), C.byref(nc), _ptr(tris, C.c_int32),
                              _ptr(parent, C.c_int32), _ptr(top, C.c_uint8), _ptr(cand, C.c_int32),
                              ns.value, cand.size))
    return dict(tris=tris, parent=parent, is_top=top, candidates=cand[:nc.value])


class Context:
    """A device, a stream and an HBM budget.  stream: a torch.cuda.Stream, a
    raw hipStream_t integer, or None for a library-owned stream."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        self.lib = load()
        if stream is not None and hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        h = C.c_void_p()
        check(self.lib.tc_context_create(int(device), C.c_void_p(stream) if stream else None,
                                         int(hbm_budget), C.byref(h)))
        self.h = h
        self.device = device
        _LIVE["ctx"].add(self)

    def close(self):
        if getattr(self, "h", None):
            for srv in list(_LIVE["server"]):
                if srv.ctx is self:
                    srv.close()
            for pad in list(_LIVE["pad"]):
                if pad.ctx is self:
                    pad.close()
            self.lib.tc_context_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_mesh(self, verts, tris) -> int:
        """Register a closed, outward-oriented rigid triangle mesh (local
        frame, metres) as an indenter shape; returns its mesh_id."""
        V = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
        F = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
        mid = C.c_int32()
        check(self.lib.tc_rigid_mesh_create(self.h, V.shape[0], V.ctypes.data_as(C.POINTER(C.c_double)),
                                            F.shape[0], F.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(mid)))
        return mid.value

    def remove_mesh(self, mesh_id: int):
        check(self.lib.tc_rigid_mesh_destroy(self.h, int(mesh_id)))

    def memory(self):
        u, b = C.c_uint64(), C.c_uint64()
        check(self.lib.tc_context_memory(self.h, C.byref(u), C.byref(b)))
        return u.value, b.value

    def set_timing(self, on: bool, stride: int = 1):
        """Per-kernel event timing; with stride k only every k-th launch of
        each kernel is bracketed by events."""
        check(self.lib.tc_context_set_timing(self.h, int(stride) if on else 0))

    def reset_timing(self):
        check(self.lib.tc_context_reset_timing(self.h))

    def timing(self):
        """{kernel: (avg_ms, launches, algorithmic bytes per launch)}"""
        cap = 64
        n = C.c_int32()
        names = (C.c_char * _abi.TIMER_NAME_LEN * cap)()
        avg = (C.c_double * cap)()
        cnt = (C.c_int64 * cap)()
        byt = (C.c_double * cap)()
        check(self.lib.tc_context_timing(self.h, cap, C.byref(n), names, avg, cnt, byt))
        return {names[i].value.decode(): (avg[i], cnt[i], byt[i]) for i in range(n.value)}

    def set_launch(self, cg_block=0, elem_block=0, spmv_block=0, cg_per_replay=0, use_graphs=-1):
        check(self.lib.tc_set_launch(self.h, cg_block, elem_block, spmv_block, cg_per_replay, use_graphs))

    def set_streams(self, n: int):
        """Split batch steps over n streams (1..4), one host thread each."""
        check(self.lib.tc_set_streams(self.h, int(n)))

    def set_schedule(self, staged: bool = True, line_search_evals: int = 0):
        """Batch schedule: staged (each pad through its Newton iterations at
        its own pace, in rounds of launches) or lockstep; trial energies per
        round (0 keeps the current value)."""
        check(self.lib.tc_set_schedule(self.h, int(bool(staged)), int(line_search_evals)))

    def autotune(self, pads: Sequence["Pad"], indenters: Sequence[Sequence]):
        n = len(pads)
        ph = (C.c_void_p * n)(*[p.h for p in pads])
        nind = (C.c_int32 * n)(*[len(i) for i in indenters])
        flat = _indenter_array([x for inds in indenters for x in inds])
        chosen = (C.c_int32 * 5)()
        check(self.lib.tc_autotune(self.h, n, ph, nind, flat, chosen))
        return tuple(chosen)


class Pad:
    """A gel pad resident in HBM (mesh, material(s), solver parameters)."""

    def __init__(self, ctx: Context, X, tets, materials, params: Optional[_abi.TcParams] = None,
                 fixed=None, tet_material=None):
        self.ctx = ctx
        self.lib = ctx.lib
        mats = materials if isinstance(materials, (list, tuple)) else [materials]
        marr = (_abi.TcMaterial * len(mats))()
        for i, m in enumerate(mats):
            get = (lambda k: m[k]) if isinstance(m, dict) else (lambda k: getattr(m, k))
            marr[i] = _abi.TcMaterial(float(get("E")), float(get("nu")), float(get("density")))
        params = params if params is not None else make_params()
        mesh, keep = _mesh(X, tets, fixed, tet_material)
        h = C.c_void_p()
        check(self.lib.tc_pad_create(ctx.h, C.byref(mesh), len(mats), marr, C.byref(params), C.byref(h)))
        self.h = h
        self.params = params
        _LIVE["pad"].add(self)
        info = _abi.TcPadInfo()
        check(self.lib.tc_pad_get_info(self.h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in _abi.TcPadInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.tc_pad_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        check(self.lib.tc_pad_set_params(self.h, C.byref(params)))
        self.params = params

    def reset(self):
        check(self.lib.tc_pad_reset(self.h))

    def release_scratch(self):
        check(self.lib.tc_pad_release_scratch(self.h))

    def step(self, indenters: Sequence = (), raise_on_error=True) -> StepStats:
        arr = _indenter_array(indenters)
        st = _abi.TcStepStats()
        s = self.lib.tc_step(self.h, len(indenters), arr, C.byref(st))
        if raise_on_error:
            check(s)
        return StepStats(st)

    def extract(self, indenters: Sequence = ()):
        check(self.lib.tc_extract(self.h, len(indenters), _indenter_array(indenters)))

    def extract_noalloc(self, indenters: Sequence = ()):
        """tc_extract without any allocation (fixed device scratch);
        returns the reaction [3]."""
        r = (C.c_double * 3)()
        check(self.lib.tc_extract_noalloc(self.h, len(indenters), _indenter_array(indenters), r))
        return np.array(r[:])

    def newton_direction(self, indenters: Sequence = ()):
        """(p, dE/dx) at the committed positions, both [V,3] float64."""
        V = self.info["n_verts"]
        d = np.zeros((V, 3))
        g = np.zeros((V, 3))
        check(self.lib.tc_pad_newton_direction(self.h, len(indenters), _indenter_array(indenters),
                                               d.ctypes.data_as(C.POINTER(C.c_double)),
                                               g.ctypes.data_as(C.POINTER(C.c_double))))
        return d, g

    def field_info(self, field):
        f = FIELDS[field] if isinstance(field, str) else int(field)
        dt, n, c = C.c_int32(), C.c_int64(), C.c_int32()
        check(self.lib.tc_field_info(self.h, f, C.byref(dt), C.byref(n), C.byref(c)))
        return f, dt.value, n.value, c.value

    def read(self, field, device: bool = False):
        """numpy array (host) or torch tensor on the context's device."""
        f, dt, n, c = self.field_info(field)
        shape = (n, c) if c > 1 else (n,)
        if device:
            import torch
            tdt = {_abi.DT_F64: torch.float64, _abi.DT_F32: torch.float32,
                   _abi.DT_I32: torch.int32, _abi.DT_U8: torch.uint8}[dt]
            out = torch.empty(shape, dtype=tdt, device=f"cuda:{self.ctx.device}")
            check(self.lib.tc_pad_read(self.h, f, C.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size(), 1))
            return out
        out = np.empty(shape, dtype=_DT_NP[dt])
        check(self.lib.tc_pad_read(self.h, f, out.ctypes.data_as(C.c_void_p), out.nbytes, 0))
        return out

    def write(self, field, value):
        f = FIELDS[field] if isinstance(field, str) else int(field)
        if hasattr(value, "data_ptr"):
            check(self.lib.tc_pad_write(self.h, f, C.c_void_p(value.data_ptr()),
                                        value.numel() * value.element_size(), 1))
        else:
            a = np.ascontiguousarray(value, dtype=np.float64)
            check(self.lib.tc_pad_write(self.h, f, a.ctypes.data_as(C.c_void_p), a.nbytes, 0))

    def save_state(self) -> bytes:
        n = C.c_size_t()
        check(self.lib.tc_pad_save_state(self.h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        check(self.lib.tc_pad_save_state(self.h, buf, C.byref(n)))
        return bytes(buf)

    def load_state(self, data: bytes):
        buf = C.create_string_buffer(data, len(data))
        check(self.lib.tc_pad_load_state(self.h, buf, len(data)))


def step_batch(ctx: Context, pads: Sequence[Pad], indenters: Sequence[Sequence],
               raise_on_error=True) -> List[StepStats]:
    """One fused step of every pad; indenters[i] are pad i's poses."""
    n = len(pads)
    ph = (C.c_void_p * n)(*[p.h for p in pads])
    nind = (C.c_int32 * n)(*[len(i) for i in indenters])
    flat = _indenter_array([x for inds in indenters for x in inds])
    st = (_abi.TcStepStats * n)()
    s = ctx.lib.tc_step_batch(ctx.h, n, ph, nind, flat, st)
    if raise_on_error:
        check(s)
    return [StepStats(st[i]) for i in range(n)]


class Server:
    """Continuous-batching step server on its own host thread."""

    def __init__(self, ctx: Context, max_slots: int):
        self.ctx = ctx
        self.lib = ctx.lib
        h = C.c_void_p()
        check(self.lib.tc_server_create(ctx.h, int(max_slots), C.byref(h)))
        self.h = h
        _LIVE["server"].add(self)

    def submit(self, pad: Pad, indenters: Sequence = (), tag: int = 0) -> int:
        t = C.c_uint64()
        check(self.lib.tc_server_submit(self.h, pad.h, int(tag), len(indenters),
                                        _indenter_array(indenters), C.byref(t)))
        return t.value

    def poll(self, cap: int = 256, wait_us: int = 0):
        out = (_abi.TcResult * cap)()
        n = C.c_int32()
        check(self.lib.tc_server_poll(self.h, out, cap, C.byref(n), int(wait_us)))
        res = []
        for i in range(n.value):
            r = out[i]
            res.append(dict(ticket=r.ticket, status=r.status, tag=r.pad_index, t_arrive_ms=r.t_arrive_ms,
                            t_admit_ms=r.t_admit_ms, t_done_ms=r.t_done_ms, stats=StepStats(r.stats)))
        return res

    def stats(self):
        s = _abi.TcServerStats()
        check(self.lib.tc_server_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _abi.TcServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.tc_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate(mesh=None, materials=None, params=None, indenters=None, rigid_mesh=None):
    """Host-only argument checks; raises TcError on the first problem.
    rigid_mesh: (verts, tris) of a TC_MESH indenter shape."""
    lib = load()
    if rigid_mesh is not None:
        V = np.ascontiguousarray(rigid_mesh[0], dtype=np.float64).reshape(-1, 3)
        F = np.ascontiguousarray(rigid_mesh[1], dtype=np.int32).reshape(-1, 3)
        check(lib.tc_validate_rigid_mesh(V.shape[0], V.ctypes.data_as(C.POINTER(C.c_double)),
                                         F.shape[0], F.ctypes.data_as(C.POINTER(C.c_int32))))
    if mesh is not None:
        X, tets = mesh[0], mesh[1]
        fixed = mesh[2] if len(mesh) > 2 else None
        m, keep = _mesh(X, tets, fixed)
        check(lib.tc_validate_mesh(C.byref(m), 8))
    if materials is not None:
        mats = materials if isinstance(materials, (list, tuple)) else [materials]
        arr = (_abi.TcMaterial * max(len(mats), 1))()
        for i, mm in enumerate(mats):
            arr[i] = _abi.TcMaterial(*[float(mm[k]) if isinstance(mm, dict) else float(getattr(mm, k))
                                       for k in ("E", "nu", "density")])
        check(lib.tc_validate_materials(len(mats), arr))
    if params is not None:
        check(lib.tc_validate_params(C.byref(params)))
    if indenters is not None:
        check(lib.tc_validate_indenters(len(indenters), _indenter_array(indenters)))
