"""ctypes mirror of include/tacauchy.h (structures, constants, prototypes)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtacauchy.so")

# status codes
OK, E_INVALID_ARG, E_BAD_MESH, E_NO_MEMORY, E_HIP = 0, -1, -2, -3, -4
E_INFEASIBLE, E_NOT_CONVERGED, E_LINESEARCH, E_NO_DEVICE, E_BUSY = -5, -6, -7, -8, -9
PREC_FP64, PREC_MIXED = 0, 1
PRECOND_BLOCK_JACOBI, PRECOND_JACOBI = 0, 1
SPHERE, CYLINDER, BOX, TORUS, TEXTURE, MESH = 0, 1, 2, 3, 4, 5
MAX_MESHES = 64
MAX_INDENTERS, MAX_MATERIALS = 5, 8
DT_F64, DT_F32, DT_I32, DT_U8 = 0, 1, 2, 3
TIMER_NAME_LEN = 32

FIELDS = {
    "positions": 0, "velocities": 1, "rest": 2, "sigma": 3, "traction": 4, "pressure": 5,
    "tangential": 6, "tri_area": 7, "tri_normal": 8, "contact_force": 9, "contact_normal": 10,
    "contact_area": 11, "contact_fn": 12, "contact_ft": 13, "contact_pressure": 14,
    "reaction": 15, "traction_sum": 16, "surface_tris": 17, "surface_parent": 18,
    "surface_is_top": 19, "candidates": 20, "cand_rest_area": 21, "mass": 22, "fixed": 23,
    "tets": 24,
}


class TcMesh(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32),
                ("rest_xyz", C.POINTER(C.c_double)), ("tets", C.POINTER(C.c_int32)),
                ("fixed", C.POINTER(C.c_uint8)), ("tet_material", C.POINTER(C.c_int32))]


class TcMaterial(C.Structure):
    _fields_ = [("E", C.c_double), ("nu", C.c_double), ("density", C.c_double)]


class TcParams(C.Structure):
    _fields_ = [("dt", C.c_double), ("dhat", C.c_double), ("kappa", C.c_double),
                ("newton_tol", C.c_double), ("cg_rel_tol", C.c_double),
                ("max_newton", C.c_int32), ("max_cg", C.c_int32), ("quasi_static", C.c_int32),
                ("precision", C.c_int32), ("gravity", C.c_double * 3),
                ("literal_alpha", C.c_int32), ("precond", C.c_int32),
                ("max_halvings", C.c_int32), ("cg_forcing", C.c_int32),
                ("hess_proj", C.c_int32), ("init_guess", C.c_int32),
                ("cg_conv_tol", C.c_double), ("cg_eta_max", C.c_double),
                ("ls_expand", C.c_int32), ("mesh_contact", C.c_int32),
                ("friction", C.c_double), ("eps_v", C.c_double),
                ("cg_warm", C.c_int32), ("reserved0", C.c_int32)]


class TcSizing(C.Structure):
    _fields_ = [("axis", C.c_int32), ("side", C.c_int32), ("band", C.c_double), ("inner", C.c_double),
                ("transition", C.c_double), ("l_contact", C.c_double), ("l_global", C.c_double),
                ("centre", C.c_double * 2), ("max_tets", C.c_int64)]


class TcIndenter(C.Structure):
    _fields_ = [("shape", C.c_int32), ("reserved", C.c_int32), ("R", C.c_double * 9),
                ("c", C.c_double * 3), ("prm", C.c_double * 4)]


class TcStepStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("cg_iters", C.c_int32),
                ("ls_halvings", C.c_int32), ("final_step_inf", C.c_double), ("energy", C.c_double),
                ("reaction", C.c_double * 3), ("ms", C.c_double)]


class TcPadInfo(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("n_surface_tris", C.c_int32),
                ("n_top_tris", C.c_int32), ("n_candidates", C.c_int32), ("ell_width", C.c_int32),
                ("precision", C.c_int32), ("n_materials", C.c_int32),
                ("resident_bytes", C.c_uint64), ("scratch_bytes", C.c_uint64),
                ("bbox_diag", C.c_double)]


class TcResult(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("pad_index", C.c_int32),
                ("t_arrive_ms", C.c_double), ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double),
                ("stats", TcStepStats)]


class TcServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("rejected", C.c_int64), ("queued", C.c_int32), ("running", C.c_int32),
                ("max_running_seen", C.c_int32), ("ticks", C.c_int64),
                ("scratch_in_use", C.c_uint64), ("evictions", C.c_int64)]


P = C.c_void_p
S = C.c_int32
PROTOS = {
    "tc_version": (C.c_char_p, []),
    "tc_status_string": (C.c_char_p, [S]),
    "tc_last_error": (C.c_char_p, []),
    "tc_params_default": (S, [C.POINTER(TcParams)]),
    "tc_validate_mesh": (S, [C.POINTER(TcMesh), S]),
    "tc_validate_materials": (S, [S, C.POINTER(TcMaterial)]),
    "tc_validate_params": (S, [C.POINTER(TcParams)]),
    "tc_validate_indenters": (S, [S, C.POINTER(TcIndenter)]),
    "tc_mesh_surface": (S, [C.POINTER(TcMesh), C.POINTER(S), C.POINTER(S), C.POINTER(S), C.POINTER(S),
                            C.POINTER(C.c_uint8), C.POINTER(S), S, S]),
    "tc_context_create": (S, [S, P, C.c_uint64, C.POINTER(P)]),
    "tc_context_destroy": (S, [P]),
    "tc_context_memory": (S, [P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    "tc_context_set_timing": (S, [P, S]),
    "tc_context_timing": (S, [P, S, C.POINTER(S), P, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                              C.POINTER(C.c_double)]),
    "tc_context_reset_timing": (S, [P]),
    "tc_autotune": (S, [P, S, C.POINTER(P), C.POINTER(S), C.POINTER(TcIndenter), C.POINTER(S)]),
    "tc_set_launch": (S, [P, S, S, S, S, S]),
    "tc_set_streams": (S, [P, S]),
    "tc_set_schedule": (S, [P, S, S]),
    "tc_rigid_mesh_create": (S, [P, S, C.POINTER(C.c_double), S, C.POINTER(S), C.POINTER(S)]),
    "tc_rigid_mesh_destroy": (S, [P, S]),
    "tc_validate_rigid_mesh": (S, [S, C.POINTER(C.c_double), S, C.POINTER(S)]),
    "tc_sizing_default": (S, [C.POINTER(TcSizing)]),
    "tc_refine_mesh": (S, [C.POINTER(TcMesh), C.POINTER(TcSizing), S, S, C.POINTER(C.c_double), C.POINTER(S),
                           C.POINTER(S), C.POINTER(S), C.POINTER(S)]),
    "tc_pad_create": (S, [P, C.POINTER(TcMesh), S, C.POINTER(TcMaterial), C.POINTER(TcParams), C.POINTER(P)]),
    "tc_pad_destroy": (S, [P]),
    "tc_pad_get_info": (S, [P, C.POINTER(TcPadInfo)]),
    "tc_pad_set_params": (S, [P, C.POINTER(TcParams)]),
    "tc_pad_reset": (S, [P]),
    "tc_pad_release_scratch": (S, [P]),
    "tc_step": (S, [P, S, C.POINTER(TcIndenter), C.POINTER(TcStepStats)]),
    "tc_step_batch": (S, [P, S, C.POINTER(P), C.POINTER(S), C.POINTER(TcIndenter), C.POINTER(TcStepStats)]),
    "tc_extract": (S, [P, S, C.POINTER(TcIndenter)]),
    "tc_extract_noalloc": (S, [P, S, C.POINTER(TcIndenter), C.POINTER(C.c_double)]),
    "tc_pad_newton_direction": (S, [P, S, C.POINTER(TcIndenter), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "tc_field_info": (S, [P, S, C.POINTER(S), C.POINTER(C.c_int64), C.POINTER(S)]),
    "tc_pad_read": (S, [P, S, P, C.c_size_t, S]),
    "tc_pad_write": (S, [P, S, P, C.c_size_t, S]),
    "tc_pad_save_state": (S, [P, P, C.POINTER(C.c_size_t)]),
    "tc_pad_load_state": (S, [P, P, C.c_size_t]),
    "tc_server_create": (S, [P, S, C.POINTER(P)]),
    "tc_server_submit": (S, [P, P, S, S, C.POINTER(TcIndenter), C.POINTER(C.c_uint64)]),
    "tc_server_poll": (S, [P, C.POINTER(TcResult), S, C.POINTER(S), S]),
    "tc_server_get_stats": (S, [P, C.POINTER(TcServerStats)]),
    "tc_server_destroy": (S, [P]),
}

_lib = None


def load():
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2606_20426_amd.build` (there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


def status_name(s):
    return load().tc_status_string(int(s)).decode()


def check(status):
    if status != OK:
        raise TcError(status, load().tc_last_error().decode())
    return status
