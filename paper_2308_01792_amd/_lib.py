"""ctypes declarations of the hytet C ABI (include/hytet.h)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HYTET_LIB names another build of the library (the sanitized host build
# used by the CPU tests); the default is the in-tree one.
LIB_PATH = os.environ.get("HYTET_LIB") or os.path.join(HERE, "libhytet.so")

HT_OK, HT_ERR_ARG, HT_ERR_MESH, HT_ERR_LEVEL, HT_ERR_OOM, HT_ERR_HIP, \
    HT_ERR_NOT_CONVERGED, HT_ERR_STATE = range(8)
HT_F64, HT_F32 = 0, 1
HT_PREC_F64, HT_PREC_MIXED = 0, 1
HT_SLOT_OWNER, HT_SLOT_GHOST, HT_SLOT_DIRICHLET, HT_SLOT_PAD = 1, 2, 4, 8

ERROR_NAMES = {HT_ERR_ARG: "HT_ERR_ARG", HT_ERR_MESH: "HT_ERR_MESH",
               HT_ERR_LEVEL: "HT_ERR_LEVEL", HT_ERR_OOM: "HT_ERR_OOM",
               HT_ERR_HIP: "HT_ERR_HIP",
               HT_ERR_NOT_CONVERGED: "HT_ERR_NOT_CONVERGED",
               HT_ERR_STATE: "HT_ERR_STATE"}


class LevelInfo(C.Structure):
    _fields_ = [("n_slots", C.c_int64), ("n_dofs", C.c_int64),
                ("n_unique", C.c_int64), ("n_cells", C.c_int64),
                ("n_faces", C.c_int64), ("n_edges", C.c_int64),
                ("n_vertices", C.c_int64), ("cell_stride", C.c_int64)]


HT_SMOOTH_JACOBI, HT_SMOOTH_CHEBYSHEV = 0, 1


class CycleOpts(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("omega", C.c_double),
                ("coarse_level", C.c_int), ("smoother", C.c_int),
                ("degree", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("cyc", CycleOpts), ("precision", C.c_int),
                ("rel_tol", C.c_double), ("max_cycles", C.c_int),
                ("use_graph", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("converged", C.c_int),
                ("rel_res", C.c_double), ("seconds", C.c_double),
                ("res_history", C.c_double * 257), ("stagnated", C.c_int)]


# name -> (restype, argtypes); every exported symbol of include/hytet.h
P, I, D, L = C.c_void_p, C.c_int, C.c_double, C.c_int64
SIGNATURES = {
    "ht_last_error": (C.c_char_p, []),
    "ht_version": (I, []),
    "ht_index_tw": (L, [L, L, L, L]),
    "ht_mesh_create": (I, [P, L, P, L, I, I, C.POINTER(P)]),
    "ht_mesh_destroy": (I, [P]),
    "ht_mesh_query": (I, [P, I, C.POINTER(LevelInfo)]),
    "ht_vertex_keys": (I, [P, I, L, L, P, P]),
    "ht_vertex_coords": (I, [P, I, L, L, P]),
    "ht_vertex_coords_device": (I, [P, I, I, P, P]),
    "ht_slot_flags_device": (I, [P, I, P, P]),
    "ht_slot_index": (I, [P, I, L, I, I, I, C.POINTER(L)]),
    "ht_cell_stencils": (I, [P, I, P]),
    "ht_p2_offsets": (I, [P, P]),
    "ht_p2_stencils": (I, [P, I, P]),
    "ht_sync": (I, [P, I, I, P, P]),
    "ht_fill_dirichlet": (I, [P, I, I, P, D, P]),
    "ht_lumped_mass": (I, [P, I, I, P, P]),
    "ht_norm": (I, [P, I, I, P, C.POINTER(D), P]),
    "ht_dot": (I, [P, I, I, P, P, C.POINTER(D), P]),
    "ht_copy": (I, [P, I, I, P, P, P]),
    "ht_apply": (I, [P, I, I, P, P, P]),
    "ht_apply_divkgrad": (I, [P, I, I, P, P, P, P]),
    "ht_apply_p2": (I, [P, I, I, P, P, P]),
    "ht_p2_pack": (I, [P, I, I, I, I, P, P, P]),
    "ht_p2_unpack": (I, [P, I, I, I, I, P, P, P]),
    "ht_assemble_divkgrad": (I, [P, I, I, P, P, P]),
    "ht_apply_stored": (I, [P, I, I, P, P, P, P]),
    "ht_residual": (I, [P, I, I, P, P, P, C.POINTER(D), P]),
    "ht_residual_noalloc": (I, [P, I, I, P, P, P, P, P]),
    "ht_smooth_jacobi": (I, [P, I, I, D, I, P, P, P]),
    "ht_restrict": (I, [P, I, I, P, P, P]),
    "ht_prolongate_add": (I, [P, I, I, P, P, P]),
    "ht_coarse_solve": (I, [P, I, I, P, P, P]),
    "ht_vcycle": (I, [P, I, I, C.POINTER(CycleOpts), P, P, P]),
    "ht_solve": (I, [P, I, C.POINTER(SolveOpts), P, P,
                     C.POINTER(SolveStats), P]),
    "ht_fmg": (I, [P, I, C.POINTER(CycleOpts), I, P, P, C.POINTER(D), P]),
    "ht_lambda_max": (I, [P, I, C.POINTER(D), P]),
    "ht_set_lambda_max": (I, [P, I, D]),
    "ht_batch_create": (I, [C.POINTER(P), C.POINTER(I), I, C.POINTER(P)]),
    "ht_batch_destroy": (I, [P]),
    "ht_batch_query": (I, [P, C.POINTER(I), C.POINTER(L), C.POINTER(L)]),
    "ht_batch_solve": (I, [P, C.POINTER(SolveOpts), C.POINTER(P),
                           C.POINTER(P), C.POINTER(SolveStats), P]),
    "ht_set_tile_rows": (I, [P, I, I, I]),
    "ht_get_tile_rows": (I, [P, I, I, C.POINTER(I)]),
    "ht_set_sweep_shape": (I, [P, I, I, I, I]),
    "ht_get_sweep_shape": (I, [P, I, I, C.POINTER(I), C.POINTER(I)]),
    "ht_set_march_segment": (I, [P, I, I, I]),
    "ht_get_march_segment": (I, [P, I, I, C.POINTER(I)]),
    "ht_batch_mesh": (I, [P, C.POINTER(P)]),
    "ht_batch_autotune": (I, [P, C.c_char_p, P]),
    "ht_autotune": (I, [P, I, I, C.c_char_p, C.POINTER(I), P]),
    "ht_profile_enable": (I, [P, I]),
    "ht_profile_query": (I, [P, C.c_char_p, C.POINTER(D), C.POINTER(L)]),
    "ht_profile_reset": (I, [P]),
    "ht_selftest_lane_shift": (I, [C.POINTER(I)]),
}

_LIB = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load the in-tree libhytet.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with "
            "`python -m paper_2308_01792_amd._build` (hipcc, gfx950)")
    # torch's ROCm build ships its own HIP runtime: load it first so that
    # the library and torch share one runtime (one device context)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class HytetError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int) -> None:
    if code != HT_OK:
        msg = load().ht_last_error()
        raise HytetError(code, msg.decode() if msg else "")
