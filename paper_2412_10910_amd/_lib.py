"""ctypes declarations of the C ABI in include/nnmg.h.

The shared library is built in-tree (``paper_2412_10910_amd/libnnmg.so``).
Importing this module fails loudly if it is missing: there is no fallback.
"""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnnmg.so")

NNMG_OK = 0
ERRORS = {
    -1: "INVALID_ARG",
    -2: "UNSUPPORTED",
    -3: "OOM",
    -4: "MESH",
    -5: "POINT_NOT_FOUND",
    -6: "NOT_CONVERGED",
    -7: "BREAKDOWN",
    -8: "HIP",
}
FP64, FP32 = 0, 1


class NNMGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nnmg error {ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Mesh(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n_vertices", C.c_int64),
        ("vertices", C.POINTER(C.c_double)),
        ("n_cells", C.c_int64),
        ("cells", C.POINTER(C.c_int32)),
        ("dirichlet_vertex", C.POINTER(C.c_uint8)),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("user", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


OP_LAPLACE, OP_ELASTICITY = 0, 1


class LevelOpts(C.Structure):
    _fields_ = [("op", C.c_int), ("lam", C.c_double), ("mu", C.c_double)]


class TransferOpts(C.Structure):
    _fields_ = [
        ("bbox_expand", C.c_double),
        ("inside_tol", C.c_double),
        ("newton_tol", C.c_double),
        ("newton_max_it", C.c_int),
        ("allow_projection", C.c_int),
        ("nested_p", C.c_int),
    ]


class MgOpts(C.Structure):
    _fields_ = [
        ("cheb_degree", C.c_int),
        ("smoothing_range", C.c_double),
        ("eig_safety", C.c_double),
        ("eig_iters", C.c_int),
        ("eig_start", C.POINTER(C.c_void_p)),
    ]


class CgOpts(C.Structure):
    _fields_ = [
        ("rtol", C.c_double),
        ("max_it", C.c_int),
        ("vcycle_prec", C.c_int),
        ("history", C.POINTER(C.c_double)),
        ("use_graph", C.c_int),
    ]


class CgResult(C.Structure):
    _fields_ = [("iterations", C.c_int), ("relres", C.c_double), ("status", C.c_int)]


class TuneResult(C.Structure):
    _fields_ = [("n_variants", C.c_int), ("ms", C.c_double * 16), ("chosen", C.c_int),
                ("rhs_split", C.c_int), ("ms_rhs", C.c_double * 2),
                ("cells_per_block", C.c_int), ("ms_cpb", C.c_double * 2)]


class ServerOpts(C.Structure):
    _fields_ = [("max_active", C.c_int), ("memory_budget", C.c_size_t), ("policy", C.c_int),
                ("aging_ms", C.c_double), ("large_work", C.c_double), ("max_large", C.c_int)]


class RequestTimes(C.Structure):
    _fields_ = [("queued_ms", C.c_double), ("run_ms", C.c_double), ("total_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("running", C.c_int), ("pending", C.c_int),
                ("max_running", C.c_int), ("reserved", C.c_size_t), ("max_reserved", C.c_size_t)]


# every symbol declared in include/nnmg.h, with its ctypes signature
_vp = C.c_void_p
_i64p = C.POINTER(C.c_int64)
SIGNATURES = {
    "nnmg_ctx_create": (C.c_int, [C.c_int, C.POINTER(Allocator), C.POINTER(_vp)]),
    "nnmg_ctx_destroy": (None, [_vp]),
    "nnmg_last_error": (C.c_char_p, []),
    "nnmg_default_level_opts": (None, [C.POINTER(LevelOpts)]),
    "nnmg_default_transfer_opts": (None, [C.POINTER(TransferOpts)]),
    "nnmg_default_mg_opts": (None, [C.POINTER(MgOpts)]),
    "nnmg_default_cg_opts": (None, [C.POINTER(CgOpts)]),
    "nnmg_level_create": (C.c_int, [_vp, C.POINTER(Mesh), C.c_int, C.POINTER(_vp)]),
    "nnmg_level_create_ex": (C.c_int, [_vp, C.POINTER(Mesh), C.c_int, C.POINTER(LevelOpts), C.POINTER(_vp)]),
    "nnmg_level_components": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "nnmg_level_destroy": (None, [_vp]),
    "nnmg_level_info": (C.c_int, [_vp, _i64p, _i64p, _i64p]),
    "nnmg_level_support_points": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "nnmg_level_constrained": (C.c_int, [_vp, C.POINTER(C.c_uint8)]),
    "nnmg_level_quadrature_points": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "nnmg_level_assemble_rhs": (C.c_int, [_vp, _vp, _vp, _vp]),
    "nnmg_vmult": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_vmult_add": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_vmult_noalloc": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_vmult_multi": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "nnmg_vmult_add_multi": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "nnmg_level_diagonal": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "nnmg_transfer_create": (C.c_int, [_vp, _vp, _vp, C.POINTER(TransferOpts), C.POINTER(_vp)]),
    "nnmg_transfer_destroy": (None, [_vp]),
    "nnmg_transfer_points": (C.c_int, [_vp, _i64p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), _i64p]),
    "nnmg_prolongate": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_restrict": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_prolongate_multi": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "nnmg_restrict_multi": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "nnmg_hierarchy_create": (C.c_int, [_vp, C.POINTER(_vp), C.c_int, C.POINTER(_vp), C.POINTER(MgOpts),
                                        C.POINTER(_vp)]),
    "nnmg_hierarchy_destroy": (None, [_vp]),
    "nnmg_get_cheb_bounds": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "nnmg_set_cheb_bounds": (C.c_int, [_vp, C.c_int, C.c_double, C.c_double]),
    "nnmg_vcycle": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp]),
    "nnmg_vcycle_multi": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "nnmg_pcg_solve": (C.c_int, [_vp, _vp, _vp, C.POINTER(CgOpts), C.POINTER(CgResult), _vp]),
    "nnmg_pcg_solve_multi": (C.c_int, [_vp, C.c_int, _vp, _vp, C.POINTER(CgOpts), C.POINTER(CgResult), _vp]),
    "nnmg_hierarchy_set_profiling": (C.c_int, [_vp, C.c_int]),
    "nnmg_hierarchy_footprint": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_size_t)]),
    "nnmg_default_server_opts": (None, [C.POINTER(ServerOpts)]),
    "nnmg_server_create": (C.c_int, [_vp, C.POINTER(ServerOpts), C.POINTER(_vp)]),
    "nnmg_server_destroy": (None, [_vp]),
    "nnmg_server_submit": (C.c_int, [_vp, _vp, C.c_int, _vp, _vp, C.POINTER(CgOpts), C.POINTER(C.c_int64)]),
    "nnmg_server_submit_any": (C.c_int, [_vp, C.POINTER(_vp), C.c_int, C.c_int, _vp, _vp, C.POINTER(CgOpts),
                                         C.POINTER(C.c_int64)]),
    "nnmg_server_poll": (C.c_int, [_vp, C.c_int64, C.POINTER(C.c_int)]),
    "nnmg_server_wait": (C.c_int, [_vp, C.c_int64, C.POINTER(CgResult), C.POINTER(RequestTimes)]),
    "nnmg_server_get_stats": (C.c_int, [_vp, C.POINTER(ServerStats)]),
    "nnmg_level_tune": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(TuneResult)]),
    "nnmg_level_set_variant": (C.c_int, [_vp, C.c_int]),
    "nnmg_level_set_variant_prec": (C.c_int, [_vp, C.c_int, C.c_int]),
    "nnmg_level_variant": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int)]),
    "nnmg_level_set_rhs_split": (C.c_int, [_vp, C.c_int, C.c_int]),
    "nnmg_level_set_cells_per_block": (C.c_int, [_vp, C.c_int, C.c_int]),
    "nnmg_level_cells_per_block": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _i64p]),
    "nnmg_transfer_tune": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(TuneResult)]),
    "nnmg_transfer_set_team": (C.c_int, [_vp, C.c_int]),
    "nnmg_transfer_team": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "nnmg_hierarchy_profile": (C.c_int, [_vp, C.POINTER(C.c_double)]),
}


def load(path: str = LIB_PATH) -> C.CDLL:
    # PyTorch's HIP runtime must be the one in the process before the library
    # is loaded: both carry the soname libamdhip64.so.7, so the library then
    # binds to torch's runtime, and the streams and pointers torch hands over
    # belong to the same runtime as the library's kernel launches
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it first (python paper_2412_10910_amd/csrc/build.py); "
            "there is no non-HIP fallback")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib() -> C.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load()
    return _LIB


def check(code: int) -> int:
    if code != NNMG_OK:
        msg = lib().nnmg_last_error()
        raise NNMGError(code, msg.decode() if msg else "")
    return code
