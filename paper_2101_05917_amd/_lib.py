"""ctypes binding of libdiffpd.so (the C ABI declared in include/diffpd.h).

Argument marshalling only: every step of the simulation runs inside the
library's HIP kernels.  The library is built in-tree by ``_build.py``; if it
is missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffpd.so")

DPD_OK, DPD_NOT_CONVERGED = 0, 1
DPD_FP64, DPD_MIXED = 0, 1
DPD_BWD_FIXED_POINT, DPD_BWD_PCG = 0, 1
DPD_FWD_PD, DPD_FWD_NEWTON_PCG = 0, 1

STATUS_NAMES = {0: "DPD_OK", 1: "DPD_NOT_CONVERGED", -1: "DPD_EINVAL", -2: "DPD_ENOTSPD",
                -3: "DPD_ENOMEM", -4: "DPD_EHIP", -5: "DPD_ESTATE", -6: "DPD_ENONFINITE",
                -7: "DPD_ECURVATURE"}


class Options(C.Structure):
    _fields_ = [
        ("dx", C.c_double), ("rho", C.c_double), ("nu", C.c_double), ("h", C.c_double),
        ("gravity", C.c_double * 3), ("origin", C.c_double * 3),
        ("contact_k", C.c_double), ("friction_mu", C.c_double), ("friction_eps", C.c_double),
        ("muscle_k", C.c_double), ("fiber", C.c_double * 3),
        ("fwd_max_iter", C.c_int32), ("fwd_fixed_iters", C.c_int32),
        ("fwd_rel_tol", C.c_double), ("fwd_abs_tol_rel", C.c_double),
        ("fwd_solver", C.c_int32), ("fwd_inner_max_iter", C.c_int32), ("fwd_inner_tol", C.c_double),
        ("bwd_max_iter", C.c_int32), ("bwd_solver", C.c_int32), ("bwd_rel_tol", C.c_double),
        ("precision", C.c_int32), ("check_every", C.c_int32), ("use_graphs", C.c_int32),
        ("fused_cg", C.c_int32), ("contact_fused", C.c_int32), ("sweep_launch", C.c_int32),
        ("volume_scale", C.c_double), ("leaf_nodes", C.c_int32), ("deflation", C.c_int32),
        ("deflation_refresh", C.c_int32), ("factor_on_host", C.c_int32),
        ("bwd_warm_start", C.c_int32), ("pad_opt", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("fwd_iters", C.c_int32), ("fwd_outer", C.c_int32), ("bwd_iters", C.c_int32),
        ("converged", C.c_int32), ("fallbacks", C.c_int32), ("inverted_qps", C.c_int32),
        ("fwd_rel_res", C.c_double), ("bwd_rel_res", C.c_double), ("ms_total", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MeshInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_nodes", "n_elements", "n_free", "n_fixed", "n_contact", "n_supernodes", "n_levels",
        "factor_nnz", "factor_bytes", "device_bytes", "leaf_nodes", "fused_blocks", "fused_lds",
        "solve_workgroups", "solve_entries", "qp_per_element", "factor_us", "factor_flops")]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double), ("iterations", C.c_int64), ("event_ms", C.c_double)]


class Request(C.Structure):
    _fields_ = [("cells_ijk", C.POINTER(C.c_int32)), ("n_cells", C.c_int64),
                ("youngs", C.POINTER(C.c_double)), ("fixed_ijk", C.POINTER(C.c_int32)),
                ("n_fixed", C.c_int64), ("loss_x", C.POINTER(C.c_double)), ("n_nodes", C.c_int64),
                ("steps", C.c_int32), ("pad", C.c_int32), ("opt", Options)]


class Result(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("loss", C.c_double),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("n_nodes", C.c_int64), ("n_elements", C.c_int64), ("footprint_bytes", C.c_int64),
                ("fwd_iters", C.c_int64), ("bwd_iters", C.c_int64)]


class BatchStats(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("slot_iterations", C.c_int64), ("launches", C.c_int64),
                ("solves", C.c_int64), ("peak_slots", C.c_int32), ("pad", C.c_int32)]


DPD_PROF = {"off": 0, "sweep_fwd": 1, "sweep_bwd": 2, "elem_hvp": 3, "elem_forces": 4, "solve": 5,
            "sweep_fwd_wide": 6, "sweep_bwd_narrow": 7, "cg_dense": 8, "contact_update": 9,
            "contact_descend": 10, "contact_dense": 11, "contact_fused": 12,
            "contact_fused_cg": 13, "solve_dag": 14}

_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)

# name -> (restype, argtypes); the CPU tests check this list against the header
PROTOTYPES = {
    "dpd_default_options": (C.c_int, [C.POINTER(Options)]),
    "dpd_create_mesh": (C.c_int, [_I32, C.c_int64, _D, _I32, C.c_int64, C.POINTER(Options),
                                  C.POINTER(_P)]),
    "dpd_create_tet_mesh": (C.c_int, [_D, C.c_int64, _I32, C.c_int64, _D, _I32, C.c_int64,
                                      C.POINTER(Options), C.POINTER(_P)]),
    "dpd_destroy_mesh": (None, [_P]),
    "dpd_get_info": (C.c_int, [_P, C.POINTER(MeshInfo)]),
    "dpd_node_ijk": (C.c_int, [_P, _I32]),
    "dpd_rest_positions": (C.c_int, [_P, _D]),
    "dpd_contact_nodes": (C.c_int, [_P, _I32]),
    "dpd_set_options": (C.c_int, [_P, C.POINTER(Options)]),
    "dpd_set_youngs": (C.c_int, [_P, _P, C.c_int32, _P]),
    "dpd_factorize": (C.c_int, [_P, _P]),
    "dpd_forward_step": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, C.POINTER(Stats)]),
    "dpd_backward_step": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                    C.POINTER(Stats)]),
    "dpd_apply_inverse": (C.c_int, [_P, _P, C.c_int32, _P, _P]),
    "dpd_gradient": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "dpd_gradient_noalloc": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "dpd_hessian_apply": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "dpd_rotations": (C.c_int, [_P, _P, _P, _P]),
    "dpd_contact_prepare": (C.c_int, [_P, _P, _P, C.c_int32]),
    "dpd_contact_solve": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P]),
    "dpd_contact_forward_step": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, C.POINTER(Stats)]),
    "dpd_contact_backward_step": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                            C.POINTER(Stats)]),
    "dpd_profile_start": (C.c_int, [_P, C.c_int32]),
    "dpd_profile_read": (C.c_int, [_P, _P, C.POINTER(KernelProfile)]),
    "dpd_server_create": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "dpd_server_batch_stats": (C.c_int, [_P, C.POINTER(BatchStats)]),
    "dpd_server_submit": (C.c_int, [_P, C.POINTER(Request), C.POINTER(C.c_int64)]),
    "dpd_server_poll": (C.c_int, [_P, C.c_int64, C.POINTER(Result), _P, _P, _P]),
    "dpd_server_drain": (C.c_int, [_P]),
    "dpd_server_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "dpd_server_destroy": (None, [_P]),
    "dpd_status_string": (C.c_char_p, [C.c_int]),
    "dpd_last_error": (C.c_char_p, [_P]),
}

_lib = None


def load() -> C.CDLL:
    """Load libdiffpd.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class DiffPDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, handle=None) -> int:
    """Raise on hard errors (negative codes); return soft codes."""
    if code < 0:
        lib = load()
        msg = lib.dpd_last_error(handle)
        raise DiffPDError(code, msg.decode() if msg else "")
    return code
