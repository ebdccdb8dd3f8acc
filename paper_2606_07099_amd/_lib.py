"""ctypes declarations of the C ABI in ``include/sable_pf.h``.

Argument marshalling only: every step of the power-flow path runs in the HIP
library.  Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# SABLE_PHASE_CLOCKS=1 selects the measurement build with per-phase clocks
LIB_PATH = os.path.join(HERE, "libsablepf_phases.so" if os.environ.get("SABLE_PHASE_CLOCKS") == "1"
                        else "libsablepf.so")

PF_OK, PF_EINVAL, PF_ETOPOLOGY, PF_ENOMEM, PF_EHIP, PF_ESTATE = 0, -1, -2, -3, -4, -5
PF_BUS_PQ, PF_BUS_PV, PF_BUS_SLACK = 0, 1, 2
PF_FP64, PF_MIXED = 0, 1
PF_STATUS_CONVERGED, PF_STATUS_MAX_ITER, PF_STATUS_NON_FINITE, PF_STATUS_ZERO_PIVOT = 0, 1, 2, 3
PF_EVAL_MISMATCH, PF_EVAL_JACOBIAN, PF_EVAL_STEP, PF_EVAL_ADJOINT, PF_EVAL_FILL = 0, 1, 2, 3, 4
PF_OP_BASE, PF_OP_J1, PF_OP_J1T, PF_OP_J2T, PF_OP_J3T = 0, 1, 2, 3, 4

EXPORTED = ("pf_default_options", "pf_last_error", "pf_ybus_from_branches", "pf_template_build",
            "pf_template_info", "pf_template_destroy", "pf_symbolic_analyze", "pf_solve_batch",
            "pf_adjoint_batch", "pf_eval_batch", "pf_recover_batch", "pf_adjoint_completed_batch",
            "pf_operator_pattern", "pf_operator_values", "pf_operator_bde_csr", "pf_template_block_pattern",
            "pf_operator_values_static", "pf_debug_phase_clocks")


class PFOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("keep_factors", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("refine_adaptive", ctypes.c_int32)]


class PFStats(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_pv", ctypes.c_int32), ("n_pq", ctypes.c_int32),
                ("n_j", ctypes.c_int32), ("nnz_ybus", ctypes.c_int32), ("nnz_j1", ctypes.c_int64),
                ("n_blocks", ctypes.c_int32), ("nnzb_lu", ctypes.c_int32), ("nnz_lu", ctypes.c_int64),
                ("n_block_updates", ctypes.c_int64), ("n_levels_l", ctypes.c_int32),
                ("n_levels_u", ctypes.c_int32), ("max_row_blocks", ctypes.c_int32),
                ("fill_ratio", ctypes.c_double), ("factor_flops", ctypes.c_double),
                ("workspace_bytes", ctypes.c_size_t), ("batch", ctypes.c_int32),
                ("lds_resident", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("slice_width", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class PFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run python -m paper_2606_07099_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    L.pf_default_options.argtypes = [ctypes.POINTER(PFOptions)]
    L.pf_default_options.restype = None
    L.pf_last_error.argtypes = []
    L.pf_last_error.restype = ctypes.c_char_p
    L.pf_ybus_from_branches.argtypes = [ctypes.c_int32, ctypes.c_int32, _I32P, _I32P, _F64P, _F64P,
                                        _F64P, _I32P, _I32P, _F64P, _F64P, ctypes.c_int32, _I32P]
    L.pf_template_build.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P, _F64P, _F64P,
                                    ctypes.c_int32, ctypes.POINTER(PFOptions), ctypes.POINTER(_P)]
    L.pf_template_info.argtypes = [_P, ctypes.POINTER(PFStats)]
    L.pf_template_destroy.argtypes = [_P]
    L.pf_symbolic_analyze.argtypes = [ctypes.c_int32, _I32P, _I32P, _I32P,
                                      ctypes.POINTER(PFStats), _I32P]
    L.pf_solve_batch.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.pf_adjoint_batch.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P]
    L.pf_eval_batch.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P]
    L.pf_operator_bde_csr.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]
    L.pf_template_block_pattern.argtypes = [_P, _I32P, _I32P]
    L.pf_debug_phase_clocks.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_double)]
    for name in EXPORTED[2:]:
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(rc: int):
    if rc != PF_OK:
        raise PFError(rc, lib().pf_last_error().decode())
