"""ctypes declarations of the C ABI in include/tamm_mi.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtamm_mi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tamm_mi.h")

c_int, c_i32, c_i64, c_dbl, c_vp, c_char_p, c_size_t = (ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                        ctypes.c_void_p, ctypes.c_char_p, ctypes.c_size_t)
P = ctypes.POINTER

NONZERO_FN = ctypes.CFUNCTYPE(c_int, P(ctypes.c_int32), P(ctypes.c_int8), c_i32, c_vp)


class PlanStats(ctypes.Structure):
    _fields_ = [
        ("out_blocks", c_i64),
        ("candidates", c_i64),
        ("tasks", c_i64),
        ("dropped", c_i64),
        ("useful_flops", c_dbl),
        ("algorithmic_bytes", c_dbl),
        ("work_items", c_i64),
        ("kernel_config", c_i32),
        ("k_splits", c_i32),
        ("gather_layout", c_i32),
        ("xcd_chunk", c_i32),
        ("tile_order", c_i32),
        ("reserved", c_i32),
    ]


SIGNATURES = {
    "tamm_last_error": (c_char_p, []),
    "tamm_version": (c_i32, []),
    "tamm_space_create": (c_int, [P(c_i64), P(ctypes.c_int8), c_i32, P(c_vp)]),
    "tamm_space_create_fixed": (c_int, [c_i64, c_i64, P(c_vp)]),
    "tamm_space_create_spin": (c_int, [c_i64, c_i64, c_i64, P(c_vp)]),
    "tamm_space_info": (c_int, [c_vp, P(c_i32), P(c_i64)]),
    "tamm_space_tiles": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "tamm_space_destroy": (c_int, [c_vp]),
    "tamm_tensor_create": (c_int, [P(c_vp), c_i32, c_vp, c_vp, P(c_vp)]),
    "tamm_tensor_numel": (c_int, [c_vp, P(c_i64)]),
    "tamm_tensor_nbytes": (c_int, [c_vp, P(c_size_t)]),
    "tamm_tensor_blocks": (c_int, [c_vp, P(c_i64), c_vp, c_vp]),
    "tamm_tensor_bind": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_tensor_destroy": (c_int, [c_vp]),
    "tamm_plan_create": (c_int, [c_vp, c_char_p, c_vp, c_char_p, c_vp, c_char_p, c_int, P(c_vp)]),
    "tamm_plan_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_plan_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_plan_stats_get": (c_int, [c_vp, P(PlanStats)]),
    "tamm_plan_config_count": (c_int, [c_vp, P(c_i32)]),
    "tamm_plan_set_config": (c_int, [c_vp, c_i32, c_i32]),
    "tamm_plan_set_order": (c_int, [c_vp, c_i32, c_i32]),
    "tamm_plan_set_constant": (c_int, [c_vp, c_i32, c_i32]),
    "tamm_config_name": (c_char_p, [c_i32, c_i32]),
    "tamm_plan_autotune_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_plan_autotune": (c_int, [c_vp, c_vp, c_size_t, c_vp, c_char_p, c_i32]),
    "tamm_plan_execute": (c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    "tamm_plan_screen": (c_int, [c_vp, c_vp]),
    "tamm_plan_contract": (c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    "tamm_plan_screen_result": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "tamm_plan_split_operand": (c_int, [c_vp, c_i32, c_vp, c_size_t, c_vp]),
    "tamm_plan_destroy": (c_int, [c_vp]),
    "tamm_contract_workspace_size": (c_int, [c_vp, c_char_p, c_vp, c_char_p, c_vp, c_char_p, c_i32, P(c_size_t)]),
    "tamm_contract": (c_int, [c_vp, c_char_p, c_vp, c_char_p, c_vp, c_char_p, c_i32, c_dbl, c_dbl, c_vp, c_size_t, c_vp]),
    "tamm_contract_cache_count": (c_int, [P(c_i64)]),
    "tamm_contract_cache_clear": (c_int, []),
    "tamm_contract_noalloc": (c_int, [c_vp, c_char_p, c_vp, c_char_p, c_vp, c_char_p, c_i32, c_dbl, c_dbl, c_vp]),
    "tamm_group_create": (c_int, [P(c_vp), c_i32, P(c_vp)]),
    "tamm_group_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_group_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_group_set_config": (c_int, [c_vp, c_i32, c_i32]),
    "tamm_group_execute": (c_int, [c_vp, P(c_dbl), P(c_dbl), c_vp]),
    "tamm_group_capture": (c_int, [c_vp, P(c_dbl), P(c_dbl), c_vp]),
    "tamm_group_autotune": (c_int, [c_vp, c_vp, c_char_p, c_i32]),
    "tamm_group_stats": (c_int, [c_vp, P(c_i32), P(c_i32), P(c_i64)]),
    "tamm_group_destroy": (c_int, [c_vp]),
    "tamm_denominator_create": (c_int, [c_vp, c_vp, P(ctypes.c_int8), P(c_vp)]),
    "tamm_denominator_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_denominator_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_denominator_execute": (c_int, [c_vp, P(c_vp), c_vp]),
    "tamm_denominator_destroy": (c_int, [c_vp]),
    "tamm_set": (c_int, [c_vp, c_dbl, c_vp]),
    "tamm_add_create": (c_int, [c_vp, c_char_p, c_vp, c_char_p, P(c_vp)]),
    "tamm_add_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_add_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_add_execute": (c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    "tamm_add_destroy": (c_int, [c_vp]),
    "tamm_diag_mfma": (c_int, [c_i32, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "tamm_sched_create": (c_int, [P(c_vp)]),
    "tamm_sched_set": (c_int, [c_vp, c_vp, c_dbl]),
    "tamm_sched_add": (c_int, [c_vp, c_vp, c_dbl, c_dbl]),
    "tamm_sched_contract": (c_int, [c_vp, c_vp, c_dbl, c_dbl]),
    "tamm_sched_denominator": (c_int, [c_vp, c_vp, P(c_vp)]),
    "tamm_sched_build": (c_int, [c_vp]),
    "tamm_sched_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_sched_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_sched_autotune": (c_int, [c_vp, c_vp, c_char_p, c_i32]),
    "tamm_sched_execute": (c_int, [c_vp, c_vp]),
    "tamm_sched_capture": (c_int, [c_vp, c_vp]),
    "tamm_sched_info": (c_int, [c_vp, P(c_i32), P(c_i32), P(c_i32)]),
    "tamm_sched_op_info": (c_int, [c_vp, c_i32, P(c_i32), P(c_i32)]),
    "tamm_sched_destroy": (c_int, [c_vp]),
    "tamm_tensor_view_rows": (c_int, [c_vp, c_i32, c_i32, P(c_vp), P(c_i64)]),
    "tamm_chol_ladder_create": (c_int, [c_vp, c_vp, c_vp, c_i32, P(c_vp)]),
    "tamm_chol_ladder_workspace_size": (c_int, [c_vp, P(c_size_t)]),
    "tamm_chol_ladder_bind_workspace": (c_int, [c_vp, c_vp, c_size_t]),
    "tamm_chol_ladder_execute": (c_int, [c_vp, c_dbl, c_dbl, c_vp]),
    "tamm_chol_ladder_autotune": (c_int, [c_vp, c_vp, c_char_p, c_i32]),
    "tamm_chol_ladder_stats": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_i64), P(c_i64), P(c_i64)]),
    "tamm_chol_ladder_strip_plans": (c_int, [c_vp, c_i32, P(c_vp), P(c_vp)]),
    "tamm_chol_ladder_destroy": (c_int, [c_vp]),
}

NOALLOC_WORKSPACE_BYTES = 64 << 20  # TAMM_NOALLOC_WORKSPACE_BYTES of the header

STATUS = {
    0: "TAMM_OK",
    -1: "TAMM_ERR_ARG",
    -2: "TAMM_ERR_LABEL",
    -3: "TAMM_ERR_SHAPE",
    -4: "TAMM_ERR_SPARSITY",
    -5: "TAMM_ERR_UNSUPPORTED",
    -6: "TAMM_ERR_UNBOUND",
    -7: "TAMM_ERR_WORKSPACE",
    -8: "TAMM_ERR_HIP",
}


class TammError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS.get(code, code)}: {message}")
        self.code = code
        self.status = STATUS.get(code, str(code))


_lib = None


def header_functions():
    """Names of the functions declared in include/tamm_mi.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tamm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def load():
    """Load the HIP library (the in-tree build, or the file named by TAMM_MI_LIBRARY); raise if it
    does not exist (there is no fallback)."""
    global _lib
    if _lib is None:
        path = os.environ.get("TAMM_MI_LIBRARY") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(
                f"{path} is missing: build the HIP library first (python -m paper_2201_01257_amd.build)")
        # The library resolves libamdhip64.so.7 by soname.  torch ships its own HIP runtime under
        # that soname; loading torch first makes both use that single runtime instead of two.
        try:
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover - C-only use without torch
            pass
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def check(code: int):
    if code != 0:
        msg = load().tamm_last_error()
        raise TammError(code, msg.decode() if msg else "")
