"""ctypes declarations of include/qgm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqgm.so")


class QgmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qgm status {status}: {msg}")
        self.status = status


STATUS = {0: "QGM_OK", -1: "QGM_E_ARG", -2: "QGM_E_PARSE", -3: "QGM_E_ORDER", -4: "QGM_E_SLICE",
          -5: "QGM_E_WORKSPACE", -6: "QGM_E_HIP", -7: "QGM_E_UNSUPPORTED"}


class VarInfo(C.Structure):
    _fields_ = [("id", C.c_int32), ("qubit", C.c_int32), ("cycle_created", C.c_int32), ("is_output", C.c_int32)]


class PlanOpts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("profile", C.c_int32), ("workspace_cap", C.c_size_t),
                ("engine", C.c_int32), ("gradient", C.c_int32), ("waves", C.c_int32),
                ("vector_only", C.c_int32), ("checkpoint_every", C.c_int32), ("persistent", C.c_int32),
                ("deterministic", C.c_int32), ("n_open", C.c_int32), ("tile_table_path", C.c_char_p),
                ("open_qubits", C.POINTER(C.c_int32))]


class Tile(C.Structure):
    _fields_ = [("per", C.c_int32), ("lds_budget", C.c_int32), ("jband", C.c_int32), ("layout", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_steps", C.c_int32), ("n_const_steps", C.c_int32), ("max_rank", C.c_int32),
                ("item_elems", C.c_int32), ("n_leaves", C.c_int32), ("k", C.c_int32),
                ("flops_item", C.c_double), ("flops_const", C.c_double), ("bytes_item", C.c_double),
                ("cost", C.c_double), ("engine", C.c_int32), ("waves", C.c_int32), ("compile_s", C.c_double),
                ("launches", C.c_int32), ("mfma_steps", C.c_int32), ("flops_mfma", C.c_double),
                ("roof_s_item", C.c_double), ("n_open", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1805_01450_amd/build.py` "
                          "(there is no fallback implementation)")
    try:
        import torch  # noqa: F401  (loads the HIP runtime the library is linked against)
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32, u64, sz, dbl = C.c_int32, C.c_uint64, C.c_size_t, C.c_double
    pi32 = C.POINTER(C.c_int32)
    pd = C.POINTER(C.c_double)
    pu8 = C.POINTER(C.c_uint8)
    sig = {
        "qgm_circuit_parse": (i32, [C.c_char_p, sz, C.POINTER(P)]),
        "qgm_circuit_info": (i32, [P, pi32, pi32, pi32]),
        "qgm_circuit_vars": (i32, [P, C.POINTER(VarInfo), i32]),
        "qgm_circuit_graph": (i32, [P, pi32, i32, pi32]),
        "qgm_circuit_free": (None, [P]),
        "qgm_plan_slices": (i32, [P, i32, i32, dbl, u64, pi32, pi32, pi32, pi32]),
        "qgm_plan_slices_ex": (i32, [P, i32, i32, dbl, u64, i32, pi32, pi32, pi32, pi32]),
        "qgm_order_cost": (i32, [P, pi32, i32, pi32, i32, pd, pi32]),
        "qgm_sliced_order_for_groups": (i32, [P, pi32, i32, pi32, i32, pi32, pd]),
        "qgm_order_search": (i32, [P, pi32, i32, pi32, i32, C.c_int64, i32, pi32, pd, pi32, pi32]),
        "qgm_plan_create": (i32, [P, pi32, i32, pi32, i32, C.POINTER(PlanOpts), C.POINTER(P)]),
        "qgm_plan_stats": (i32, [P, C.POINTER(Stats)]),
        "qgm_workspace_size": (i32, [P, i32, u64, C.POINTER(sz)]),
        "qgm_amplitudes": (i32, [P, pu8, i32, pd, P, sz, P, pd]),
        "qgm_amplitudes_range": (i32, [P, pu8, i32, pd, u64, u64, P, sz, P, pd]),
        "qgm_amplitudes_device": (i32, [P, P, i32, P, u64, u64, P, sz, P, P]),
        "qgm_plan_timing": (i32, [P, i32, pd, pi32]),
        "qgm_plan_level_timing": (i32, [P, i32, pd, pd, pd, pi32, i32, pi32, pi32, C.POINTER(u64), pd]),
        "qgm_plan_autotune": (i32, [P, i32, u64, P, sz, P, pi32]),
        "qgm_gradients_device": (i32, [P, P, i32, P, u64, u64, P, sz, P, P, P]),
        "qgm_amplitude_grad": (i32, [P, pu8, pd, P, sz, P, pd, pd]),
        "qgm_graph_create": (i32, [P, P, i32, P, u64, u64, P, sz, P, i32, C.POINTER(P)]),
        "qgm_graph_launch": (i32, [P, P]),
        "qgm_graph_free": (None, [P]),
        "qgm_plan_free": (None, [P]),
        "qgm_last_error": (C.c_char_p, []),
        "qgm_amplitude": (i32, [C.c_char_p, sz, pu8, pi32, i32, pi32, i32, pd, pd]),
        "qgm_amplitudes_device_noalloc": (i32, [P, P, i32, P, u64, u64, P, P]),
        "qgm_contraction_create": (i32, [i32, i32, i32, i32, i32, i32, C.POINTER(Tile), C.POINTER(P)]),
        "qgm_plan_tune_tiles": (i32, [P, C.c_char_p, P, pi32]),
        "qgm_contraction_info": (i32, [P, pi32, C.POINTER(u64), pd]),
        "qgm_contraction_run": (i32, [P, P, C.c_int64, P]),
        "qgm_contraction_free": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()
DECLARED = ("qgm_circuit_parse", "qgm_circuit_info", "qgm_circuit_vars", "qgm_circuit_graph", "qgm_circuit_free",
            "qgm_plan_slices", "qgm_plan_slices_ex", "qgm_order_cost", "qgm_sliced_order_for_groups", "qgm_order_search", "qgm_plan_create", "qgm_plan_stats", "qgm_workspace_size",
            "qgm_amplitudes", "qgm_amplitudes_range", "qgm_amplitudes_device", "qgm_amplitudes_device_noalloc",
            "qgm_gradients_device", "qgm_amplitude_grad", "qgm_graph_create", "qgm_graph_launch", "qgm_graph_free",
            "qgm_plan_timing", "qgm_plan_level_timing", "qgm_plan_autotune", "qgm_plan_free",
            "qgm_last_error", "qgm_amplitude", "qgm_contraction_create", "qgm_contraction_info",
            "qgm_contraction_run", "qgm_contraction_free", "qgm_plan_tune_tiles")


def check(status: int) -> None:
    if status != 0:
        msg = lib.qgm_last_error()
        raise QgmError(status, f"{STATUS.get(status, '?')}: {msg.decode() if msg else ''}")
