"""ctypes declarations of the aderweno C ABI (include/aderweno.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaderweno.so")

E_ARG = -1
# ADER_STATIC_SCRATCH_BYTES: the fixed device array of ader_adjoint_gts_step_static
STATIC_SCRATCH_BYTES = 256 << 20
E_NAMES = {0: "OK", -1: "E_ARG", -2: "E_MESH", -3: "E_STATE", -4: "E_GEOM", -5: "E_GCL",
           -6: "E_DEADLOCK", -7: "E_HIP", -8: "E_ORDER"}

DBG = dict(Q=0, A=1, XE=2, TICK=3, STEP=4, DTCFL=5, QM=6, HM=7, WNOD=8, AVG=9, TRACE=10,
           VVEL=11, X=12, NTICK=13, SCAL=14,
           TOPO_EDGES=32, TOPO_STENCILS=33, TOPO_SCHED_PTR=34, TOPO_SCHED_IDX=35,
           TOPO_TSTEN_PTR=36, TOPO_TSTEN_IDX=37,
           TAB_DXI=48, TAB_DETA=49, TAB_AMEAN=50, TAB_EDGE=51, TAB_AT=52, TAB_BT=53, TAB_DT=54,
           TAB_PSIC=55, TAB_SIGMA=56, TAB_GAUSS=57)
INT_ARRAYS = {"TICK", "STEP", "NTICK", "TOPO_EDGES", "TOPO_STENCILS", "TOPO_SCHED_PTR",
              "TOPO_SCHED_IDX", "TOPO_TSTEN_PTR", "TOPO_TSTEN_IDX"}

EXPORTED = ["ader_create", "ader_upload_mesh", "ader_workspace_size", "ader_bind_workspace",
            "ader_upload_state", "ader_step_gts", "ader_step_lts", "ader_download_state",
            "ader_get_stats", "ader_debug_size", "ader_debug_dump", "ader_debug_inject",
            "ader_debug_cycles", "ader_debug_macro_begin", "ader_set_profiling", "ader_set_graphs",
            "ader_set_instances", "ader_instance_times", "ader_set_tune", "ader_autotune",
            "ader_kernel_times", "ader_adjoint_workspace_size", "ader_adjoint_gts_step",
            "ader_adjoint_gts_step_static", "ader_set_schedule_replay",
            "ader_adjoint_lagrangian_workspace_size", "ader_adjoint_lagrangian_step", "ader_upload_state_xy",
            "ader_probe_contraction", "ader_adjoint_lts", "ader_set_delta_replay", "ader_set_schedule_record",
            "ader_get_schedule_record",
            "ader_last_error", "ader_destroy"]
KERNELS = ["sched", "node", "patch", "update", "recon", "predict", "macro", "status", "adjoint"]


class AderConfig(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("flux", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("cfl", ctypes.c_double), ("lts_levels", ctypes.c_int32),
                ("n_picard", ctypes.c_int32), ("mesh_velocity", ctypes.c_int32),
                ("weno_eps", ctypes.c_double), ("weno_r", ctypes.c_double),
                ("weno_lambda", ctypes.c_double), ("lts_step_fraction", ctypes.c_double)]


class AderTune(ctypes.Structure):
    _fields_ = [("sched_chunk", ctypes.c_int32), ("list_wg_per_cu", ctypes.c_int32),
                ("ms_per_macro_step", ctypes.c_double), ("sweep_wg_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class AderStats(ctypes.Structure):
    _fields_ = [("element_updates", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("macro_steps", ctypes.c_int64), ("cfl_overshoots", ctypes.c_int64),
                ("max_gcl_residual", ctypes.c_double), ("t", ctypes.c_double),
                ("delta", ctypes.c_double), ("predictor_evals", ctypes.c_int64),
                ("patches", ctypes.c_int64), ("node_moves", ctypes.c_int64),
                ("extra_cycles", ctypes.c_int64), ("long_macro_steps", ctypes.c_int64),
                ("replay_overrides", ctypes.c_int64)]


class AderError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{E_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libaderweno.so (built in-tree by paper_1408_3719_amd.build).  Fails
    loudly when it is missing: there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1408_3719_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, dbl, sz = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    lib.ader_create.argtypes = [ctypes.POINTER(AderConfig), P, ctypes.POINTER(P)]
    lib.ader_upload_mesh.argtypes = [P, i32, P, i32, P, i32, P]
    lib.ader_workspace_size.argtypes = [P, ctypes.POINTER(sz)]
    lib.ader_bind_workspace.argtypes = [P, P, sz]
    lib.ader_upload_state.argtypes = [P, P, dbl]
    lib.ader_step_gts.argtypes = [P, dbl, i32, ctypes.POINTER(AderStats)]
    lib.ader_step_lts.argtypes = [P, dbl, i32, ctypes.POINTER(AderStats)]
    lib.ader_download_state.argtypes = [P, P, P, P]
    lib.ader_get_stats.argtypes = [P, ctypes.POINTER(AderStats)]
    lib.ader_debug_size.argtypes = [P, i32, ctypes.POINTER(sz)]
    lib.ader_debug_dump.argtypes = [P, i32, P, sz]
    lib.ader_debug_inject.argtypes = [P, i32, P, sz]
    lib.ader_debug_cycles.argtypes = [P, i32]
    lib.ader_debug_macro_begin.argtypes = [P, dbl, i32]
    lib.ader_set_profiling.argtypes = [P, i32]
    lib.ader_set_graphs.argtypes = [P, i32]
    lib.ader_set_instances.argtypes = [P, i32, P]
    lib.ader_set_tune.argtypes = [P, ctypes.POINTER(AderTune)]
    lib.ader_autotune.argtypes = [P, i32, ctypes.POINTER(AderTune)]
    lib.ader_instance_times.argtypes = [P, i32, P]
    lib.ader_kernel_times.argtypes = [P, i32, P, P]
    lib.ader_adjoint_workspace_size.argtypes = [P, P]
    lib.ader_adjoint_gts_step.argtypes = [P, dbl, P, P, P, P, ctypes.c_size_t]
    lib.ader_adjoint_gts_step_static.argtypes = [P, dbl, P, P, P]
    lib.ader_adjoint_lagrangian_workspace_size.argtypes = [P, P]
    lib.ader_upload_state_xy.argtypes = [P, P, P, dbl]
    lib.ader_probe_contraction.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P, P, P]
    lib.ader_adjoint_lagrangian_step.argtypes = [P, dbl, P, P, P, P, P, P, P, P, P, ctypes.c_size_t]
    lib.ader_set_schedule_replay.argtypes = [P, P, P, ctypes.c_int64]
    lib.ader_adjoint_lts.argtypes = [P, i32, i32, dbl, P, P, P, P, ctypes.POINTER(i32)]
    lib.ader_set_delta_replay.argtypes = [P, P, i32]
    lib.ader_set_schedule_record.argtypes = [P, i32, i32]
    lib.ader_get_schedule_record.argtypes = [P, P, P, ctypes.c_int64, P, i32, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(i32)]
    lib.ader_last_error.argtypes = [P]
    lib.ader_last_error.restype = ctypes.c_char_p
    lib.ader_destroy.argtypes = [P]
    lib.ader_destroy.restype = None
    for name in EXPORTED:
        if name not in ("ader_last_error", "ader_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib
