"""ctypes view of the C ABI in include/dpba.h (libdpba.so, built for gfx950).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  Importing this module does not load the library; the first call
to `lib()` does, and raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpba.so")

BA_OK, BA_E_INVAL, BA_E_CAPACITY, BA_E_HIP, BA_E_STATE = 0, -1, -2, -3, -4
BA_PREC_FP64, BA_PREC_FP32 = 0, 1
BA_SCHED_AUTO, BA_SCHED_SPLIT, BA_SCHED_FUSED = 0, 1, 2
BA_W_OK, BA_W_NOT_SPD, BA_W_NONFINITE, BA_W_BAD_INDEX, BA_W_DEGREE = 0, 1, 2, 4, 8

EXPORTED = ("ba_create", "ba_solve", "ba_backward", "ba_prepare", "ba_launch", "ba_set_timing",
            "ba_kernel_times", "ba_status", "ba_last_error", "ba_destroy",
            "ba_debug_reduced_system", "ba_debug_mfma", "ba_solve_noalloc",
            "dpc_correlation", "dpc_avg_pool", "dpc_debug_mfma_bf16",
            "dpa_softagg", "dpa_workspace_bytes",
            "vo_create", "vo_set_sensor", "vo_step", "vo_read", "vo_read_events", "vo_read_window", "vo_status", "vo_destroy")
STAGES = ("prep", "assemble", "chol", "backsub", "finalize", "fused")


class BAConfig(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("z_min", ctypes.c_double),
                ("schedule", ctypes.c_int32), ("max_windows", ctypes.c_int32),
                ("max_frames_per_window", ctypes.c_int32), ("chunk_frames", ctypes.c_int32),
                ("max_frames", ctypes.c_int64), ("max_patches", ctypes.c_int64),
                ("max_edges", ctypes.c_int64)]


class BAProblem(ctypes.Structure):
    _fields_ = [("n_windows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("frame_off", ctypes.c_void_p), ("patch_off", ctypes.c_void_p),
                ("edge_off", ctypes.c_void_p), ("n_fixed", ctypes.c_void_p),
                ("intrinsics", ctypes.c_void_p),
                ("poses_in", ctypes.c_void_p), ("patches_in", ctypes.c_void_p),
                ("anchor", ctypes.c_void_p), ("kk", ctypes.c_void_p), ("jj", ctypes.c_void_p),
                ("targets", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("poses_out", ctypes.c_void_p), ("depth_out", ctypes.c_void_p)]


class DPCProblem(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("height0", ctypes.c_int32), ("width0", ctypes.c_int32),
                ("height1", ctypes.c_int32), ("width1", ctypes.c_int32),
                ("scale1", ctypes.c_float), ("patch_pixels", ctypes.c_int32),
                ("n_patches", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("level0", ctypes.c_void_p), ("level1", ctypes.c_void_p), ("gmap", ctypes.c_void_p),
                ("coords", ctypes.c_void_p), ("kk", ctypes.c_void_p), ("jj", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class DPAProblem(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("n_edges", ctypes.c_int64), ("n_patches", ctypes.c_int64),
                ("n_frames", ctypes.c_int32), ("graph_ready", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("kk", ctypes.c_void_p), ("jj", ctypes.c_void_p),
                ("anchor", ctypes.c_void_p), ("w_gate", ctypes.c_void_p), ("b_gate", ctypes.c_void_p),
                ("w_val", ctypes.c_void_p), ("b_val", ctypes.c_void_p), ("w_out", ctypes.c_void_p),
                ("b_out", ctypes.c_void_p), ("out", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_int64), ("status", ctypes.c_void_p)]


class VOConfig(ctypes.Structure):
    _fields_ = [("n_streams", ctypes.c_int32), ("window", ctypes.c_int32),
                ("patches_per_frame", ctypes.c_int32), ("radius", ctypes.c_int32),
                ("n_free", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("iterations", ctypes.c_int32), ("table_radius", ctypes.c_int32),
                ("flow_thresh", ctypes.c_double), ("lambda_", ctypes.c_double), ("z_min", ctypes.c_double),
                ("intrinsics", ctypes.c_double * 4)]


_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises RuntimeError when it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(the solver has no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i32p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)
        L.ba_create.argtypes = [ctypes.POINTER(BAConfig), ctypes.POINTER(vp)]
        L.ba_create.restype = ctypes.c_int
        L.ba_solve.argtypes = [vp, ctypes.POINTER(BAProblem), vp]
        L.ba_solve.restype = ctypes.c_int
        L.ba_backward.argtypes = [vp, ctypes.POINTER(BAProblem), vp, vp, vp, vp, vp]
        L.ba_backward.restype = ctypes.c_int
        L.ba_prepare.argtypes = [vp, ctypes.POINTER(BAProblem), vp]
        L.ba_prepare.restype = ctypes.c_int
        L.ba_launch.argtypes = [vp, vp]
        L.ba_launch.restype = ctypes.c_int
        L.ba_set_timing.argtypes = [vp, i32]
        L.ba_set_timing.restype = ctypes.c_int
        L.ba_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32p]
        L.ba_kernel_times.restype = ctypes.c_int
        L.ba_status.argtypes = [vp, i32p]
        L.ba_status.restype = ctypes.c_int
        L.ba_last_error.argtypes = [vp]
        L.ba_last_error.restype = ctypes.c_char_p
        L.ba_destroy.argtypes = [vp]
        L.ba_destroy.restype = None
        L.ba_debug_reduced_system.argtypes = [vp, ctypes.POINTER(BAProblem), i32, vp, vp, vp]
        L.ba_debug_reduced_system.restype = ctypes.c_int
        L.ba_debug_mfma.argtypes = [i32, vp, vp, vp, vp]
        L.ba_debug_mfma.restype = ctypes.c_int
        L.ba_solve_noalloc.argtypes = [ctypes.POINTER(BAConfig), ctypes.POINTER(BAProblem), vp, vp]
        L.ba_solve_noalloc.restype = ctypes.c_int
        L.dpc_correlation.argtypes = [ctypes.POINTER(DPCProblem), vp]
        L.dpc_correlation.restype = ctypes.c_int
        L.dpc_avg_pool.argtypes = [vp, i32, i32, i32, i32, i32, vp, vp]
        L.dpc_avg_pool.restype = ctypes.c_int
        L.dpc_debug_mfma_bf16.argtypes = [vp, vp, vp, vp]
        L.dpc_debug_mfma_bf16.restype = ctypes.c_int
        L.dpa_softagg.argtypes = [ctypes.POINTER(DPAProblem), vp]
        L.dpa_softagg.restype = ctypes.c_int
        L.dpa_workspace_bytes.argtypes = [i32, i32, ctypes.c_int64, ctypes.c_int64, i32]
        L.dpa_workspace_bytes.restype = ctypes.c_int64
        L.vo_create.argtypes = [ctypes.POINTER(VOConfig), ctypes.POINTER(vp)]
        L.vo_create.restype = ctypes.c_int
        L.vo_set_sensor.argtypes = [vp, vp, vp, vp, vp]
        L.vo_set_sensor.restype = ctypes.c_int
        L.vo_step.argtypes = [vp, vp, vp, vp, vp, vp]
        L.vo_step.restype = ctypes.c_int
        L.vo_read.argtypes = [vp, vp, vp, vp, vp]
        L.vo_read.restype = ctypes.c_int
        L.vo_read_events.argtypes = [vp, vp, vp, vp, vp, vp]
        L.vo_read_events.restype = ctypes.c_int
        L.vo_read_window.argtypes = [vp, i32, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int64)]
        L.vo_read_window.restype = ctypes.c_int
        L.vo_status.argtypes = [vp, vp]
        L.vo_status.restype = ctypes.c_int
        L.vo_destroy.argtypes = [vp]
        L.vo_destroy.restype = None
        _LIB = L
    return _LIB


class BAError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpba error {code}: {msg}")
        self.code = code
