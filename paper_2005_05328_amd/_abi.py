"""ctypes mirror of include/dzs.h and argument marshalling for libdzs.so.

Nothing here computes any part of the gravity step: every call goes through the C ABI into
the HIP kernels.  PyTorch supplies device memory (tensors) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdzs.so")

DZS_OK, DZS_EINVAL, DZS_ENOMEM, DZS_ECAPACITY, DZS_EHIP = 0, -1, -2, -3, -4
DZS_CHEB_MAX = 24
DZS_FP64, DZS_FP32 = 0, 1
DZS_CAP_FP32_MESHES, DZS_CAP_NO_COPIES, DZS_CAP_HIER_SPLIT = 1, 2, 4
DZS_CRIT_GEOMETRIC, DZS_CRIT_DYNAMICAL = 0, 1
DZS_OPEN_GEOMETRIC, DZS_OPEN_RELATIVE = 0, 1

# every entry point include/dzs.h declares
EXPORTS = ("dzs_ctx_create", "dzs_ctx_destroy", "dzs_last_error", "dzs_step_factors",
           "dzs_coarsen", "pm_force", "tree_force", "lightcone_emit", "kdk_step",
           "kdk_step_batch", "kdk_step_batch_stage", "dzs_check", "dzs_morton_keys",
           "dzs_sort_state", "dzs_counters", "dzs_timing", "dzs_halt_check",
           "dzs_forecast_speedup", "kdk_step_hier", "dzs_source_hash", "pm_force_noalloc")
DZS_HIER_MAX_BIN = 6
DZS_HALT_BALANCE, DZS_HALT_RATIO, DZS_HALT_PREDICTED = 1, 2, 4
DZS_BATCH_MAX = 512
DZS_PM_CHUNK_MIN, DZS_PM_CHUNK_MAX, DZS_PM_CHUNK_DEFAULT = 256, 16384, 2048
DZS_PM_NOALLOC_MAX_SIDE = 64


class HierParams(C.Structure):
    _fields_ = [("max_bin", C.c_int32), ("limiter", C.c_int32), ("eta", C.c_double),
                ("R_lim", C.c_double), ("a0", C.c_double), ("a1", C.c_double),
                ("omega_m", C.c_double), ("pm_global", C.c_int32), ("reserved", C.c_int32)]


class HaltParams(C.Structure):
    _fields_ = [("max_balance", C.c_double), ("min_ratio", C.c_double),
                ("runtime_limit_s", C.c_double), ("restart_window_s", C.c_double)]


class HaltState(C.Structure):
    _fields_ = [("balance", C.c_double), ("ratio", C.c_double), ("ratio_prev", C.c_double),
                ("t", C.c_double), ("t_prev", C.c_double)]


class Forecast(C.Structure):
    _fields_ = [("a_dzs", C.c_double), ("r", C.c_double), ("speedup", C.c_double),
                ("particle_mass", C.c_double)]


class Capacity(C.Structure):
    _fields_ = [("max_particles", C.c_uint64), ("max_mesh_side", C.c_uint32),
                ("flags", C.c_uint32), ("max_boxes", C.c_uint32), ("reserved", C.c_uint32)]


class Box(C.Structure):
    _fields_ = [("L", C.c_double), ("m0", C.c_double), ("eps0", C.c_double), ("G", C.c_double)]


class Particles(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "px", "py", "pz", "gx", "gy", "gz",
                                          "mult", "id", "type")] + \
               [("n", C.c_uint64), ("capacity", C.c_uint64)]


class CoarsenParams(C.Structure):
    _fields_ = [("x_obs", C.c_double * 3), ("R_lc", C.c_double), ("b", C.c_double),
                ("theta", C.c_double), ("k_min", C.c_int32), ("criterion", C.c_int32),
                ("alpha_dyn", C.c_double)]


class CoarsenReport(C.Structure):
    _fields_ = [("n_before", C.c_uint64), ("n_after", C.c_uint64), ("n_groups", C.c_uint64),
                ("a_min", C.c_double)]


class PMParams(C.Structure):
    _fields_ = [("ng", C.c_int32), ("precision", C.c_int32), ("r_s", C.c_double),
                ("accumulate", C.c_int32), ("tile_chunk", C.c_int32)]


class TreeParams(C.Structure):
    _fields_ = [("r_s", C.c_double), ("r_cut", C.c_double), ("theta", C.c_double),
                ("leaf_size", C.c_int32), ("group_size", C.c_int32), ("precision", C.c_int32),
                ("accumulate", C.c_int32), ("opening", C.c_int32), ("presorted", C.c_int32),
                ("alpha_open", C.c_double)]


class LCParams(C.Structure):
    _fields_ = [("x_obs", C.c_double * 3), ("a0", C.c_double), ("a1", C.c_double),
                ("D", C.c_double), ("chi2_0", C.c_double), ("chi2_1", C.c_double),
                ("n_cheb", C.c_int32), ("reserved", C.c_int32),
                ("cheb_chi", C.c_double * DZS_CHEB_MAX), ("cheb_drift", C.c_double * DZS_CHEB_MAX)]


class LCRecord(C.Structure):
    _fields_ = [("id", C.c_uint32), ("mult", C.c_uint32), ("a_cross", C.c_double),
                ("d", C.c_double * 3), ("p", C.c_double * 3)]


class LCRing(C.Structure):
    _fields_ = [("records", C.c_void_p), ("capacity", C.c_uint64), ("count", C.c_void_p),
                ("overflow", C.c_void_p)]


class StepParams(C.Structure):
    _fields_ = [("K1", C.c_double), ("K2", C.c_double), ("lc", LCParams),
                ("do_lightcone", C.c_int32), ("do_coarsen", C.c_int32),
                ("coarsen", CoarsenParams), ("pm", PMParams), ("tree", TreeParams)]


class Batch(C.Structure):
    _fields_ = [("n_boxes", C.c_uint32), ("reserved", C.c_uint32), ("boxes", C.POINTER(Box)),
                ("first", C.POINTER(C.c_uint64)), ("ng", C.POINTER(C.c_int32)),
                ("r_s", C.POINTER(C.c_double)), ("r_cut", C.POINTER(C.c_double))]


assert C.sizeof(LCRecord) == 64


def _source_hash():
    """The build script's hash of the sources in this tree (None if the script is absent)."""
    import importlib.util
    path = os.path.join(HERE, "build.py")
    if not os.path.exists(path):
        return None
    spec = importlib.util.spec_from_file_location("_dzs_build_hash", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.source_hash()


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libdzs.so not found at {LIB_PATH}: build it with "
                          "`python paper_2005_05328_amd/build.py` (the GPU path has no fallback)")
    # torch ships its own HIP runtime under the same soname as /opt/rocm's; the first one loaded
    # serves the whole process, so torch is imported before the library resolves its runtime
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    L.dzs_source_hash.argtypes = []
    L.dzs_source_hash.restype = C.c_char_p
    built = L.dzs_source_hash().decode()
    want = _source_hash()
    if want is not None and built != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (hash {built}, sources "
                          f"{want}): rebuild it with `python paper_2005_05328_amd/build.py`")
    P, i32, st = C.c_void_p, C.c_int32, C.c_int32
    L.dzs_ctx_create.argtypes = [C.POINTER(P), i32, C.POINTER(Capacity)]
    L.dzs_ctx_destroy.argtypes = [P]
    L.dzs_last_error.argtypes = [P]
    L.dzs_last_error.restype = C.c_char_p
    L.dzs_step_factors.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(StepParams)]
    L.kdk_step_hier.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(StepParams),
                                C.POINTER(HierParams), C.POINTER(LCRing),
                                C.POINTER(CoarsenReport), P, P]
    L.dzs_halt_check.argtypes = [C.POINTER(HaltParams), C.POINTER(HaltState)]
    L.dzs_halt_check.restype = C.c_uint32
    L.dzs_forecast_speedup.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(Forecast)]
    L.dzs_coarsen.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(CoarsenParams),
                              P, C.POINTER(CoarsenReport), P]
    L.pm_force.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(PMParams), P]
    L.pm_force_noalloc.argtypes = [C.POINTER(Box), C.POINTER(Particles), C.POINTER(PMParams), P]
    L.pm_force_noalloc.restype = st
    L.tree_force.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(TreeParams), P,
                             C.c_uint64, P]
    L.lightcone_emit.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(LCParams),
                                 C.POINTER(LCRing), P]
    L.kdk_step.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), C.POINTER(StepParams),
                           C.POINTER(LCRing), C.POINTER(CoarsenReport), P]
    L.kdk_step_batch.argtypes = [P, C.POINTER(Batch), C.POINTER(Particles), C.POINTER(StepParams),
                                 C.POINTER(LCRing), P]
    L.kdk_step_batch_stage.argtypes = [P, C.POINTER(StepParams)]
    L.dzs_check.argtypes = [P, P]
    L.dzs_morton_keys.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), P, P]
    L.dzs_sort_state.argtypes = [P, C.POINTER(Box), C.POINTER(Particles), i32, P, P]
    L.dzs_counters.argtypes = [P, i32, C.POINTER(C.c_uint64)]
    L.dzs_timing.argtypes = [P, i32, i32, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                             C.POINTER(C.c_uint64), i32]
    for name in ("dzs_ctx_create", "dzs_ctx_destroy", "dzs_step_factors", "dzs_coarsen",
                 "pm_force", "tree_force", "lightcone_emit", "kdk_step", "kdk_step_batch",
                 "kdk_step_batch_stage", "dzs_check", "dzs_morton_keys",
                 "dzs_sort_state", "dzs_counters", "dzs_timing", "dzs_forecast_speedup",
                 "kdk_step_hier"):
        getattr(L, name).restype = st
    return L
