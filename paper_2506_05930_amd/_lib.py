"""ctypes view of libnvc.so: the structs, status codes and raw entry points of include/nvc.h.

Loading fails loudly when the library has not been built; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_float, c_int32, c_int64, c_uint32, c_uint64, c_void_p, c_char_p, POINTER

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnvc.so")

NVC_OK = 0
NVC_ERR_NULL = -1
NVC_ERR_SHAPE = -2
NVC_ERR_DTYPE = -3
NVC_ERR_UNSUPPORTED = -4
NVC_ERR_HIP = -5
NVC_ERR_WORKSPACE = -6

NVC_F32, NVC_F16, NVC_BF16 = 0, 1, 2
NVC_ACT_RELU, NVC_ACT_LEAKY = 0, 1
NVC_LOSS_BCE, NVC_LOSS_L2 = 0, 1
NVC_SELECT_PIXELS_NOALLOC_MAX_PIX = 1 << 23
NVC_TRAIN_SHADOW_MAX_LIGHTS = 32
NVC_TRAIN_SHADOW_MAX_SPHERES = 512

EXPORTS = [
    "nvc_version", "nvc_status_string", "nvc_grid_levels", "nvc_mlp_param_count", "nvc_mlp_packed_bytes",
    "nvc_pack_mlp", "nvc_encode", "nvc_infer", "nvc_mlp_forward", "nvc_sample_wrs", "nvc_select_pixels_workspace_bytes",
    "nvc_select_pixels", "nvc_shadow_labels",
    "nvc_train_workspace_bytes", "nvc_train_step", "nvc_adam", "nvc_counters_advance",
    "nvc_cluster_lights", "nvc_shadow_labels_clustered", "nvc_sample_clustered", "nvc_world_samples",
    "nvc_graph_begin", "nvc_graph_end", "nvc_graph_launch", "nvc_graph_destroy", "nvc_select_pixels_noalloc",
    "nvc_forward_f64", "nvc_train_step_shadow", "nvc_train_plan_bytes", "nvc_train_plan",
    "nvc_train_step_planned",
]


class NvcGrid(ctypes.Structure):
    _fields_ = [("n_levels", c_int32), ("n_feat", c_int32), ("log2_T", c_int32), ("base_res", c_int32),
                ("growth", c_double)]


class NvcMlp(ctypes.Structure):
    _fields_ = [("n_in", c_int32), ("width", c_int32), ("n_hidden", c_int32), ("n_out", c_int32),
                ("act", c_int32), ("leaky_slope", c_float), ("dtype", c_int32)]


class NvcError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


_SIGS = {
    "nvc_version": (c_int32, []),
    "nvc_status_string": (c_char_p, [c_int32]),
    "nvc_grid_levels": (c_int32, [POINTER(NvcGrid), c_void_p, c_void_p]),
    "nvc_mlp_param_count": (c_int64, [POINTER(NvcMlp)]),
    "nvc_mlp_packed_bytes": (c_int64, [POINTER(NvcMlp)]),
    "nvc_pack_mlp": (c_int32, [POINTER(NvcMlp), c_void_p, c_void_p, c_void_p]),
    "nvc_encode": (c_int32, [POINTER(NvcGrid), c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p]),
    "nvc_infer": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                            c_int32, c_void_p]),
    "nvc_mlp_forward": (c_int32, [POINTER(NvcMlp), c_void_p, c_void_p, c_int32, c_int64, c_void_p, c_int32, c_void_p]),
    "nvc_sample_wrs": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_float,
                                 c_uint64, c_uint32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p]),
    "nvc_select_pixels_workspace_bytes": (c_int64, [c_int64]),
    "nvc_select_pixels": (c_int32, [c_uint64, c_uint32, c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_int64,
                                    c_void_p]),
    "nvc_select_pixels_noalloc": (c_int32, [c_uint64, c_uint32, c_void_p, c_int64, c_int64, c_void_p, c_void_p]),
    "nvc_shadow_labels": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_int32, c_void_p,
                                    c_void_p]),
    "nvc_train_workspace_bytes": (c_int64, [POINTER(NvcGrid), POINTER(NvcMlp), c_int64]),
    "nvc_train_step": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                 c_void_p, c_void_p, c_int32, c_float, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int64, c_void_p]),
    "nvc_train_plan_bytes": (c_int64, [POINTER(NvcGrid), POINTER(NvcMlp), c_int64]),
    "nvc_train_plan": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_int64, c_void_p, c_int64,
                                 c_void_p]),
    "nvc_train_step_planned": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_int64, c_void_p, c_void_p, c_int32, c_float, c_void_p, c_void_p, c_void_p,
                                         c_void_p, c_int64, c_void_p, c_int64, c_void_p]),
    "nvc_train_step_shadow": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_int32, c_int32, c_float,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_void_p]),
    "nvc_adam": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int32, c_void_p, c_float, c_float,
                           c_int32, c_float, c_float, c_float, c_int32, c_void_p]),
    "nvc_counters_advance": (c_int32, [c_void_p, c_void_p]),
    "nvc_graph_begin": (c_int32, [c_void_p]),
    "nvc_graph_end": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "nvc_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "nvc_graph_destroy": (c_int32, [c_void_p]),
    "nvc_forward_f64": (c_int32, [POINTER(NvcGrid), POINTER(NvcMlp), c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                                  c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nvc_world_samples": (c_int32, [c_uint64, c_uint32, c_void_p, c_int64, c_void_p, c_float, c_void_p, c_void_p,
                                    c_void_p]),
    "nvc_cluster_lights": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "nvc_shadow_labels_clustered": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p,
                                              c_int32, c_void_p, c_int32, c_uint64, c_uint32, c_void_p, c_void_p,
                                              c_void_p]),
    "nvc_sample_clustered": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32,
                                       c_void_p, c_void_p, c_float, c_int32, c_uint64, c_uint32, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libnvc.so once; raise if it is missing (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes libnvc.so bind to that runtime, so the streams
    # and device pointers torch hands over belong to the runtime that launches
    # the kernels.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() or "
                           "python paper_2506_05930_amd/build.py first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().nvc_status_string(status).decode()


def check(fn: str, status: int) -> int:
    if status < 0:
        raise NvcError(fn, status, status_string(status))
    return status
