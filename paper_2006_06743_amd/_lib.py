"""ctypes view of libsng.so (the C ABI declared in include/sng.h).

Loading fails loudly when the HIP library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsng.so")

SNG_OK, SNG_EINVAL, SNG_ERANGE, SNG_EWORKSPACE, SNG_EHIP, SNG_EOVERFLOW, SNG_ENOTIMPL, SNG_EIO = \
    0, -1, -2, -3, -4, -5, -6, -7
SNG_FP32, SNG_BF16, SNG_FP16 = 0, 1, 2
SNG_SIM_DOT, SNG_SIM_COSINE = 1, 2
SNG_WS_DIRECT, SNG_WS_SIMPLE_GRAPH = 0x100, 0x200

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = [
    "sng_status_string", "sng_samples_per_point", "sng_workspace_size", "sng_degrees",
    "sng_cluster", "sng_dbscan", "sng_dbscan_lowp", "sng_graph_workspace_size", "sng_graph_labels",
    "sng_compact_labels", "sng_sample", "sng_autotune", "sng_autotune_lookup",
    "sng_autotune_clear", "sng_autotune_lowp", "sng_autotune_hook", "sng_autotune_batch",
    "sng_autotune_save", "sng_autotune_load",
    "sng_sweep_workspace_size", "sng_dbscan_sweep", "sng_batch_workspace_size",
    "sng_dbscan_batch", "sng_batch_plan_create", "sng_batch_plan_launch",
    "sng_batch_plan_destroy", "sng_stats_read",
    "sng_similarity_workspace_size", "sng_dbscan_similarity", "sng_dbscan_noalloc",
]


class sng_config(ctypes.Structure):
    _fields_ = [("lanes_per_pair", ctypes.c_int32), ("chunks_per_wave", ctypes.c_int32),
                ("stage_lds", ctypes.c_int32), ("prefetch", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("reuse_sample", ctypes.c_int32),
                ("out_degree", ctypes.c_int32), ("simple_graph", ctypes.c_int32),
                ("mfma_waves", ctypes.c_int32), ("mfma_ksteps", ctypes.c_int32),
                ("hook_blocks", ctypes.c_int32)]


class sng_stats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint64), ("self_pairs", ctypes.c_uint64),
                ("accepted", ctypes.c_uint64), ("rechecked", ctypes.c_uint64),
                ("n_core", ctypes.c_uint64), ("n_clusters", ctypes.c_uint64),
                ("n_noise", ctypes.c_uint64), ("overflow", ctypes.c_uint64),
                ("band_rel", ctypes.c_double), ("filter_gamma", ctypes.c_double),
                ("filter_r_max", ctypes.c_double), ("filter_r_mean", ctypes.c_double),
                ("filter_rel_width", ctypes.c_double)]


class SNGError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, status_string(code), code))


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsng.so is not built (run __graft_entry__.build() or "
                          "python paper_2006_06743_amd/build.py); no fallback exists")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u64, dbl, f32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_uint64, ctypes.c_double, ctypes.c_float)
    sz = ctypes.c_size_t
    cfgp = ctypes.POINTER(sng_config)
    sig = {
        "sng_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "sng_samples_per_point": ([dbl, i64, ctypes.POINTER(i64)], ctypes.c_int),
        "sng_workspace_size": ([i64, i32, i64, i32, ctypes.POINTER(sz)], ctypes.c_int),
        "sng_degrees": ([P, i64, i32, i64, i64, dbl, u64, P, P, sz, cfgp, P], ctypes.c_int),
        "sng_cluster": ([P, i64, i32, i64, i64, dbl, u64, i32, P, P, P, sz, P], ctypes.c_int),
        "sng_dbscan": ([P, i64, i32, i64, dbl, dbl, i32, u64, P, P, P, sz, cfgp, P],
                       ctypes.c_int),
        "sng_dbscan_noalloc": ([P, i64, i32, i64, dbl, dbl, i32, u64, P, P, cfgp, P],
                               ctypes.c_int),
        "sng_dbscan_lowp": ([P, i64, i32, i64, P, i64, f32, i32, dbl, dbl, i32, u64, P, P, P,
                             sz, cfgp, P], ctypes.c_int),
        "sng_similarity_workspace_size": ([i64, i32, i64, i32, i32, ctypes.POINTER(sz)],
                                          ctypes.c_int),
        "sng_dbscan_similarity": ([P, i64, i32, i64, dbl, i32, dbl, i32, u64, P, P, P, sz, cfgp,
                                   P], ctypes.c_int),
        "sng_graph_workspace_size": ([i64, ctypes.POINTER(sz)], ctypes.c_int),
        "sng_graph_labels": ([i64, P, i64, i32, P, P, P, sz, P], ctypes.c_int),
        "sng_compact_labels": ([P, i64, P, P, P], ctypes.c_int),
        "sng_sample": ([i64, i32, i64, u64, P, sz, P], ctypes.c_int),
        "sng_autotune": ([P, i64, i32, i64, i64, dbl, u64, P, sz, i32, cfgp, P, P, P],
                         ctypes.c_int),
        "sng_autotune_lookup": ([P, i64, i32, i64, i64, cfgp], ctypes.c_int),
        "sng_autotune_clear": ([], ctypes.c_int),
        "sng_autotune_lowp": ([P, i64, i32, i64, P, i64, f32, i32, dbl, dbl, i32, u64, P, P, P,
                               sz, i32, cfgp, P, P, P], ctypes.c_int),
        "sng_autotune_hook": ([P, i64, i32, i64, i64, dbl, u64, i32, P, P, P, sz, i32, cfgp, P,
                               P, P], ctypes.c_int),
        "sng_autotune_batch": ([i32, P, P, i32, P, P, P, P, P, P, P, P, sz, i32, cfgp, P, P, P],
                               ctypes.c_int),
        "sng_autotune_save": ([ctypes.c_char_p], ctypes.c_int),
        "sng_autotune_load": ([ctypes.c_char_p], ctypes.c_int),
        "sng_sweep_workspace_size": ([i64, i32, i64, i32, i32, ctypes.POINTER(sz)],
                                     ctypes.c_int),
        "sng_dbscan_sweep": ([P, i64, i32, i64, dbl, P, i32, P, i32, u64, P, P, P, sz, cfgp, P],
                             ctypes.c_int),
        "sng_batch_workspace_size": ([i32, P, i32, P, ctypes.POINTER(sz)], ctypes.c_int),
        "sng_dbscan_batch": ([i32, P, P, i32, P, P, P, P, P, P, P, P, sz, P], ctypes.c_int),
        "sng_batch_plan_create": ([i32, P, P, i32, P, P, P, P, P, P, P, P, sz, P,
                                   ctypes.POINTER(P)], ctypes.c_int),
        "sng_batch_plan_launch": ([P, P], ctypes.c_int),
        "sng_batch_plan_destroy": ([P], ctypes.c_int),
        "sng_stats_read": ([P, i32, ctypes.POINTER(sng_stats), P], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load().sng_status_string(int(code)).decode()
    except ImportError:
        return "status %d" % code


def check(code: int, what: str):
    if code != SNG_OK:
        raise SNGError(code, what)
