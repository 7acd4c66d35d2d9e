"""ctypes binding of libmpgbs.so (include/mpgbs.h): argument marshalling only.

The library is loaded from this package directory; there is no fallback of any
kind, so a missing or unloadable library raises at import of the binding."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpgbs.so")

MP_OK, MP_ERR_ARG, MP_ERR_SHAPE, MP_ERR_HIP, MP_ERR_UNSUPPORTED, MP_ERR_WORKSPACE = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "split_bf16": 2, "split_fp16": 3, "split1_fp16": 4,
              "split1t_fp16": 5, "split1t_f8": 6}
BIN_MODES = {"joint": 0, "marginals": 1, "marginals_and_total": 2}
ESTIMATORS = {"matrix_p": 0, "plus_p": 1}
MP_MAX_BINS = 8
MP_MAX_RUNS = 16
MP_MAX_MOMENTS = 8
MP_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTS = [
    "mp_ld_modes", "mp_ab_bytes", "mp_c_bytes", "mp_sample", "mp_propagate_workspace",
    "mp_propagate", "mp_pack_transmission", "mp_propagate_packed", "mp_occupations",
    "mp_moments_accumulate", "mp_observable_histogram", "mp_subensemble_stats", "mp_acc_entries",
    "mp_mode_occupations_bytes", "mp_mode_occupations", "mp_pair_correlations_accumulate",
    "mp_check_finite", "mp_pair_correlations_workspace",
    "mp_binned_workspace", "mp_binned_counts", "mp_propagate_counts_workspace",
    "mp_propagate_counts", "mp_propagate_counts_noalloc", "mp_bilinear_workspace",
    "mp_bilinear_packed_bytes",
    "mp_pack_bilinear", "mp_propagate_counts_bilinear", "mp_counts_finalize", "mp_finalize_workspace", "mp_last_error", "mp_version",
    "mp_mfma_sustained", "mp_plan_create", "mp_plan_launch", "mp_plan_result", "mp_plan_info", "mp_plan_tile",
    "mp_plan_destroy",
    "mp_mlp_param_count", "mp_mlp_workspace", "mp_mlp_round", "mp_mlp_forward", "mp_mlp_loss_grad",
    "mp_mlp_adam",
]

MP_MLP_MAX_LAYERS = 8


class MlpShape(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("width", ctypes.c_int32 * (MP_MLP_MAX_LAYERS + 1))]


class NetDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("T", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("net", ctypes.c_uint32), ("E", ctypes.c_int64),
                ("n_sub", ctypes.c_int32), ("m_lo", ctypes.c_int32), ("K", ctypes.c_int32),
                ("d", ctypes.c_int32), ("mode", ctypes.c_int), ("bin_of_mode", ctypes.c_void_p),
                ("m_lo_b", ctypes.c_void_p), ("K_b", ctypes.c_void_p)]


class MPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libmpgbs status {status}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Loads the library once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2503_12749_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    c_i32, c_i64, c_u64, c_u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    i32p = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "mp_ld_modes": (c_i64, [c_i32]),
        "mp_ab_bytes": (sz, [c_i32, c_i64, ctypes.c_int]),
        "mp_c_bytes": (sz, [c_i32, c_i64, ctypes.c_int]),
        "mp_sample": (ctypes.c_int, [c_i32, c_i64, c_i64, vp, c_u64, c_u32, ctypes.c_int, vp, vp, vp]),
        "mp_propagate_workspace": (sz, [c_i32, ctypes.c_int]),
        "mp_propagate": (ctypes.c_int, [c_i32, c_i64, vp, ctypes.c_int, vp, vp, vp, sz, vp]),
        "mp_pack_transmission": (ctypes.c_int, [c_i32, vp, ctypes.c_int, vp, sz, vp]),
        "mp_propagate_packed": (ctypes.c_int, [c_i32, c_i64, ctypes.c_int, vp, vp, vp, sz, vp]),
        "mp_propagate_counts_workspace": (sz, [c_i32, c_i64, c_i32, vp, ctypes.c_int, vp, c_i32,
                                                c_i64, c_i64]),
        "mp_propagate_counts": (ctypes.c_int, [c_i32, c_i64, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                               sz, c_i32, vp, ctypes.c_int, vp, vp, c_i32, c_i64,
                                               c_i64, vp, vp, sz, vp]),
        "mp_bilinear_workspace": (sz, [c_i32]),
        "mp_bilinear_packed_bytes": (sz, [c_i32]),
        "mp_pack_bilinear": (ctypes.c_int, [c_i32, vp, vp, ctypes.c_int, vp, sz, vp, sz, vp]),
        "mp_propagate_counts_bilinear": (ctypes.c_int, [c_i32, c_i64, ctypes.c_int, ctypes.c_int,
                                                        vp, vp, vp, sz, vp, vp, c_i32, c_i64,
                                                        c_i64, vp, vp, sz, vp]),
        "mp_propagate_counts_noalloc": (ctypes.c_int, [c_i32, c_i64, ctypes.c_int, ctypes.c_int, vp,
                                                       vp, vp, sz, c_i32, vp, ctypes.c_int, vp, vp,
                                                       c_i32, c_i64, c_i64, vp, vp]),
        "mp_occupations": (ctypes.c_int, [c_i32, c_i64, vp, ctypes.c_int, c_i32, vp, ctypes.c_int,
                                          vp, vp]),
        "mp_moments_accumulate": (ctypes.c_int, [c_i64, vp, vp, c_i32, c_i32, ctypes.c_int, c_i32,
                                                 c_i64, c_i64, vp, vp]),
        "mp_observable_histogram": (ctypes.c_int, [c_i64, vp, vp, c_i32, c_i32, c_i32, ctypes.c_int,
                                                   ctypes.c_double, ctypes.c_double, c_i32, c_i32,
                                                   c_i64, c_i64, vp, vp]),
        "mp_subensemble_stats": (ctypes.c_int, [c_i32, c_i64, c_i64, c_i32, ctypes.c_double, vp, vp,
                                                vp, vp]),
        "mp_acc_entries": (c_i64, [c_i32, ctypes.c_int, i32p]),
        "mp_check_finite": (ctypes.c_int, [vp, c_i64, vp, ctypes.POINTER(c_i64), vp]),
        "mp_mode_occupations_bytes": (sz, [c_i32, c_i64, ctypes.c_int]),
        "mp_mode_occupations": (ctypes.c_int, [c_i32, c_i64, vp, ctypes.c_int, vp, vp]),
        "mp_pair_correlations_workspace": (sz, [c_i32, c_i64, ctypes.c_int, c_i64, c_i64]),
        "mp_pair_correlations_accumulate": (ctypes.c_int, [c_i32, c_i64, vp, ctypes.c_int, c_i32,
                                                           c_i64, c_i64, vp, vp, sz, vp]),
        "mp_binned_workspace": (sz, [c_i32, ctypes.c_int, i32p, c_i64, c_i32, c_i64, c_i64]),
        "mp_binned_counts": (ctypes.c_int, [c_i32, c_i64, vp, vp, ctypes.c_int, ctypes.c_int, c_i32,
                                            i32p, ctypes.c_int, i32p, i32p, c_i32, c_i64, c_i64,
                                            vp, vp, sz, vp]),
        "mp_finalize_workspace": (sz, [c_i32, ctypes.c_int, i32p, c_i32]),
        "mp_counts_finalize": (ctypes.c_int, [c_i32, ctypes.c_int, i32p, c_i32, c_i64, vp, vp, vp,
                                              vp, vp, sz, vp]),
        "mp_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), c_i32,
                                          ctypes.POINTER(NetDesc), ctypes.c_int, ctypes.c_int, c_i64,
                                          ctypes.c_char_p]),
        "mp_plan_launch": (ctypes.c_int, [vp, vp]),
        "mp_plan_result": (ctypes.c_int, [vp, c_i32, ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p)]),
        "mp_plan_info": (ctypes.c_int, [vp, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(sz)]),
        "mp_plan_tile": (ctypes.c_int, [vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32)]),
        "mp_mfma_sustained": (ctypes.c_int, [c_i32, c_i64, vp, sz, ctypes.POINTER(ctypes.c_double), vp]),
        "mp_plan_destroy": (ctypes.c_int, [vp]),
        "mp_mlp_param_count": (c_i64, [ctypes.POINTER(MlpShape)]),
        "mp_mlp_workspace": (sz, [ctypes.POINTER(MlpShape), c_i32]),
        "mp_mlp_round": (ctypes.c_int, [ctypes.POINTER(MlpShape), vp, vp, vp]),
        "mp_mlp_forward": (ctypes.c_int, [ctypes.POINTER(MlpShape), vp, vp, vp, c_i32, vp, vp, sz, vp]),
        "mp_mlp_loss_grad": (ctypes.c_int, [ctypes.POINTER(MlpShape), vp, vp, vp, vp, c_i32, vp, vp,
                                            vp, sz, vp]),
        "mp_mlp_adam": (ctypes.c_int, [ctypes.POINTER(MlpShape), vp, vp, vp, vp, vp, ctypes.c_float,
                                       ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       c_i32, vp]),
        "mp_last_error": (ctypes.c_char_p, []),
        "mp_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != MP_OK:
        raise MPError(status, load().mp_last_error().decode())


def i32_array(values) -> ctypes.Array:
    vals = [int(v) for v in values]
    return (ctypes.c_int32 * max(1, len(vals)))(*vals)
