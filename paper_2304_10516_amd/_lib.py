"""ctypes declarations of the C ABI in include/dvnr.h (argument marshalling only).

Loading fails loudly when libdvnr.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvnr.so")

DVNR_OK, DVNR_E_INVALID, DVNR_E_UNSUPPORTED, DVNR_E_HIP, DVNR_E_STATE, DVNR_E_NONFINITE = range(6)
DVNR_FP32, DVNR_MIXED_BF16, DVNR_FP64 = 0, 1, 2


class Encoding(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_features", C.c_int32), ("log2_table_size", C.c_int32),
                ("base_resolution", C.c_int32), ("per_level_scale", C.c_double), ("finest_resolution", C.c_int32)]


class Mlp(C.Structure):
    _fields_ = [("n_hidden_layers", C.c_int32), ("width", C.c_int32), ("out_dim", C.c_int32)]


class Optim(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("weight_decay", C.c_double), ("lr_decay_base", C.c_double), ("lr_decay_start", C.c_int64),
                ("lr_decay_interval", C.c_int64)]


class Block(C.Structure):
    _fields_ = [("dims", C.c_int32 * 3), ("ghost", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("n_levels", C.c_int64), ("n_entries", C.c_int64), ("n_table_params", C.c_int64),
                ("n_mlp_params", C.c_int64), ("block_stride", C.c_int64), ("n_params", C.c_int64),
                ("param_bytes", C.c_int64), ("work16_bytes", C.c_int64), ("workspace_bytes", C.c_int64)]


class Buffers(C.Structure):
    _fields_ = [("params", C.c_void_p), ("grads", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("work16", C.c_void_p), ("workspace", C.c_void_p), ("volumes", C.POINTER(C.c_void_p))]


class StopPolicy(C.Structure):
    _fields_ = [("min_steps", C.c_int64), ("epochs", C.c_int64), ("loss_threshold", C.c_double),
                ("window", C.c_int32), ("check_every", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("center", C.c_float * 3), ("up", C.c_float * 3), ("fovy_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class RenderParams(C.Structure):
    _fields_ = [("step", C.c_float), ("ref_step", C.c_float), ("alpha_stop", C.c_float), ("tf_lo", C.c_float),
                ("tf_hi", C.c_float), ("n_tf", C.c_int32), ("samples_per_round", C.c_int32)]


class DvnrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dvnr error {code}: {msg}")
        self.code = code


_lib = None

P, I32, I64, U64, VP = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_void_p
FP = C.POINTER(C.c_float)

SIGNATURES = {
    "dvnr_create": [C.POINTER(Encoding), C.POINTER(Mlp), C.POINTER(Optim), I32, I32, C.POINTER(Block), I64, U64,
                    C.POINTER(P)],
    "dvnr_destroy": [P],
    "dvnr_get_sizes": [P, C.POINTER(Sizes)],
    "dvnr_level_info": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "dvnr_bind": [P, C.POINTER(Buffers)],
    "dvnr_prepare": [P, VP],
    "dvnr_get_ranges": [P, FP, FP, VP],
    "dvnr_init_params": [P, U64, VP],
    "dvnr_params_updated": [P, VP],
    "dvnr_reset_optimizer": [P, VP],
    "dvnr_train_steps": [P, I32, I64, VP, VP],
    "dvnr_train_step_coords": [P, VP, C.POINTER(C.c_int64), VP, VP],
    "dvnr_draw_training_samples": [P, I32, I64, I64, VP, VP, VP],
    "dvnr_sample": [P, I32, I64, VP, VP, VP],
    "dvnr_decode": [P, I32, VP, VP],
    "dvnr_mse_fp64": [P, I32, VP, C.POINTER(C.c_double), C.POINTER(C.c_int64), VP],
    "dvnr_encode_forward": [P, I32, I64, VP, VP, VP, VP],
    "dvnr_encode_backward": [P, I32, I64, VP, VP, VP, VP],
    "dvnr_mlp_forward": [P, I32, I64, VP, VP, VP, VP],
    "dvnr_mlp_backward": [P, I32, I64, VP, VP, VP, VP, VP, VP],
    "dvnr_adam_step": [P, VP],
    "dvnr_debug_indices": [P, I32, I64, VP, VP, VP, VP],
    "dvnr_sync": [P, VP],
    "dvnr_set_option": [P, C.c_char_p, I64],
    "dvnr_set_loss": [P, I32, C.c_double, C.c_double],
    "dvnr_cache_snapshot_bytes": [P, C.POINTER(C.c_int64)],
    "dvnr_render_workspace_bytes": [P, I32, I32, C.POINTER(C.c_int64)],
    "dvnr_render": [P, I32, C.POINTER(Camera), C.POINTER(RenderParams), VP, VP, VP, C.POINTER(C.c_int64), VP],
    "dvnr_render_static": [P, I32, C.POINTER(Camera), C.POINTER(RenderParams), VP, VP, C.POINTER(C.c_int64), VP],
    "dvnr_cache_bind": [P, I32, VP],
    "dvnr_cache_push": [P, I64, VP],
    "dvnr_cache_keys": [P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)],
    "dvnr_cache_decode": [P, I64, I32, VP, VP],
    "dvnr_cache_sample": [P, I64, I32, I64, VP, VP, VP],
    "dvnr_train_until": [P, C.POINTER(StopPolicy), I64, C.POINTER(C.c_int64), C.POINTER(C.c_double), VP],
    "dvnr_phase_times": [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "dvnr_plan_info": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "dvnr_plan_partition": [P, C.POINTER(C.c_int32)],
    "dvnr_autotune": [P, I64, I32, C.POINTER(C.c_double), VP],
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2304_10516_amd.build_lib` "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None if name == "dvnr_destroy" else C.c_int32
        L.dvnr_last_error.argtypes = []
        L.dvnr_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def check(code: int):
    if code != DVNR_OK:
        msg = lib().dvnr_last_error()
        raise DvnrError(code, msg.decode() if msg else "")
