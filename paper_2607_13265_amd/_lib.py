"""ctypes binding of the C ABI declared in include/ppt.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppt.so")

PPT_OK = 0
ERRORS = {-1: "PPT_EINVAL", -2: "PPT_ENOMEM", -3: "PPT_EDEVICE", -4: "PPT_EUNSUPPORTED"}

# every entry point of include/ppt.h: name -> (restype, argtypes)
_vp, _i32, _i64, _u32, _u64, _sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_uint64, ctypes.c_size_t)
SIGNATURES = {
    "ppt_scene_create": (_i32, [_vp, _sz, _vp]),
    "ppt_scene_destroy": (None, [_vp]),
    "ppt_scene_slots": (_i32, [_vp, _vp, _vp, _i32]),
    "ppt_plan_create": (_i32, [_vp, _vp, _i32, _i32, _u32, _vp, _vp]),
    "ppt_plan_destroy": (None, [_vp]),
    "ppt_plan_image_numel": (_i64, [_vp]),
    "ppt_plan_num_paths": (_i64, [_vp]),
    "ppt_plan_workspace_bytes": (_sz, [_vp, _i32]),
    "ppt_plan_set_path_mask": (_i32, [_vp, _vp]),
    "ppt_plan_set_stats": (_i32, [_vp, _i32]),
    "ppt_plan_set_timing": (_i32, [_vp, _i32]),
    "ppt_plan_kernel_times": (_i32, [_vp, _i32, _vp, _vp, _i32]),
    "ppt_render": (_i32, [_vp, _vp, _i32, _u64, _vp, _vp, _sz, _vp]),
    "ppt_backward": (_i32, [_vp, _vp, _i32, _u64, _vp, _vp, _vp, _sz, _vp]),
    "ppt_backward_noalloc": (_i32, [_vp, _vp, _i32, _u64, _vp, _vp, _vp]),
    "ppt_signatures": (_i32, [_vp, _vp, _i32, _u64, _vp, _vp, _sz, _vp]),
    "ppt_read_stats": (_i32, [_vp, _vp, _vp]),
    "ppt_read_hybrid_stats": (_i32, [_vp, _vp, _vp]),
    "ppt_debug_rng": (_i32, [_u64, _vp, _vp, _i64, _vp]),
    "ppt_plan_launch_info": (_i32, [_vp, _vp, _vp, _vp]),
    "ppt_last_error": (ctypes.c_char_p, []),
}


class PPTError(RuntimeError):
    pass


class PlanOpts(ctypes.Structure):
    _fields_ = [("chunk_paths", ctypes.c_int64), ("checkpoint_interval", ctypes.c_int64),
                ("hybrid_rule", ctypes.c_int32), ("hybrid_gamma", ctypes.c_float), ("hybrid_eps", ctypes.c_float),
                ("adjoint", ctypes.c_int32), ("pprb_sigma", ctypes.c_float)]


_lib = None


def lib():
    """Load the in-tree HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PPTError(f"{LIB_PATH} is missing: build it with paper_2607_13265_amd.build.build() "
                           "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != PPT_OK:
        msg = lib().ppt_last_error()
        raise PPTError(f"{ERRORS.get(rc, rc)}: {msg.decode() if msg else ''}")
    return rc


def ptr_table(tensors):
    """Host array of device pointers (None -> NULL)."""
    t = (ctypes.c_void_p * max(len(tensors), 1))()
    for i, x in enumerate(tensors):
        t[i] = None if x is None else x.data_ptr()
    return t
