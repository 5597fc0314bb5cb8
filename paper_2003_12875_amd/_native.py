"""ctypes declarations mirroring include/nll.h."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnllmi.so")

MAX_OBS, MAX_PARAMS, MAX_NODES, MAX_NODE_PARAMS, MAX_NODE_CHILDREN = 4, 32, 16, 12, 8

STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported model shape", -3: "parameter out of range",
          -4: "event outside observable range", -5: "invalid density", -6: "device error",
          -7: "out of device memory", -8: "call out of order", -9: "request larger than the fixed scratch array"}

# every entry point declared in include/nll.h
EXPORTS = ("nll_create_model", "nll_destroy_model", "nll_set_stream", "nll_set_data", "nll_set_weights", "nll_eval",
           "nll_eval_grad", "nll_eval_batched", "nll_eval_batched_noalloc", "nll_eval_points", "nll_fit_batched", "nll_fit", "nll_eval_bhhh",
           "nll_fit_bhhh", "nll_sync", "nll_get_schedule",
           "nll_set_schedule", "nll_autotune", "nll_set_option", "nll_step_times", "nll_get_info", "nll_read_probe",
           "nll_status_string", "nll_hf_create", "nll_hf_destroy", "nll_hf_set_data", "nll_hf_eval", "nll_hf_sync",
           "nll_hf_set_staterror", "nll_hf_set_shapesys", "nll_hf_eval_stat",
           "nll_jit_create", "nll_jit_destroy", "nll_jit_set_data", "nll_jit_eval", "nll_jit_sync")

HF_MAX_SAMPLES, HF_MAX_HISTOSYS = 8, 24
HF_MODIFIER = {"normfactor": 1, "normsys": 2, "histosys": 3}


class NLLError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({status})" if where else STATUS.get(status, str(status)))


class NodeDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("obs", ctypes.c_int32), ("n_param", ctypes.c_int32),
                ("param", ctypes.c_int32 * MAX_NODE_PARAMS), ("n_child", ctypes.c_int32),
                ("child", ctypes.c_int32 * MAX_NODE_CHILDREN), ("norm", ctypes.c_int32),
                ("density", ctypes.c_char_p)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_obs", ctypes.c_int32), ("obs_lo", ctypes.POINTER(ctypes.c_double)),
                ("obs_hi", ctypes.POINTER(ctypes.c_double)), ("n_param", ctypes.c_int32),
                ("param_lo", ctypes.POINTER(ctypes.c_double)), ("param_hi", ctypes.POINTER(ctypes.c_double)),
                ("param_free", ctypes.POINTER(ctypes.c_uint8)), ("n_node", ctypes.c_int32),
                ("nodes", ctypes.POINTER(NodeDesc)), ("root", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("extended", ctypes.c_int32), ("yield_param", ctypes.c_int32), ("device", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class HFModifier(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("sample", ctypes.c_int32), ("param", ctypes.c_int32),
                ("interp", ctypes.c_int32), ("hi", ctypes.c_double), ("lo", ctypes.c_double)]


class HFDesc(ctypes.Structure):
    _fields_ = [("n_bins", ctypes.c_int64), ("n_samples", ctypes.c_int32), ("n_param", ctypes.c_int32),
                ("param_lo", ctypes.POINTER(ctypes.c_double)), ("param_hi", ctypes.POINTER(ctypes.c_double)),
                ("param_free", ctypes.POINTER(ctypes.c_uint8)), ("param_constrained", ctypes.POINTER(ctypes.c_uint8)),
                ("param_mean", ctypes.POINTER(ctypes.c_double)), ("param_sigma", ctypes.POINTER(ctypes.c_double)),
                ("n_modifiers", ctypes.c_int32), ("modifiers", ctypes.POINTER(HFModifier)),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class JitDesc(ctypes.Structure):
    _fields_ = [("density", ctypes.c_char_p), ("obs_lo", ctypes.c_double), ("obs_hi", ctypes.c_double),
                ("n_param", ctypes.c_int32), ("param_lo", ctypes.POINTER(ctypes.c_double)),
                ("param_hi", ctypes.POINTER(ctypes.c_double)), ("param_free", ctypes.POINTER(ctypes.c_uint8)),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("unroll", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("tile_events", ctypes.c_int32),
                ("sets_blocks_per_cu", ctypes.c_int32), ("sets_unroll", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_char * 64), ("n_leaf", ctypes.c_int32), ("n_term", ctypes.c_int32),
                ("n_accumulators", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_cu", ctypes.c_int32),
                ("n_events", ctypes.c_int64), ("per_set_bytes", ctypes.c_int32)]


_lib = None


def lib():
    """The HIP library.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2003_12875_amd.build` "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.nll_create_model.argtypes = [ctypes.POINTER(ModelDesc), ctypes.POINTER(vp)]
        L.nll_destroy_model.argtypes = [vp]
        L.nll_destroy_model.restype = None
        L.nll_set_stream.argtypes = [vp, vp]
        L.nll_set_data.argtypes = [vp, ctypes.POINTER(vp), i64]
        L.nll_set_weights.argtypes = [vp, vp]
        L.nll_eval.argtypes = [vp, vp, vp]
        L.nll_eval_grad.argtypes = [vp, vp, vp, vp]
        L.nll_eval_batched.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.nll_eval_batched_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.nll_eval_points.argtypes = [vp, i32, vp, vp, vp, vp]
        L.nll_fit_batched.argtypes = [vp, i32, vp, vp, i32, d, vp, vp, vp]
        L.nll_fit.argtypes = [vp, vp, i32, d, vp, vp, vp]
        L.nll_eval_bhhh.argtypes = [vp, vp, vp, vp, vp]
        L.nll_fit_bhhh.argtypes = [vp, vp, i32, d, vp, vp, vp]
        L.nll_sync.argtypes = [vp, ctypes.POINTER(i32)]
        L.nll_get_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.nll_set_schedule.argtypes = [vp, ctypes.POINTER(Schedule)]
        L.nll_autotune.argtypes = [vp, i32, i32, vp, vp]
        L.nll_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.nll_read_probe.argtypes = [vp, i64, vp, i32, vp]
        L.nll_set_option.argtypes = [vp, i32, i32]
        L.nll_step_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)]
        L.nll_status_string.argtypes = [i32]
        L.nll_status_string.restype = ctypes.c_char_p
        L.nll_hf_create.argtypes = [ctypes.POINTER(HFDesc), ctypes.POINTER(vp)]
        L.nll_hf_destroy.argtypes = [vp]
        L.nll_hf_destroy.restype = None
        L.nll_hf_set_data.argtypes = [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.nll_hf_eval.argtypes = [vp, vp, vp, vp]
        L.nll_hf_set_staterror.argtypes = [vp, ctypes.c_uint32, vp]
        L.nll_hf_set_shapesys.argtypes = [vp, ctypes.c_uint32, vp]
        L.nll_hf_eval_stat.argtypes = [vp, vp, vp, vp, vp, vp]
        L.nll_hf_sync.argtypes = [vp, ctypes.POINTER(i32)]
        L.nll_jit_create.argtypes = [ctypes.POINTER(JitDesc), ctypes.POINTER(vp), ctypes.c_char_p, i32]
        L.nll_jit_destroy.argtypes = [vp]
        L.nll_jit_destroy.restype = None
        L.nll_jit_set_data.argtypes = [vp, vp, i64]
        L.nll_jit_eval.argtypes = [vp, vp, vp, vp]
        L.nll_jit_sync.argtypes = [vp, ctypes.POINTER(i32)]
        for f in EXPORTS:
            if f not in ("nll_destroy_model", "nll_status_string", "nll_hf_destroy", "nll_jit_destroy"):
                getattr(L, f).restype = ctypes.c_int32
        _lib = L
    return _lib


def check(status: int, where: str = ""):
    if status != 0:
        raise NLLError(status, where)
    return status
