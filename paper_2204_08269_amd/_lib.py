"""ctypes binding of libjtfs.so (the C ABI declared in include/jtfs.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Importing this module does not touch the GPU; loading the library
fails loudly if it has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjtfs.so")

JTFS_OK = 0
JTFS_EINVAL = -1
JTFS_ENOMEM = -2
JTFS_EHIP = -3
JTFS_EWORKSPACE = -4
JTFS_ESHAPE = -5
JTFS_ENOTSUP = -6
JTFS_BWD_REUSE_FORWARD = 1
JTFS_NOALLOC_SCRATCH_BYTES = 256 << 20
JTFS_NO_FREQ_AVERAGE = 1
JTFS_TIME_SCATTERING = 2
JTFS_LOWPASS_PAIRS = 4
JTFS_UNPAD_LAMBDA = 8
JTFS_BUCKET_AUTOTUNE = 0x100
JTFS_CONTRACTION_FP32 = 0
JTFS_CONTRACTION_SPLIT_F16 = 1
JTFS_CONTRACTION_SPLIT_F16_PHASE = 2
CONTRACTIONS = {"fp32": JTFS_CONTRACTION_FP32, "split16": JTFS_CONTRACTION_SPLIT_F16,
                "split16_phase": JTFS_CONTRACTION_SPLIT_F16_PHASE}
STAGES = ["input_fft", "scalogram", "s1", "second_order", "operand_split", "freq_fwd", "freq_lowpass",
          "lowpass_adj", "freq_adj_pq", "freq_adj_wh", "second_adj_fft", "second_adj", "first_adj", "band_accum",
          "output_fft"]


class Tuning(ctypes.Structure):
    _fields_ = [("contraction", ctypes.c_int32), ("reg_rows", ctypes.c_int32), ("step_ms", ctypes.c_double),
                ("candidates_ms", ctypes.c_double * 6), ("fwd_ms", ctypes.c_double * 2),
                ("bwd_ms", ctypes.c_double * 2), ("from_cache", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("J", ctypes.c_int32), ("Q1", ctypes.c_int32), ("Q2", ctypes.c_int32),
                ("J_fr", ctypes.c_int32), ("Q_fr", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("T", ctypes.c_int64), ("F", ctypes.c_int64)]


class Info(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int32), ("n_alpha", ctypes.c_int32), ("n_beta", ctypes.c_int32),
                ("L", ctypes.c_int32), ("kX", ctypes.c_int32), ("M_h", ctypes.c_int32),
                ("NX", ctypes.c_int64), ("out_t", ctypes.c_int64), ("out_l", ctypes.c_int64),
                ("sum_T", ctypes.c_int64), ("s1_per_signal", ctypes.c_int64), ("s2_per_signal", ctypes.c_int64),
                ("ws_fwd", ctypes.c_int64), ("ws_bwd", ctypes.c_int64)]


EXPORTS = ["jtfs_query", "jtfs_query_filters", "jtfs_plan_create", "jtfs_plan_create_ex", "jtfs_plan_info",
           "jtfs_plan_destroy", "jtfs_workspace_size", "jtfs_forward_workspace_size", "jtfs_forward", "jtfs_backward", "jtfs_plan_table",
           "jtfs_plan_set_contraction", "jtfs_plan_get_contraction", "jtfs_bucket_create", "jtfs_bucket_offsets",
           "jtfs_bucket_run", "jtfs_bucket_destroy", "jtfs_path_means", "jtfs_mulog", "jtfs_mulog_backward",
           "jtfs_forward_mulog", "jtfs_backward_mulog",
           "jtfs_zeroth_order", "jtfs_zeroth_order_backward", "jtfs_plan_tables",
           "jtfs_texture_create", "jtfs_texture_set_target", "jtfs_texture_set_start", "jtfs_texture_iterate",
           "jtfs_texture_read", "jtfs_texture_destroy", "jtfs_plan_autotune", "jtfs_plan_set_tuning",
           "jtfs_plan_get_tuning", "jtfs_forward_noalloc",
           "jtfs_timing_enable", "jtfs_timing_read", "jtfs_last_error"]

_lib = None


class JTFSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libjtfs error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libjtfs.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2204_08269_amd.build` "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(path)
    vp, i64, i32, u32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    P = ctypes.POINTER
    L.jtfs_query.argtypes = [P(Params), P(Info)]
    L.jtfs_query_filters.argtypes = [P(Params), ctypes.c_int, i32, P(ctypes.c_double), P(ctypes.c_double),
                                     P(i32), P(i32)]
    L.jtfs_plan_create.argtypes = [P(vp), i64, ctypes.c_int, P(ctypes.c_int), ctypes.c_int, ctypes.c_int, i64, i64]
    L.jtfs_plan_create_ex.argtypes = [P(vp), P(Params)]
    L.jtfs_plan_info.argtypes = [vp, P(Info)]
    L.jtfs_plan_destroy.argtypes = [vp]
    L.jtfs_plan_destroy.restype = None
    L.jtfs_workspace_size.argtypes = [vp, i64, P(sz)]
    L.jtfs_forward_workspace_size.argtypes = [vp, i64, P(sz)]
    L.jtfs_forward.argtypes = [vp, vp, i64, vp, vp, vp, sz, vp]
    L.jtfs_forward_noalloc.argtypes = [vp, vp, i64, vp, vp, vp]
    L.jtfs_backward.argtypes = [vp, vp, vp, vp, vp, i64, vp, sz, u32, vp]
    L.jtfs_plan_table.argtypes = [vp, ctypes.c_int, vp, sz]
    L.jtfs_plan_set_contraction.argtypes = [vp, ctypes.c_int]
    L.jtfs_plan_get_contraction.argtypes = [vp, P(ctypes.c_int)]
    L.jtfs_bucket_create.argtypes = [P(vp), P(i64), ctypes.c_int, P(Params)]
    L.jtfs_bucket_offsets.argtypes = [vp, P(i64), P(i64)]
    L.jtfs_bucket_run.argtypes = [vp, vp, vp, vp, vp, vp]
    L.jtfs_bucket_destroy.argtypes = [vp]
    L.jtfs_bucket_destroy.restype = None
    L.jtfs_path_means.argtypes = [vp, vp, vp, i64, vp, vp, vp]
    L.jtfs_mulog.argtypes = [vp, vp, vp, i64, vp, vp, ctypes.c_float, vp, vp, vp]
    L.jtfs_mulog_backward.argtypes = [vp, vp, vp, i64, vp, vp, ctypes.c_float, vp, vp, vp, vp, vp]
    L.jtfs_plan_tables.argtypes = [vp, vp, vp]
    L.jtfs_zeroth_order.argtypes = [vp, vp, i64, vp, vp]
    L.jtfs_zeroth_order_backward.argtypes = [vp, vp, i64, vp, vp]
    L.jtfs_forward_mulog.argtypes = [vp, vp, i64, vp, vp, ctypes.c_float, vp, vp, vp, sz, vp]
    L.jtfs_backward_mulog.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.c_float, vp, vp, vp, i64, vp, sz, u32, vp]
    L.jtfs_plan_autotune.argtypes = [vp, vp, i64, ctypes.c_int, vp, P(Tuning)]
    L.jtfs_plan_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.jtfs_plan_get_tuning.argtypes = [vp, P(ctypes.c_int), P(ctypes.c_int)]
    L.jtfs_texture_create.argtypes = [P(vp), vp, i64, ctypes.c_float]
    L.jtfs_texture_set_target.argtypes = [vp, vp, vp]
    L.jtfs_texture_set_start.argtypes = [vp, vp, vp]
    L.jtfs_texture_iterate.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp]
    L.jtfs_texture_read.argtypes = [vp, vp, vp, vp, vp]
    L.jtfs_texture_destroy.argtypes = [vp]
    L.jtfs_texture_destroy.restype = None
    L.jtfs_timing_enable.argtypes = [ctypes.c_int]
    L.jtfs_timing_read.argtypes = [ctypes.c_int, P(ctypes.c_double), P(i64)]
    L.jtfs_last_error.argtypes = []
    L.jtfs_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("jtfs_plan_destroy", "jtfs_bucket_destroy", "jtfs_texture_destroy", "jtfs_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(code: int):
    if code != JTFS_OK:
        raise JTFSError(code, load().jtfs_last_error().decode())
    return code


def params(N, J, Q, J_fr, Q_fr, T, F, average_fr=True, time_scattering=False, lowpass_pairs=False,
           unpad_lambda=False) -> Params:
    flags = ((0 if average_fr else JTFS_NO_FREQ_AVERAGE) | (JTFS_TIME_SCATTERING if time_scattering else 0) |
             (JTFS_LOWPASS_PAIRS if lowpass_pairs else 0) | (JTFS_UNPAD_LAMBDA if unpad_lambda else 0))
    return Params(N=int(N), J=int(J), Q1=int(Q[0]), Q2=int(Q[1]), J_fr=int(J_fr), Q_fr=int(Q_fr),
                  flags=flags, T=int(T), F=int(F))


def query(p: Params) -> Info:
    info = Info()
    check(load().jtfs_query(ctypes.byref(p), ctypes.byref(info)))
    return info


def query_filters(p: Params, family: int):
    """(xi, sigma, log2_decim) of one family from the host FP64 solve."""
    import numpy as np
    L = load()
    cnt = ctypes.c_int32(0)
    cap = 4096
    xi = (ctypes.c_double * cap)()
    sg = (ctypes.c_double * cap)()
    k = (ctypes.c_int32 * cap)()
    check(L.jtfs_query_filters(ctypes.byref(p), family, cap, xi, sg, k, ctypes.byref(cnt)))
    n = cnt.value
    return np.array(xi[:n]), np.array(sg[:n]), np.array(k[:n])


def timing_enable(on: bool):
    check(load().jtfs_timing_enable(1 if on else 0))


def timing_read():
    """{stage name: (total ms, launches)} for every stage; clears the records."""
    out = {}
    for i, name in enumerate(STAGES):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        check(load().jtfs_timing_read(i, ctypes.byref(ms), ctypes.byref(n)))
        out[name] = (ms.value, n.value)
    return out
