"""ctypes declarations of the C ABI in include/mivit.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmivit.so")

MIVIT_OK, MIVIT_EINVAL, MIVIT_ENOMEM, MIVIT_EHIP, MIVIT_EUNSUPPORTED = 0, -1, -2, -3, -4
MIVIT_F32, MIVIT_I8, MIVIT_F16 = 0, 1, 2
MIVIT_START_KNOWN, MIVIT_END_ZERO = 1, 2

# every symbol include/mivit.h declares
EXPORTS = (
    "mivit_plan_create", "mivit_plan_create_on", "mivit_decode", "mivit_forward", "mivit_traceback", "mivit_decode_grad", "mivit_plan_destroy",
    "mivit_plan_get_info", "mivit_plan_describe", "mivit_quantize_i8", "mivit_strerror",
    "mivit_version", "mivit_pipe_create", "mivit_pipe_run", "mivit_pipe_destroy",
    "mivit_stream_create", "mivit_stream_push", "mivit_stream_finish", "mivit_stream_destroy",
    "mivit_decode_uniform", "mivit_decode_uniform_noalloc",
)
MIVIT_PLAN_GRAPH, MIVIT_PLAN_AUTOTUNE, MIVIT_PLAN_PERSISTENT, MIVIT_PLAN_NO_SPLIT = 1, 2, 4, 8


class Code(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("beta", ctypes.c_int32), ("gen", ctypes.c_uint32 * 4)]


class Frame(ctypes.Structure):
    _fields_ = [
        ("llr_offset", ctypes.c_int64),
        ("bit_offset", ctypes.c_int64),
        ("n_stages", ctypes.c_int32),
        ("out_begin", ctypes.c_int32),
        ("n_out", ctypes.c_int32),
        ("code", ctypes.c_int16),
        ("flags", ctypes.c_uint16),
    ]


FRAME_DTYPE = np.dtype([
    ("llr_offset", np.int64), ("bit_offset", np.int64), ("n_stages", np.int32),
    ("out_begin", np.int32), ("n_out", np.int32), ("code", np.int16), ("flags", np.uint16)])
assert FRAME_DTYPE.itemsize == ctypes.sizeof(Frame) == 32


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("radix", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32 * 2)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_items", ctypes.c_int64), ("survivor_bytes", ctypes.c_int64),
                ("total_stages", ctypes.c_int64), ("radix", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("llr_elems", ctypes.c_int64),
                ("bit_words", ctypes.c_int64), ("n_frames", ctypes.c_int32),
                ("device", ctypes.c_int32)]


class MivitError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(status), status))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmivit.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2011_13579_amd.build" % path)
    # The library takes torch's device pointers and streams, so it must bind to
    # the HIP runtime torch ships: load torch first, then the library resolves
    # its libamdhip64 to that copy instead of loading a second runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mivit_plan_create.restype = ctypes.c_int
    lib.mivit_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Code), i32,
                                      ctypes.c_void_p, i32, ctypes.POINTER(Opts)]
    lib.mivit_plan_create_on.restype = ctypes.c_int
    lib.mivit_plan_create_on.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(Code), i32,
                                         ctypes.c_void_p, i32, ctypes.POINTER(Opts)]
    lib.mivit_decode.restype = ctypes.c_int
    lib.mivit_decode.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mivit_forward.restype = ctypes.c_int
    lib.mivit_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.mivit_traceback.restype = ctypes.c_int
    lib.mivit_traceback.argtypes = [vp, vp, vp]
    lib.mivit_decode_grad.restype = ctypes.c_int
    lib.mivit_decode_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.mivit_plan_destroy.restype = ctypes.c_int
    lib.mivit_plan_destroy.argtypes = [vp]
    lib.mivit_plan_get_info.restype = ctypes.c_int
    lib.mivit_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.mivit_plan_describe.restype = ctypes.c_int
    lib.mivit_plan_describe.argtypes = [vp, ctypes.c_char_p, i32]
    lib.mivit_quantize_i8.restype = ctypes.c_int
    lib.mivit_quantize_i8.argtypes = [vp, vp, i64, ctypes.c_float, vp]
    lib.mivit_strerror.restype = ctypes.c_char_p
    lib.mivit_strerror.argtypes = [ctypes.c_int]
    lib.mivit_version.restype = ctypes.c_char_p
    lib.mivit_version.argtypes = []
    lib.mivit_pipe_create.restype = ctypes.c_int
    lib.mivit_pipe_create.argtypes = [ctypes.POINTER(vp), vp, i32]
    lib.mivit_pipe_run.restype = ctypes.c_int
    lib.mivit_pipe_run.argtypes = [vp, vp, vp, vp, i64]
    lib.mivit_pipe_destroy.restype = ctypes.c_int
    lib.mivit_pipe_destroy.argtypes = [vp]
    lib.mivit_stream_create.restype = ctypes.c_int
    lib.mivit_stream_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Code),
                                        ctypes.POINTER(Opts), ctypes.c_uint32, i64]
    lib.mivit_stream_push.restype = ctypes.c_int
    lib.mivit_stream_push.argtypes = [vp, vp, i64, vp, ctypes.POINTER(i64), vp]
    lib.mivit_stream_finish.restype = ctypes.c_int
    lib.mivit_stream_finish.argtypes = [vp, vp, ctypes.POINTER(i64), vp]
    lib.mivit_stream_destroy.restype = ctypes.c_int
    lib.mivit_stream_destroy.argtypes = [vp]
    lib.mivit_decode_uniform.restype = ctypes.c_int
    lib.mivit_decode_uniform.argtypes = [vp, i32, ctypes.POINTER(Code), i32, i32, i32, vp, vp, vp]
    lib.mivit_decode_uniform_noalloc.restype = ctypes.c_int
    lib.mivit_decode_uniform_noalloc.argtypes = [vp, i32, ctypes.POINTER(Code), i32, i32, i32, vp,
                                                 vp, vp]
    _lib = lib
    return lib


def strerror(status: int) -> str:
    try:
        return load().mivit_strerror(status).decode()
    except Exception:  # pragma: no cover - library missing
        return "status %d" % status


def check(status: int, what: str):
    if status != MIVIT_OK:
        raise MivitError(status, what)
