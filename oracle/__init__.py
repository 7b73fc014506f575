"""CPU oracle for the soft-decision Viterbi decoder.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the decoder product never does.  It
shares no code with the GPU library (own trellis tables, own encoder, own
quantiser); the only thing both sides take in common is the seeded input
generator package ``workload``.

What each function follows (arXiv 2011.13579):

* ``decode_*``      Algorithm 1 (forward procedure with Eqs. (BM), (PM), (SP0))
                    and Algorithm 2 (traceback), radix-2, in the C library.
* ``decode_r4``     §VIII-A, Eqs. (radix4:BM), (radix4:PM), (radix4:SP0),
                    exact integers; an odd stage count starts with one
                    radix-2 stage.
* ``decode_chunked`` the frame/overlap split of one long stream described in
                    §III: every frame is decoded on its own window and only
                    its own bits are kept.
* ``bruteforce``    (module) exhaustive maximum-likelihood search, numpy.
* ``metric_grad``   derivative of the best path metric with respect to the
                    soft values: by Eq. (BM) the metric is a sum of
                    (-1)^{bit} l terms along the decoded path.

Readings where the paper is silent: a tie in
Eq. (PM) keeps the lower-index previous state; the final state of a
terminated frame is state 0, otherwise the best state with ties to the lowest
index; a known start gives every other state minus infinity, an unknown start
gives all-zero path metrics as Algorithm 1 initialises them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "viterbi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, I64, R4_I64 = 0, 1, 2, 3

_lock = threading.Lock()
_lib = None


class _Code(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("beta", ctypes.c_int32), ("gen", ctypes.c_uint32 * 4)]


class _Frame(ctypes.Structure):
    _fields_ = [
        ("llr_offset", ctypes.c_int64),
        ("bit_offset", ctypes.c_int64),
        ("n_stages", ctypes.c_int32),
        ("out_begin", ctypes.c_int32),
        ("n_out", ctypes.c_int32),
        ("start_known", ctypes.c_int32),
        ("end_state", ctypes.c_int32),
        ("code", ctypes.c_int32),
    ]


FRAME_DTYPE = np.dtype([
    ("llr_offset", np.int64), ("bit_offset", np.int64), ("n_stages", np.int32),
    ("out_begin", np.int32), ("n_out", np.int32), ("start_known", np.int32),
    ("end_state", np.int32), ("code", np.int32)])
assert FRAME_DTYPE.itemsize == ctypes.sizeof(_Frame)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no contraction)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                                   "-shared", "-o", tmp, _SRC, "-lpthread", "-lm"])
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_decode.restype = ctypes.c_int
        lib.orc_decode.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_int32]
        lib.orc_encode.restype = ctypes.c_int
        lib.orc_encode.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p]
        lib.orc_trellis_tables.restype = ctypes.c_int
        lib.orc_trellis_tables.argtypes = [ctypes.c_void_p] * 4
        lib.orc_forward_spread_i64.restype = ctypes.c_int
        lib.orc_forward_spread_i64.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_void_p]
        lib.orc_quantize_i8.restype = None
        lib.orc_quantize_i8.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_float]
        _lib = lib
    return _lib


def _ccode(code) -> _Code:
    c = _Code()
    c.K = int(code.K)
    c.beta = len(code.gens)
    for b, g in enumerate(code.gens):
        c.gen[b] = int(g)
    return c


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


# --------------------------------------------------------------------------
# tables and encoder
# --------------------------------------------------------------------------

def trellis(code):
    """(next[ns,2], out[ns,2], prv[ns,2]) built from the encoder equation."""
    lib = _load()
    ns = 1 << (code.K - 1)
    nxt = np.zeros((ns, 2), np.int32)
    out = np.zeros((ns, 2), np.int32)
    prv = np.zeros((ns, 2), np.int32)
    c = _ccode(code)
    rc = lib.orc_trellis_tables(ctypes.byref(c), nxt.ctypes.data, out.ctypes.data, prv.ctypes.data)
    if rc:
        raise ValueError("bad code")
    return nxt, out, prv


def encode(code, msg, terminate: bool = True) -> np.ndarray:
    """uint8 message [N] -> coded uint8 [S, beta] (oracle's own encoder)."""
    lib = _load()
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    S = msg.shape[0] + (code.K - 1 if terminate else 0)
    coded = np.zeros((S, len(code.gens)), np.uint8)
    c = _ccode(code)
    lib.orc_encode(ctypes.byref(c), msg.ctypes.data, msg.shape[0], int(terminate), coded.ctypes.data)
    return coded


def quantize_i8(llr, scale: float) -> np.ndarray:
    """q = saturate_127(round_half_even(fl32(l * scale)))."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    q = np.zeros(llr.shape, np.int8)
    lib.orc_quantize_i8(llr.ctypes.data, q.ctypes.data, llr.size, ctypes.c_float(scale))
    return q


def forward_spread_i64(code, llr_i8, n_stages: int, start_known: bool = True) -> np.ndarray:
    """max_j PM_j - min_j PM_j over reachable states after each stage (exact ints)."""
    lib = _load()
    llr_i8 = np.ascontiguousarray(llr_i8, dtype=np.int8)
    if llr_i8.size < n_stages * len(code.gens):
        raise ValueError("too few soft values")
    out = np.zeros(n_stages, np.int64)
    c = _ccode(code)
    lib.orc_forward_spread_i64(ctypes.byref(c), llr_i8.ctypes.data, n_stages, int(start_known),
                               out.ctypes.data)
    return out


# --------------------------------------------------------------------------
# decoding
# --------------------------------------------------------------------------

def decode_frames(codes: Sequence, frames: np.ndarray, llr: np.ndarray, mode: int,
                  n_bits_out: int, want_gap: bool = False, n_threads: Optional[int] = None):
    """General batch: ``frames`` is a FRAME_DTYPE array.

    Returns (bits uint8 [n_bits_out], metric [F], end_state int32 [F], gap or None).
    """
    lib = _load()
    frames = np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
    F = frames.shape[0]
    want_i8 = mode in (I64, R4_I64)
    llr = np.ascontiguousarray(llr, dtype=np.int8 if want_i8 else np.float32)
    for f in range(F):
        c = codes[int(frames["code"][f])]
        end = int(frames["llr_offset"][f]) + int(frames["n_stages"][f]) * len(c.gens)
        if frames["llr_offset"][f] < 0 or end > llr.size:
            raise ValueError("frame %d reads outside the soft-value array" % f)
        if frames["bit_offset"][f] < 0 or frames["bit_offset"][f] + frames["n_out"][f] > n_bits_out:
            raise ValueError("frame %d writes outside the output" % f)
    ccodes = (_Code * len(codes))(*[_ccode(c) for c in codes])
    bits = np.zeros(n_bits_out, np.uint8)
    mdt = {F64: np.float64, F32: np.float32, I64: np.int64, R4_I64: np.int64}[mode]
    metric = np.zeros(F, mdt)
    end_state = np.zeros(F, np.int32)
    gap = np.zeros(F, np.float64) if want_gap else None
    rc = lib.orc_decode(mode, ctypes.addressof(ccodes), len(codes), frames.ctypes.data, F,
                        llr.ctypes.data, bits.ctypes.data, metric.ctypes.data,
                        end_state.ctypes.data, gap.ctypes.data if want_gap else None,
                        int(n_threads or default_threads()))
    if rc:
        raise RuntimeError("oracle decode failed (%d)" % rc)
    return bits, metric, end_state, gap


def uniform_frames(code, n_frames: int, n_info: int, terminated: bool = True) -> np.ndarray:
    S = n_info + (code.K - 1 if terminated else 0)
    fr = np.zeros(n_frames, FRAME_DTYPE)
    fr["llr_offset"] = np.arange(n_frames, dtype=np.int64) * S * len(code.gens)
    fr["bit_offset"] = np.arange(n_frames, dtype=np.int64) * n_info
    fr["n_stages"] = S
    fr["out_begin"] = 0
    fr["n_out"] = n_info
    fr["start_known"] = 1
    fr["end_state"] = 0 if terminated else -1
    fr["code"] = 0
    return fr


def decode_uniform(code, llr, n_info: int, terminated: bool = True, mode: int = F64,
                   want_gap: bool = False, n_threads: Optional[int] = None):
    """Equal-length frames: llr [F, S*beta].  Returns (bits [F, N], metric [F], gap)."""
    llr = np.asarray(llr)
    F = llr.shape[0] if llr.ndim == 2 else 1
    fr = uniform_frames(code, F, n_info, terminated)
    bits, metric, _, gap = decode_frames([code], fr, llr.reshape(-1), mode, F * n_info,
                                         want_gap, n_threads)
    return bits.reshape(F, n_info), metric, gap


def decode_r4(code, llr_i8, n_info: int, terminated: bool = True, n_threads=None):
    """Literal radix-4 recursion in exact integers (int8 inputs)."""
    return decode_uniform(code, llr_i8, n_info, terminated, R4_I64, n_threads=n_threads)[:2]


def chunk_windows(n_stages: int, chunk: int, overlap: int):
    """Cores [c*chunk, (c+1)*chunk) clipped to the stream, each decoded on the
    window [core - overlap, core_end + overlap) clipped to the stream."""
    wins = []
    c0 = 0
    while c0 < n_stages:
        c1 = min(c0 + chunk, n_stages)
        w0 = max(0, c0 - overlap)
        w1 = min(n_stages, c1 + overlap)
        wins.append((w0, w1, c0, c1))
        c0 = c1
    return wins


def chunked_frames(code, n_stages: int, chunk: int, overlap: int) -> np.ndarray:
    wins = chunk_windows(n_stages, chunk, overlap)
    beta = len(code.gens)
    fr = np.zeros(len(wins), FRAME_DTYPE)
    for k, (w0, w1, c0, c1) in enumerate(wins):
        fr[k] = (w0 * beta, c0, w1 - w0, c0 - w0, c1 - c0, 1 if w0 == 0 else 0, -1, 0)
    return fr


def decode_chunked(code, llr_stream, n_info: int, chunk: int, overlap: int, mode: int = I64,
                   n_threads=None):
    """One unterminated stream split into chunks with overlap (§III tiling).

    The window starting at the stream's first stage knows its start state (0);
    every other window starts with all-zero path metrics.  Each window is traced
    back from its best final state and emits only its core bits.
    """
    fr = chunked_frames(code, n_info, chunk, overlap)
    bits, metric, end, _ = decode_frames([code], fr, np.asarray(llr_stream).reshape(-1), mode,
                                         n_info, False, n_threads)
    return bits, metric, end


def decode_stream_whole(code, llr_stream, n_info: int, mode: int = I64, n_threads=None):
    """The same stream decoded as one unterminated frame (start 0, best end)."""
    fr = np.zeros(1, FRAME_DTYPE)
    fr[0] = (0, 0, n_info, 0, n_info, 1, -1, 0)
    bits, metric, _, _ = decode_frames([code], fr, np.asarray(llr_stream).reshape(-1), mode,
                                       n_info, False, n_threads)
    return bits, metric


def path_correlation(code, bits, llr, terminated: bool = True, exact_int: bool = False):
    """<(-1)^{enc(bits)}, l>: the metric of the path that ``bits`` drive (Eq. (BM) summed)."""
    coded = encode(code, bits, terminated).reshape(-1)
    sgn = 1 - 2 * coded.astype(np.int64)
    if exact_int:
        return int(np.dot(sgn, np.asarray(llr, dtype=np.int64)))
    return float(np.dot(sgn.astype(np.float64), np.asarray(llr, dtype=np.float64)))


def metric_grad(code, bits, g, terminated: bool = True) -> np.ndarray:
    """d(best path metric)/d(l) for one frame: g * (-1)^{enc(decoded bits)}."""
    coded = encode(code, bits, terminated).reshape(-1)
    return (float(g) * (1.0 - 2.0 * coded.astype(np.float64))).astype(np.float64)
