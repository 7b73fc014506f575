"""mivit: soft-decision Viterbi decoding of convolutional codes on MI355X.

Python binding of the C ABI in include/mivit.h.  Every step of decoding runs
in the HIP library (libmivit.so); this module only marshals arguments: device
pointers of torch tensors, the current HIP stream, descriptor arrays.  There is
no CPU fallback: if the library is missing every call raises.

Entry points
  Plan(codes, frames, dtype, radix, chunk, overlap)  general batch
  decode(llr, code, n_info, terminated, radix)       equal-length frames
  decode_stream(llr, code, n_info, chunk, overlap)   one long stream, chunked
  quantize_i8(llr, scale)                            float32 -> int8 soft values
  Pipeline(plan, depth).run(host_llr, host_bits)     batches from host memory
  StreamDecoder(code, dtype, chunk, overlap, ...)    one stream pushed in pieces
  ViterbiDecode.apply(llr, code, n_info)             autograd on the best metric
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _capi
from ._capi import (FRAME_DTYPE, MIVIT_END_ZERO, MIVIT_F16, MIVIT_F32, MIVIT_I8, MIVIT_START_KNOWN,
                    MivitError)

__all__ = ["Code", "Plan", "Pipeline", "StreamDecoder", "decode", "decode_stream", "quantize_i8", "ViterbiDecode",
           "unpack_bits", "FRAME_DTYPE", "MivitError", "version"]


def _torch():
    import torch
    return torch


@dataclass(frozen=True)
class Code:
    """Convolutional code: constraint length K and one K-bit tap mask per
    output bit (bit K-1 taps the current input)."""
    K: int
    gens: tuple

    @property
    def beta(self) -> int:
        return len(self.gens)

    @staticmethod
    def from_octal(K: int, gens_octal: Sequence[str]) -> "Code":
        return Code(K, tuple(int(str(g), 8) for g in gens_octal))

    def c_struct(self) -> _capi.Code:
        c = _capi.Code()
        c.K = int(self.K)
        c.beta = len(self.gens)
        for b, g in enumerate(self.gens):
            c.gen[b] = int(g)
        return c


def _as_code(code) -> Code:
    if isinstance(code, Code):
        return code
    return Code(int(code.K), tuple(int(g) for g in code.gens))


def version() -> str:
    return _capi.load().mivit_version().decode()


def _stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


class Plan:
    """A fixed batch of frames (see mivit_plan_create and mivit_plan_create_on).

    frames: numpy array of FRAME_DTYPE (llr_offset, bit_offset, n_stages,
    out_begin, n_out, code, flags).
    """

    def __init__(self, codes: Sequence, frames: np.ndarray, dtype: str = "f32", radix: int = 0,
                 chunk: int = 0, overlap: int = 0, variant: int = 0, graph: bool = False,
                 autotune: bool = False, persistent: bool = False, split: bool = True,
                 device=None):
        lib = _capi.load()
        self.codes = [_as_code(c) for c in codes]
        self.frames = np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
        self.dtype = {"f32": MIVIT_F32, "i8": MIVIT_I8, "f16": MIVIT_F16}[dtype]
        arr = (_capi.Code * len(self.codes))(*[c.c_struct() for c in self.codes])
        opts = _capi.Opts()
        opts.dtype, opts.radix, opts.chunk, opts.overlap = self.dtype, int(radix), int(chunk), int(overlap)
        opts.variant = int(variant)
        opts.flags = ((_capi.MIVIT_PLAN_GRAPH if graph else 0) |
                      (_capi.MIVIT_PLAN_AUTOTUNE if autotune else 0) |
                      (_capi.MIVIT_PLAN_PERSISTENT if persistent else 0) |
                      (0 if split else _capi.MIVIT_PLAN_NO_SPLIT))
        h = ctypes.c_void_p()
        # device: None (or a torch device without an index) for the current
        # device, else a device index or a torch device (mivit_plan_create_on)
        if device is None:
            dev = -1
        elif isinstance(device, int):
            dev = device
        else:
            dev = -1 if device.index is None else int(device.index)
        st = lib.mivit_plan_create_on(ctypes.byref(h), dev, arr, len(self.codes),
                                      self.frames.ctypes.data if len(self.frames) else None,
                                      len(self.frames), ctypes.byref(opts))
        _capi.check(st, "mivit_plan_create_on")
        self._h = h
        self._lib = lib
        info = _capi.PlanInfo()
        _capi.check(lib.mivit_plan_get_info(h, ctypes.byref(info)), "mivit_plan_get_info")
        self.n_items = int(info.n_items)
        self.survivor_bytes = int(info.survivor_bytes)
        self.total_stages = int(info.total_stages)
        self.radix = int(info.radix)
        self.n_frames = len(self.frames)
        if len(self.frames):
            ends = self.frames["bit_offset"] + self.frames["n_out"]
            self.n_bit_words = int((ends.max() + 31) // 32)
            beta = np.array([c.beta for c in self.codes], np.int64)[self.frames["code"]]
            self.llr_extent = int((self.frames["llr_offset"] +
                                   self.frames["n_stages"].astype(np.int64) * beta).max())
        else:
            self.n_bit_words = 0
            self.llr_extent = 0

    def describe(self) -> str:
        """The plan's parts: kernel, variant and launch form per code."""
        buf = ctypes.create_string_buffer(4096)
        _capi.check(self._lib.mivit_plan_describe(self._h, buf, len(buf)), "mivit_plan_describe")
        return buf.value.decode()

    @property
    def handle(self) -> int:
        return int(self._h.value or 0)

    def empty_outputs(self, device):
        torch = _torch()
        bits = torch.zeros(max(self.n_bit_words, 1), dtype=torch.int32, device=device)
        mdt = torch.int64 if self.dtype == MIVIT_I8 else torch.float32
        metric = torch.zeros(max(self.n_frames, 1), dtype=mdt, device=device)
        end = torch.zeros(max(self.n_frames, 1), dtype=torch.int32, device=device)
        return bits, metric, end

    def _check_io(self, llr=None, bits=None, metric=None, end_state=None):
        """The library takes raw device pointers: tensors must have the plan's
        types and at least the extents its frames address."""
        torch = _torch()
        want = {MIVIT_F32: torch.float32, MIVIT_I8: torch.int8, MIVIT_F16: torch.float16}
        mdt = torch.int64 if self.dtype == MIVIT_I8 else torch.float32
        for name, t, dt, n in (("llr", llr, want[self.dtype], self.llr_extent),
                               ("bits", bits, torch.int32, self.n_bit_words),
                               ("metric", metric, mdt, self.n_frames),
                               ("end_state", end_state, torch.int32, self.n_frames)):
            if t is None:
                continue
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < n:
                raise ValueError("%s must be a contiguous device tensor of dtype %s with at "
                                 "least %d elements" % (name, dt, n))

    def decode(self, llr, bits=None, metric=None, end_state=None, stream=None):
        """Decode on the current stream; returns (bit words int32, metric, end state).
        Without bits, all three outputs are allocated; metric and end_state
        may otherwise be None (not written)."""
        if bits is None:
            bits, metric, end_state = self.empty_outputs(llr.device)
        self._check_io(llr, bits, metric, end_state)
        st = self._lib.mivit_decode(self._h, _dptr(llr), _dptr(bits), _dptr(metric),
                                    _dptr(end_state), _stream_handle(stream))
        _capi.check(st, "mivit_decode")
        return bits, metric, end_state

    def forward(self, llr, metric=None, end_state=None, stream=None):
        """Forward procedure only (decisions stay in the plan)."""
        self._check_io(llr, None, metric, end_state)
        st = self._lib.mivit_forward(self._h, _dptr(llr), _dptr(metric), _dptr(end_state),
                                     _stream_handle(stream))
        _capi.check(st, "mivit_forward")

    def traceback(self, bits, stream=None):
        """Traceback of the decisions left by the last forward call."""
        self._check_io(None, bits)
        st = self._lib.mivit_traceback(self._h, _dptr(bits), _stream_handle(stream))
        _capi.check(st, "mivit_traceback")
        return bits

    def decode_grad(self, bits, grad_metric, grad_llr, stream=None):
        """d(metric)/d(llr) of the decode that wrote bits (float32 tensors)."""
        torch = _torch()
        self._check_io(None, bits)
        for name, t, n in (("grad_metric", grad_metric, self.n_frames),
                           ("grad_llr", grad_llr, self.llr_extent)):
            if (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                    or t.numel() < n):
                raise ValueError("%s must be a contiguous float32 device tensor with at least "
                                 "%d elements" % (name, n))
        st = self._lib.mivit_decode_grad(self._h, _dptr(bits), _dptr(grad_metric),
                                         _dptr(grad_llr), _stream_handle(stream))
        _capi.check(st, "mivit_decode_grad")
        return grad_llr

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mivit_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """Host pipeline over a plan (mivit_pipe_*): batches of soft values in
    host memory, each laid out as the plan's frames describe, are copied in,
    decoded and their bits (and metrics) copied back, with copy-in, decode
    and copy-out of different batches overlapping.  The plan must stay
    alive and unused by other calls while run() runs."""

    def __init__(self, plan: "Plan", depth: int = 3):
        self._lib = _capi.load()
        self.plan = plan
        info = _capi.PlanInfo()
        _capi.check(self._lib.mivit_plan_get_info(plan._h, ctypes.byref(info)),
                    "mivit_plan_get_info")
        self.llr_elems, self.bit_words, self.n_frames = (int(info.llr_elems),
                                                         int(info.bit_words), int(info.n_frames))
        h = ctypes.c_void_p()
        _capi.check(self._lib.mivit_pipe_create(ctypes.byref(h), plan._h, int(depth)),
                    "mivit_pipe_create")
        self._h = h

    def run(self, host_llr, host_bits, host_metric=None, n_batches: Optional[int] = None):
        """Decode n_batches batches (default: as many as host_llr holds);
        blocks until the results are in host memory.  Page-locked tensors
        (pin_memory) let the copies overlap the decodes."""
        torch = _torch()
        want = {MIVIT_F32: torch.float32, MIVIT_I8: torch.int8, MIVIT_F16: torch.float16}
        mdt = torch.int64 if self.plan.dtype == MIVIT_I8 else torch.float32
        if n_batches is None:
            n_batches = host_llr.numel() // max(self.llr_elems, 1)
        for name, t, dt, n in (("host_llr", host_llr, want[self.plan.dtype], self.llr_elems),
                               ("host_bits", host_bits, torch.int32, self.bit_words),
                               ("host_metric", host_metric, mdt, self.n_frames)):
            if t is None:
                continue
            if (t.dtype != dt or t.is_cuda or not t.is_contiguous()
                    or t.numel() < n * n_batches):
                raise ValueError("%s must be a contiguous host tensor of dtype %s with at least "
                                 "%d elements" % (name, dt, n * n_batches))
        st = self._lib.mivit_pipe_run(self._h, host_llr.data_ptr(), host_bits.data_ptr(),
                                      host_metric.data_ptr() if host_metric is not None else None,
                                      int(n_batches))
        _capi.check(st, "mivit_pipe_run")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mivit_pipe_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StreamDecoder:
    """One continuous stream whose soft values arrive in pieces
    (mivit_stream_*): cut into windows of ``chunk`` core stages with
    ``overlap`` stages on each side exactly as decode_stream cuts it, each
    window decoded once its right overlap has arrived.  push() and finish()
    return the bit words of the windows completed by that call (one bit per
    stage, stream order) and their number of bits; concatenated, they equal
    the one-shot chunked decode of the whole stream."""

    def __init__(self, code, dtype: str = "i8", chunk: int = 2048, overlap: int = 64,
                 max_push_stages: int = 1 << 20, radix: int = 0, variant: int = 0,
                 start_known: bool = True, end_zero: bool = False):
        self._lib = _capi.load()
        self.code = _as_code(code)
        self.dtype = {"f32": MIVIT_F32, "i8": MIVIT_I8, "f16": MIVIT_F16}[dtype]
        self.chunk, self.overlap = int(chunk), int(overlap)
        self.max_push_stages = int(max_push_stages)
        opts = _capi.Opts()
        opts.dtype, opts.radix, opts.chunk, opts.overlap = self.dtype, int(radix), self.chunk, \
            self.overlap
        opts.variant = int(variant)
        flags = (MIVIT_START_KNOWN if start_known else 0) | (MIVIT_END_ZERO if end_zero else 0)
        h = ctypes.c_void_p()
        _capi.check(self._lib.mivit_stream_create(ctypes.byref(h), ctypes.byref(self.code.c_struct()),
                                                  ctypes.byref(opts), flags, self.max_push_stages),
                    "mivit_stream_create")
        self._h = h
        self._words = None  # output words, sized for one call

    def _out(self, device):
        torch = _torch()
        n = (self.max_push_stages + self.chunk + 2 * self.overlap + 31) // 32
        if self._words is None or self._words.device != device:
            self._words = torch.empty(n, dtype=torch.int32, device=device)
        return self._words

    def push(self, llr, stream=None):
        """llr: device tensor of whole stages (beta soft values each) of the
        stream's dtype.  Returns (bit words int32, number of bits); the words
        are a view of a buffer the next call overwrites."""
        torch = _torch()
        want = {MIVIT_F32: torch.float32, MIVIT_I8: torch.int8, MIVIT_F16: torch.float16}
        beta = self.code.beta
        if llr.dtype != want[self.dtype] or not llr.is_cuda or llr.numel() % beta:
            raise ValueError("soft values must be a device tensor of dtype %s holding whole "
                             "stages of %d values" % (want[self.dtype], beta))
        llr = llr.contiguous()
        n_st = llr.numel() // beta
        if n_st > self.max_push_stages:
            raise ValueError("push of %d stages exceeds max_push_stages=%d"
                             % (n_st, self.max_push_stages))
        words = self._out(llr.device)
        nb = ctypes.c_int64()
        _capi.check(self._lib.mivit_stream_push(self._h, _dptr(llr), n_st, _dptr(words),
                                                ctypes.byref(nb), _stream_handle(stream)),
                    "mivit_stream_push")
        return words[: (nb.value + 31) // 32], nb.value

    def finish(self, device=None, stream=None):
        """End of the stream: the remaining windows' bit words and bit count."""
        torch = _torch()
        words = self._out(torch.device(device) if device is not None else
                          (self._words.device if self._words is not None else
                           torch.device("cuda", torch.cuda.current_device())))
        nb = ctypes.c_int64()
        _capi.check(self._lib.mivit_stream_finish(self._h, _dptr(words), ctypes.byref(nb),
                                                  _stream_handle(stream)),
                    "mivit_stream_finish")
        return words[: (nb.value + 31) // 32], nb.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.mivit_stream_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def uniform_frames(code, n_frames: int, n_info: int, terminated: bool = True) -> np.ndarray:
    """Frames laid out back to back: frame f reads llr[f] and writes bit words
    [f * ceil(N/32), (f+1) * ceil(N/32))."""
    code = _as_code(code)
    S = n_info + (code.K - 1 if terminated else 0)
    wpf = (n_info + 31) // 32
    fr = np.zeros(n_frames, FRAME_DTYPE)
    fr["llr_offset"] = np.arange(n_frames, dtype=np.int64) * S * code.beta
    fr["bit_offset"] = np.arange(n_frames, dtype=np.int64) * wpf * 32
    fr["n_stages"] = S
    fr["out_begin"] = 0
    fr["n_out"] = n_info
    fr["code"] = 0
    fr["flags"] = MIVIT_START_KNOWN | (MIVIT_END_ZERO if terminated else 0)
    return fr


_plan_cache = {}


def _cached_plan(key, make):
    """Plans by (shape, device, stream): a plan owns survivor memory, so one
    plan only ever serves one stream.  An evicted plan is dropped, not
    closed: a caller that still holds it (an autograd context between
    forward and backward) keeps it alive, and it is freed with its last
    reference."""
    p = _plan_cache.get(key)
    if p is None:
        if len(_plan_cache) >= 8:
            _plan_cache.pop(next(iter(_plan_cache)))
        p = make()
        _plan_cache[key] = p
    return p


def _dtype_name(torch, llr):
    names = {torch.float32: "f32", torch.int8: "i8", torch.float16: "f16"}
    if llr.dtype not in names:
        raise ValueError("soft values must be float32, float16 or int8, not %s" % llr.dtype)
    return names[llr.dtype]


def decode(llr, code, n_info: int, terminated: bool = True, radix: int = 0, stream=None):
    """Equal-length frames.  llr: device tensor [F, S*beta] float32, float16 or int8.

    radix 0 calls mivit_decode_uniform (the library picks the kernel);
    radix 2, 4 or 8 builds (and caches) a plan with that radix.
    Returns (bit words int32 [F, ceil(N/32)], metric [F]).
    """
    torch = _torch()
    code = _as_code(code)
    F = llr.shape[0] if llr.dim() == 2 else 1
    dt = _dtype_name(torch, llr)
    wpf = (n_info + 31) // 32
    S = n_info + (code.K - 1 if terminated else 0)
    llr = llr.contiguous()
    if llr.numel() < F * S * code.beta or not llr.is_cuda:
        raise ValueError("llr must be a device tensor of at least %d soft values" % (F * S * code.beta))
    if radix == 0:
        dtc = {"f32": MIVIT_F32, "i8": MIVIT_I8, "f16": MIVIT_F16}[dt]
        bits = torch.zeros(max(F * wpf, 1), dtype=torch.int32, device=llr.device)
        metric = torch.zeros(max(F, 1), dtype=torch.int64 if dt == "i8" else torch.float32,
                             device=llr.device)
        st = _capi.load().mivit_decode_uniform(_dptr(llr), dtc, ctypes.byref(code.c_struct()),
                                               F, int(n_info), int(bool(terminated)), _dptr(bits),
                                               _dptr(metric), _stream_handle(stream))
        _capi.check(st, "mivit_decode_uniform")
        return bits[: F * wpf].view(F, wpf), metric[:F]
    key = ("u", code, F, n_info, terminated, dt, radix, llr.device.index, _stream_handle(stream))
    plan = _cached_plan(key, lambda: Plan([code], uniform_frames(code, F, n_info, terminated),
                                          dt, radix))
    bits, metric, _ = plan.decode(llr, stream=stream)
    return bits[: F * wpf].view(F, wpf), metric[:F]


def decode_stream(llr, code, n_info: int, chunk: int = 2048, overlap: int = 64, radix: int = 0,
                  stream=None):
    """One unterminated stream starting in state 0, split into chunks of
    ``chunk`` stages decoded on windows widened by ``overlap`` on each side.
    Returns bit words int32 [ceil(N/32)]."""
    torch = _torch()
    code = _as_code(code)
    dt = _dtype_name(torch, llr)
    fr = np.zeros(1, FRAME_DTYPE)
    fr[0] = (0, 0, n_info, 0, n_info, 0, MIVIT_START_KNOWN)
    key = ("s", code, n_info, chunk, overlap, dt, radix, llr.device.index, _stream_handle(stream))
    plan = _cached_plan(key, lambda: Plan([code], fr, dt, radix, chunk, overlap))
    bits, metric, end = plan.decode(llr.contiguous(), stream=stream)
    return bits[: (n_info + 31) // 32]


def quantize_i8(llr, scale: float, out=None, stream=None):
    """int8 soft values: saturate_127(round_half_even(fl32(llr * scale)))."""
    torch = _torch()
    if llr.dtype != torch.float32 or not llr.is_cuda:
        raise ValueError("llr must be a float32 device tensor")
    llr = llr.contiguous()
    if out is None:
        out = torch.empty(llr.shape, dtype=torch.int8, device=llr.device)
    elif (out.dtype != torch.int8 or out.device != llr.device or not out.is_contiguous()
          or out.numel() < llr.numel()):
        raise ValueError("out must be a contiguous int8 tensor on the device of llr with at "
                         "least llr.numel() elements")
    st = _capi.load().mivit_quantize_i8(_dptr(llr), _dptr(out), llr.numel(), float(scale),
                                        _stream_handle(stream))
    _capi.check(st, "mivit_quantize_i8")
    return out


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """Host helper: packed LSB-first words [..., W] -> uint8 bits [..., n]."""
    w = np.ascontiguousarray(words).view(np.uint32)
    b = ((w[..., :, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.uint8)
    return b.reshape(w.shape[:-1] + (w.shape[-1] * 32,))[..., :n]


def _make_autograd():
    torch = _torch()

    class ViterbiDecode(torch.autograd.Function):
        """(bits, metric) = decode(llr); d(metric)/d(llr) from the HIP backward
        kernel (the decoded codeword in +-1 form times the incoming gradient).
        Bits are not differentiable."""

        @staticmethod
        def forward(ctx, llr, code, n_info, terminated=True):
            code = _as_code(code)
            F = llr.shape[0]
            key = ("u", code, F, n_info, terminated, "f32", 2, llr.device.index,
                   _stream_handle(None))
            plan = _cached_plan(key, lambda: Plan([code], uniform_frames(code, F, n_info, terminated),
                                                  "f32", 2))
            bits, metric, _ = plan.decode(llr.contiguous())
            ctx.plan = plan
            ctx.save_for_backward(bits)
            ctx.shape = llr.shape
            wpf = (n_info + 31) // 32
            out_bits = bits[: F * wpf].view(F, wpf)
            ctx.mark_non_differentiable(out_bits)
            return out_bits, metric[:F].clone()

        @staticmethod
        def backward(ctx, g_bits, g_metric):
            (bits,) = ctx.saved_tensors
            grad = torch.empty(ctx.shape, dtype=torch.float32, device=bits.device)
            ctx.plan.decode_grad(bits, g_metric.contiguous().float(), grad)
            return grad, None, None, None

    return ViterbiDecode


class _LazyAutograd:
    _cls = None

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls, name)


ViterbiDecode = _LazyAutograd()
