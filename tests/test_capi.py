"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects invalid arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2011_13579_amd import _capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mivit.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_capi.LIB_PATH),
                                reason="libmivit.so not built")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mivit_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding():
    assert sorted(_capi.EXPORTS) == declared_symbols()


def test_exports_every_symbol():
    lib = ctypes.CDLL(_capi.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_struct_layouts():
    assert ctypes.sizeof(_capi.Code) == 24
    assert ctypes.sizeof(_capi.Frame) == 32
    assert ctypes.sizeof(_capi.Opts) == 32
    text = open(HEADER).read()
    assert "int64_t llr_offset" in text and "uint16_t flags" in text


def test_strerror_and_version():
    lib = _capi.load()
    assert lib.mivit_strerror(0) == b"ok"
    assert lib.mivit_strerror(-1) == b"invalid argument"
    assert b"gfx950" in lib.mivit_version()


def _plan_status(codes, frames, **opts):
    lib = _capi.load()
    arr = (_capi.Code * len(codes))(*codes)
    o = _capi.Opts()
    for k, v in opts.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    fr = np.ascontiguousarray(frames, dtype=_capi.FRAME_DTYPE)
    st = lib.mivit_plan_create(ctypes.byref(h), arr, len(codes),
                               fr.ctypes.data if len(fr) else None, len(fr), ctypes.byref(o))
    assert not h.value  # nothing allocated on rejection
    return st


def _code(K, gens):
    c = _capi.Code()
    c.K, c.beta = K, len(gens)
    for b, g in enumerate(gens):
        c.gen[b] = g
    return c


def _frame(**kw):
    f = np.zeros(1, _capi.FRAME_DTYPE)
    f[0] = (0, 0, 10, 0, 4, 0, 3)
    for k, v in kw.items():
        f[k] = v
    return f


K7 = _code(7, [0o133, 0o171])


@pytest.mark.parametrize("code,status", [
    (_code(2, [3, 3]), _capi.MIVIT_EINVAL),           # K too small
    (_code(10, [0o1001, 0o1001]), _capi.MIVIT_EINVAL),  # K too large
    (_code(7, [0o133]), _capi.MIVIT_EINVAL),            # beta = 1
    (_code(7, [0o333, 0o171]), _capi.MIVIT_EINVAL),     # generator >= 2^K
    (_code(7, [0o132, 0o171]), _capi.MIVIT_EUNSUPPORTED),  # LSB tap missing
    (_code(7, [0o033, 0o171]), _capi.MIVIT_EUNSUPPORTED),  # MSB tap missing
])
def test_bad_codes(code, status):
    assert _plan_status([code], _frame()) == status


@pytest.mark.parametrize("kw", [
    dict(code=1), dict(code=-1), dict(n_stages=-1), dict(n_out=11), dict(out_begin=8),
    dict(bit_offset=5), dict(llr_offset=-2), dict(flags=8),
])
def test_bad_frames(kw):
    assert _plan_status([K7], _frame(**kw)) == _capi.MIVIT_EINVAL


def test_overlapping_outputs():
    fr = np.concatenate([_frame(), _frame(bit_offset=0)])
    assert _plan_status([K7], fr) == _capi.MIVIT_EINVAL


@pytest.mark.parametrize("opts", [
    dict(dtype=3), dict(dtype=-1), dict(radix=3), dict(radix=16), dict(radix=4, dtype=0),
    dict(radix=4, dtype=2), dict(radix=8, dtype=0), dict(radix=8, dtype=2),
    dict(chunk=-1), dict(chunk=100),
    dict(overlap=-1), dict(variant=9), dict(flags=16), dict(flags=1 << 31),
])
def test_bad_opts(opts):
    assert _plan_status([K7], _frame(), **opts) == _capi.MIVIT_EINVAL


@pytest.mark.parametrize("variant", [1, 2])
def test_f16_other_variants_unsupported(variant):
    """float16 soft values run the default exchange scheme only."""
    assert _plan_status([K7], _frame(), dtype=_capi.MIVIT_F16, variant=variant) == \
        _capi.MIVIT_EUNSUPPORTED


@pytest.mark.parametrize("code,variant", [(_code(3, [7, 5]), 0), (K7, 1), (K7, 2)])
def test_radix8_unsupported(code, variant):
    """Radix 8 needs at least 8 states and runs one kernel (variant 0)."""
    assert _plan_status([code], _frame(), dtype=_capi.MIVIT_I8, radix=8, variant=variant) == \
        _capi.MIVIT_EUNSUPPORTED


def test_dtype_values():
    """The soft-value type constants of the binding match the header's."""
    text = open(os.path.join(ROOT, "include", "mivit.h")).read()
    m = re.search(r"MIVIT_F32 = (\d+), MIVIT_I8 = (\d+), MIVIT_F16 = (\d+)", text)
    assert m and tuple(int(x) for x in m.groups()) == (_capi.MIVIT_F32, _capi.MIVIT_I8,
                                                          _capi.MIVIT_F16)


def test_reserved_opts_must_be_zero():
    for k in range(2):
        lib = _capi.load()
        arr = (_capi.Code * 1)(K7)
        o = _capi.Opts()
        o.reserved[k] = 1
        h = ctypes.c_void_p()
        fr = _frame()
        assert lib.mivit_plan_create(ctypes.byref(h), arr, 1, fr.ctypes.data, 1,
                                     ctypes.byref(o)) == _capi.MIVIT_EINVAL
        assert not h.value


def test_plan_flag_values():
    """The flag constants of the binding match the header's."""
    text = open(os.path.join(ROOT, "include", "mivit.h")).read()
    for name in ("MIVIT_PLAN_GRAPH", "MIVIT_PLAN_AUTOTUNE", "MIVIT_PLAN_PERSISTENT"):
        m = re.search(r"#define %s (\d+)u" % name, text)
        assert m and int(m.group(1)) == getattr(_capi, name)


def test_pipe_null_arguments():
    lib = _capi.load()
    h = ctypes.c_void_p()
    assert lib.mivit_pipe_create(None, None, 3) == _capi.MIVIT_EINVAL
    assert lib.mivit_pipe_create(ctypes.byref(h), None, 3) == _capi.MIVIT_EINVAL
    assert not h.value
    assert lib.mivit_pipe_run(None, None, None, None, 1) == _capi.MIVIT_EINVAL
    assert lib.mivit_pipe_destroy(None) == _capi.MIVIT_EINVAL


def test_stream_invalid_arguments():
    """Stream objects: argument checks that need no device."""
    lib = _capi.load()
    h = ctypes.c_void_p()
    o = _capi.Opts()
    o.dtype, o.chunk, o.overlap = _capi.MIVIT_I8, 2048, 64
    assert lib.mivit_stream_create(None, ctypes.byref(K7), ctypes.byref(o), 1, 1024) == \
        _capi.MIVIT_EINVAL
    assert lib.mivit_stream_create(ctypes.byref(h), None, ctypes.byref(o), 1, 1024) == \
        _capi.MIVIT_EINVAL
    assert lib.mivit_stream_create(ctypes.byref(h), ctypes.byref(K7), None, 1, 1024) == \
        _capi.MIVIT_EINVAL
    for chunk, overlap, flags, maxp in [(0, 64, 1, 1024), (100, 64, 1, 1024), (2048, -1, 1, 1024),
                                        (2048, 64, 8, 1024), (2048, 64, 1, 0),
                                        (2048, 1 << 30, 1, 1024)]:
        o.chunk, o.overlap = chunk, overlap
        assert lib.mivit_stream_create(ctypes.byref(h), ctypes.byref(K7), ctypes.byref(o), flags,
                                       maxp) == _capi.MIVIT_EINVAL
        assert not h.value
    nb = ctypes.c_int64()
    assert lib.mivit_stream_push(None, None, 0, None, ctypes.byref(nb), None) == _capi.MIVIT_EINVAL
    assert lib.mivit_stream_finish(None, None, ctypes.byref(nb), None) == _capi.MIVIT_EINVAL
    assert lib.mivit_stream_destroy(None) == _capi.MIVIT_EINVAL


def test_null_and_misc():
    lib = _capi.load()
    assert lib.mivit_plan_create(None, None, 0, None, 0, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_decode(None, None, None, None, None, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_decode_grad(None, None, None, None, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_plan_destroy(None) == _capi.MIVIT_EINVAL
    assert lib.mivit_plan_get_info(None, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_plan_describe(None, None, 0) == _capi.MIVIT_EINVAL
    assert lib.mivit_quantize_i8(None, None, -1, 1.0, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_quantize_i8(None, None, 10, 1.0, None) == _capi.MIVIT_EINVAL
    assert lib.mivit_quantize_i8(None, None, 0, 0.0, None) == _capi.MIVIT_EINVAL


def test_decode_uniform_rejects_before_device_work():
    """mivit_decode_uniform validates its arguments before touching the
    device: null pointers, negative counts, bad dtype, bad terminated flag
    and bad codes are rejected; an empty batch is a no-op."""
    lib = _capi.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation
    cases = [
        ((None, 0, K7, 4, 100, 1, fake, None, None), _capi.MIVIT_EINVAL),   # no soft values
        ((fake, 0, K7, 4, 100, 1, None, None, None), _capi.MIVIT_EINVAL),   # no bits
        ((fake, 7, K7, 4, 100, 1, fake, None, None), _capi.MIVIT_EINVAL),   # dtype
        ((fake, 0, K7, -1, 100, 1, fake, None, None), _capi.MIVIT_EINVAL),  # frames
        ((fake, 0, K7, 4, -5, 1, fake, None, None), _capi.MIVIT_EINVAL),    # length
        ((fake, 0, K7, 4, 100, 2, fake, None, None), _capi.MIVIT_EINVAL),   # terminated flag
        ((fake, 0, _code(10, [0o1001, 0o1777]), 4, 100, 1, fake, None, None), _capi.MIVIT_EINVAL),
        ((fake, 0, _code(7, [0o132, 0o171]), 4, 100, 1, fake, None, None),
         _capi.MIVIT_EUNSUPPORTED),                                           # no LSB tap
        ((None, 0, K7, 0, 100, 1, None, None, None), _capi.MIVIT_OK),        # empty batch
        ((None, 1, K7, 5, 0, 0, None, None, None), _capi.MIVIT_OK),          # zero stages
    ]
    for args, want in cases:
        llr, dt, code, F, n, term, bits, metric, st = args
        got = lib.mivit_decode_uniform(llr, dt, ctypes.byref(code), F, n, term, bits, metric, st)
        assert got == want, (args, got)
    assert lib.mivit_decode_uniform(fake, 0, None, 4, 100, 1, fake, None, None) == _capi.MIVIT_EINVAL


def test_mfma_variant_rejections():
    """Variant 3 (radix 4 on the int8 matrix cores) takes int8 soft values,
    radix 4 and K = 7 rate-1/2 codes; anything else is refused at plan time."""
    fr = _frame()
    assert _plan_status([K7], fr, dtype=0, radix=4, variant=3) == _capi.MIVIT_EINVAL  # float radix 4
    assert _plan_status([K7], fr, dtype=1, radix=2, variant=3) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([_code(5, [0o23, 0o35])], fr, dtype=1, radix=4,
                        variant=3) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([_code(9, [0o557, 0o663, 0o711])], fr, dtype=1, radix=4,
                        variant=3) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K7], fr, dtype=1, radix=4, variant=9) == _capi.MIVIT_EINVAL
    # variant 4 (packed, one state per lane): int8 radix 4, K = 5 or 7 rate 1/2 only
    assert _plan_status([K7], fr, dtype=1, radix=2, variant=4) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([_code(9, [0o557, 0o663, 0o711])], fr, dtype=1, radix=4,
                        variant=4) == _capi.MIVIT_EUNSUPPORTED
    # variant 5 (packed, four states per lane): int8 radix 4, K = 7 rate 1/2 only
    assert _plan_status([K7], fr, dtype=1, radix=2, variant=5) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([_code(5, [0o23, 0o35])], fr, dtype=1, radix=4,
                        variant=5) == _capi.MIVIT_EUNSUPPORTED


def test_wide_wavefront_variant_rejections():
    """Variants 6 and 7 (two or four wavefronts per frame) take float32 soft
    values, radix 2 and codes with K >= 8 (6) or K = 9 (7); variant 8 (packed
    16-bit) takes int8, radix 2, K >= 8 and at most three outputs."""
    fr = _frame()
    K8 = _code(8, [0o247, 0o371])
    K9 = _code(9, [0o557, 0o663, 0o711])
    assert _plan_status([K7], fr, dtype=0, radix=2, variant=6) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K8], fr, dtype=0, radix=2, variant=7) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K9, K7], fr, dtype=0, radix=0, variant=6) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K9], fr, dtype=1, radix=2, variant=6) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K9], fr, dtype=2, radix=2, variant=7) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K9], fr, dtype=0, radix=4, variant=7) == _capi.MIVIT_EINVAL
    # variant 8 (two states per register, 16-bit): int8, radix 2, K >= 8, beta <= 3
    assert _plan_status([K9], fr, dtype=0, radix=2, variant=8) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K7], fr, dtype=1, radix=2, variant=8) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([K9], fr, dtype=1, radix=4, variant=8) == _capi.MIVIT_EUNSUPPORTED
    assert _plan_status([_code(9, [0o557, 0o663, 0o711, 0o755])], fr, dtype=1, radix=2,
                        variant=8) == _capi.MIVIT_EUNSUPPORTED


def test_plan_create_on_rejects_null_handle():
    """mivit_plan_create_on validates its output pointer before any device
    call (no GPU needed)."""
    lib = _capi.load()
    assert lib.mivit_plan_create_on(None, 0, None, 0, None, 0, None) == _capi.MIVIT_EINVAL
