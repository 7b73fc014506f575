"""mivit_decode_uniform_noalloc: the allocation-free one-call decode (its
tables and survivor memory live in the library's fixed device scratch
array) gives the same bits and metrics as mivit_decode_uniform, and as the
oracle, on two calls in a row, the second with a smaller batch; a batch
beyond the scratch array is refused before any launch."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2011_13579_amd as mv
from workload import CODE_K5, CODE_K7, CODE_K9, make_uniform_batch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _call(fn, t, dtc, cs, F, n, term, W, metric_dtype):
    bits = torch.full((F * W,), -1, dtype=torch.int32, device=DEV)
    metric = torch.zeros(F, dtype=metric_dtype, device=DEV)
    st = fn(t.data_ptr(), dtc, ctypes.byref(cs), F, n, term, bits.data_ptr(), metric.data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    assert st == mv._capi.MIVIT_OK, st
    torch.cuda.synchronize()
    return mv.unpack_bits(bits.cpu().numpy().reshape(F, W), n), metric.cpu().numpy()


@pytest.mark.parametrize("code,dtype", [(CODE_K7, "i8"), (CODE_K5, "i8"), (CODE_K7, "f32"),
                                        (CODE_K9, "f32"), (CODE_K9, "i8"), (CODE_K7, "f16")],
                         ids=["k7-i8", "k5-i8", "k7-f32", "k9-f32", "k9-i8", "k7-f16"])
def test_noalloc_matches_decode_uniform(code, dtype):
    lib = mv._capi.load()
    cs = mv.Code(code.K, tuple(code.gens)).c_struct()
    dtc = {"i8": mv.MIVIT_I8, "f32": mv.MIVIT_F32, "f16": mv.MIVIT_F16}[dtype]
    mdt = torch.int64 if dtype == "i8" else torch.float32
    # two calls in a row on the shared scratch, the second smaller
    for F, n, term in [(37, 2001, 1), (5, 300, 0)]:
        b = make_uniform_batch(code, F, n, 2.0, seed=8100 + F + n, terminated=bool(term))
        if dtype == "i8":
            x = oracle.quantize_i8(b.llr, 6.0)
            ref, mode = x, oracle.I64
        elif dtype == "f16":
            x = b.llr.astype(np.float16)
            ref, mode = x.astype(np.float32), oracle.F32
        else:
            x, ref, mode = b.llr, b.llr, oracle.F32
        t = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
        W = (n + 31) // 32
        print("noalloc", code.K, dtype, F, n, term, flush=True)
        got_b, got_m = _call(lib.mivit_decode_uniform_noalloc, t, dtc, cs, F, n, term, W, mdt)
        ref_b, ref_m = _call(lib.mivit_decode_uniform, t, dtc, cs, F, n, term, W, mdt)
        np.testing.assert_array_equal(got_b, ref_b)
        np.testing.assert_array_equal(got_m, ref_m)
        ob, om, _ = oracle.decode_uniform(code, ref, n, bool(term), mode)
        np.testing.assert_array_equal(got_b, ob)
        np.testing.assert_array_equal(got_m, om)


def test_noalloc_rejects_batches_beyond_scratch():
    """64 MiB of scratch: 4096 frames of 8192 K=7 stages need 269 MB of
    survivors, so the call returns MIVIT_ENOMEM and writes nothing."""
    lib = mv._capi.load()
    cs = mv.Code(CODE_K7.K, tuple(CODE_K7.gens)).c_struct()
    F, n = 4096, 8192
    t = torch.zeros(F * (n + 6) * 2, dtype=torch.int8, device=DEV)
    bits = torch.full((F * n // 32,), -1, dtype=torch.int32, device=DEV)
    st = lib.mivit_decode_uniform_noalloc(t.data_ptr(), mv.MIVIT_I8, ctypes.byref(cs), F, n, 1,
                                          bits.data_ptr(), None,
                                          torch.cuda.current_stream().cuda_stream)
    assert st == mv._capi.MIVIT_ENOMEM
    torch.cuda.synchronize()
    assert bool((bits == -1).all())
