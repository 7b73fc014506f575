"""Pins of the oracle's decoder against mathematics the paper fixes:
exhaustive maximum likelihood, error-free decoding of noiseless codewords,
path-metric certificates, the bounded path-metric spread, radix-4 = radix-2 in
exact integers, the chunked special cases, the runner-up gap and the gradient.
CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import bruteforce
from workload import CODE_K5, CODE_K7, CODE_K9, Code, make_uniform_batch, make_stream, transmit

SMALL_CODES = [
    Code.from_octal(3, ["7", "5"]),
    Code.from_octal(4, ["17", "13"]),
    CODE_K5,
    CODE_K7,
    Code.from_octal(4, ["17", "15", "13"]),
    Code.from_octal(5, ["25", "33", "37"]),
]
ids = lambda c: "K%d_" % c.K + "_".join("%o" % g for g in c.gens)


def tie_heavy(rng, n):
    return rng.integers(-2, 3, size=n).astype(np.int8)


@pytest.mark.parametrize("code", SMALL_CODES, ids=ids)
def test_bruteforce_int_exact_with_ties(code):
    """Viterbi (radix-2, exact ints) = exhaustive ML with the colex tie rule."""
    rng = np.random.default_rng(100 + code.K)
    for trial in range(40):
        n = int(rng.integers(1, 11))
        S = n + code.K - 1
        l = tie_heavy(rng, S * code.beta)
        bb, mb = bruteforce.ml_decode(code, l, n, exact_int=True)
        ob, om, _ = oracle.decode_uniform(code, l[None], n, True, oracle.I64)
        assert np.array_equal(ob[0], bb), (trial, n)
        assert int(om[0]) == int(mb)


@pytest.mark.parametrize("code", SMALL_CODES[:4], ids=ids)
def test_bruteforce_unterminated_and_unknown_start(code):
    rng = np.random.default_rng(200 + code.K)
    beta = code.beta
    for trial in range(30):
        n = int(rng.integers(1, 10))
        l = tie_heavy(rng, n * beta)
        # known start, free end
        fr = np.zeros(1, oracle.FRAME_DTYPE)
        fr[0] = (0, 0, n, 0, n, 1, -1, 0)
        ob, om, _, _ = oracle.decode_frames([code], fr, l, oracle.I64, n)
        bb, mb = bruteforce.ml_decode(code, l, n, terminated=False, exact_int=True)
        assert np.array_equal(ob, bb) and int(om[0]) == int(mb)
        # unknown start (all-zero initial metrics), free end
        fr[0] = (0, 0, n, 0, n, 0, -1, 0)
        ob, om, _, _ = oracle.decode_frames([code], fr, l, oracle.I64, n)
        bb, mb = bruteforce.ml_decode(code, l, n, terminated=False, known_start=False, exact_int=True)
        assert np.array_equal(ob, bb) and int(om[0]) == int(mb)


@pytest.mark.parametrize("code", SMALL_CODES, ids=ids)
def test_bruteforce_float(code):
    """fp64 and fp32 modes on continuous soft values (no ties)."""
    rng = np.random.default_rng(300 + code.K)
    for trial in range(20):
        n = int(rng.integers(1, 12))
        S = n + code.K - 1
        l = rng.normal(0, 2, S * code.beta).astype(np.float32)
        bb, mb = bruteforce.ml_decode(code, l, n)
        for mode in (oracle.F64, oracle.F32):
            ob, om, _ = oracle.decode_uniform(code, l[None], n, True, mode)
            assert np.array_equal(ob[0], bb)
            assert abs(float(om[0]) - mb) <= 1e-5 * max(1.0, abs(mb))


@pytest.mark.parametrize("code", [CODE_K5, CODE_K7, CODE_K9], ids=ids)
def test_noiseless(code):
    rng = np.random.default_rng(11)
    for n in (1, 7, 100):
        m = rng.integers(0, 2, n, dtype=np.uint8)
        c = oracle.encode(code, m, True).reshape(-1)
        S = n + code.K - 1
        for A in (1, 5, 127):
            l = (A * (1 - 2 * c.astype(np.int64))).astype(np.int8)
            for mode in (oracle.I64, oracle.R4_I64):
                ob, om, _ = oracle.decode_uniform(code, l[None], n, True, mode)
                assert np.array_equal(ob[0], m)
                assert int(om[0]) == code.beta * S * A
            lf = l.astype(np.float32) * 0.37
            for mode in (oracle.F64, oracle.F32):
                ob, om, _ = oracle.decode_uniform(code, lf[None], n, True, mode)
                assert np.array_equal(ob[0], m)


def test_certificates_awgn():
    """M(u_hat) >= M(m_true) and M(u_hat) is the correlation of its codeword."""
    for code in (CODE_K5, CODE_K7, CODE_K9):
        b = make_uniform_batch(code, 8, 300, 1.0, seed=5)
        ob, om, _ = oracle.decode_uniform(code, b.llr, 300, True, oracle.F64)
        for f in range(8):
            mt = oracle.path_correlation(code, b.msg[f], b.llr[f])
            mh = oracle.path_correlation(code, ob[f], b.llr[f])
            assert om[f] >= mt - 1e-9 * abs(mt)
            assert abs(mh - om[f]) <= 1e-9 * abs(om[f])
        q = oracle.quantize_i8(b.llr, 8.0)
        ob, om, _ = oracle.decode_uniform(code, q, 300, True, oracle.I64)
        for f in range(8):
            assert oracle.path_correlation(code, ob[f], q[f], exact_int=True) == int(om[f])
            assert int(om[f]) >= oracle.path_correlation(code, b.msg[f], q[f], exact_int=True)


@pytest.mark.parametrize("code", [CODE_K5, CODE_K7, CODE_K9], ids=ids)
def test_spread_invariant(code):
    """max_j PM_j - min_j PM_j <= 2 (K-1) beta L once every state is reachable
    (any state reaches any other in K-1 steps, each worth at most beta*L)."""
    rng = np.random.default_rng(17)
    L = 127
    bound = 2 * (code.K - 1) * code.beta * L
    worst = 0
    for trial in range(6):
        S = 3000
        l = rng.integers(-L, L + 1, size=S * code.beta).astype(np.int8)
        if trial % 2:
            l = np.sign(l).astype(np.int8) * L  # saturated, worst magnitude
        sp = oracle.forward_spread_i64(code, l, S, True)
        assert sp[code.K - 2:].max() <= bound
        sp0 = oracle.forward_spread_i64(code, l, S, False)
        assert sp0.max() <= bound
        worst = max(worst, int(sp.max()))
    assert worst > 0


@pytest.mark.parametrize("code", SMALL_CODES + [CODE_K9], ids=ids)
def test_radix4_equals_radix2_exact(code):
    """Eq. (radix4:PM) with smallest-y ties = radix-2 with lower-predecessor ties."""
    rng = np.random.default_rng(400 + code.K)
    for trial in range(25):
        n = int(rng.integers(0, 60))
        S = n + code.K - 1
        l = tie_heavy(rng, S * code.beta) if trial % 2 else rng.integers(-127, 128, S * code.beta).astype(np.int8)
        b2, m2, _ = oracle.decode_uniform(code, l[None], n, True, oracle.I64)
        b4, m4 = oracle.decode_r4(code, l[None], n, True)
        assert np.array_equal(b2, b4), (trial, n)
        assert int(m2[0]) == int(m4[0])
    # free end, unknown start
    for trial in range(10):
        n = int(rng.integers(1, 40))
        l = tie_heavy(rng, n * code.beta)
        for sk in (0, 1):
            fr = np.zeros(1, oracle.FRAME_DTYPE)
            fr[0] = (0, 0, n, 0, n, sk, -1, 0)
            r2 = oracle.decode_frames([code], fr, l, oracle.I64, n)
            r4 = oracle.decode_frames([code], fr, l, oracle.R4_I64, n)
            assert np.array_equal(r2[0], r4[0]) and r2[1][0] == r4[1][0]


def test_chunked_special_cases():
    code = CODE_K7
    msg, llr = make_stream(code, 5000, 2.0, seed=9)
    q = oracle.quantize_i8(llr, 16 * 0.5 / 10 ** 0.2)
    whole, _ = oracle.decode_stream_whole(code, q, 5000)
    # overlap covering the whole stream: every window is the whole stream
    ch, _, _ = oracle.decode_chunked(code, q, 5000, 512, 5000)
    assert np.array_equal(ch, whole)
    # one chunk bigger than the stream
    ch, _, _ = oracle.decode_chunked(code, q, 5000, 8192, 64)
    assert np.array_equal(ch, whole)
    # noiseless chunked decoding returns the message
    c = oracle.encode(code, msg, False).reshape(-1)
    ln = (40 * (1 - 2 * c.astype(np.int64))).astype(np.int8)
    ch, _, _ = oracle.decode_chunked(code, ln, 5000, 256, 64)
    assert np.array_equal(ch, msg)
    # windows tile the stream exactly
    wins = oracle.chunk_windows(5000, 2048, 64)
    assert [w[2] for w in wins] == [0, 2048, 4096] and wins[-1][3] == 5000
    assert wins[1][:2] == (2048 - 64, 4096 + 64)


def test_runner_up_gap():
    """Gap formula = best minus second-best over all messages (brute force)."""
    rng = np.random.default_rng(23)
    for code in SMALL_CODES[:4]:
        for trial in range(25):
            n = int(rng.integers(1, 10))
            S = n + code.K - 1
            l = rng.normal(0, 1.5, S * code.beta).astype(np.float32)
            _, om, gap = oracle.decode_uniform(code, l[None], n, True, oracle.F64, want_gap=True)
            best, second = bruteforce.best_two(code, l, n)
            if n == 0 or not np.isfinite(second):
                continue
            assert abs((best - second) - gap[0]) <= 1e-9 * max(1.0, abs(best))


def test_gradient_finite_differences():
    """Central differences of the fp64 best metric equal (-1)^{c(u_hat)} on
    frames whose runner-up gap exceeds twice the step.  The oracle reads
    float32 soft values, so the step actually taken is the float32-rounded
    one, and the quotient uses that exact step."""
    code = CODE_K7
    n = 64
    b = make_uniform_batch(code, 6, n, 2.0, seed=31)
    h = 1e-4
    bits, m0, gap = oracle.decode_uniform(code, b.llr, n, True, oracle.F64, want_gap=True)
    S = n + code.K - 1
    rng = np.random.default_rng(1)
    checked = 0
    for f in range(6):
        if gap[f] <= 1e-2:
            continue
        g = oracle.metric_grad(code, bits[f], 1.0)
        for k in rng.choice(S * 2, size=24, replace=False):
            lp = b.llr[f].copy()
            lm = b.llr[f].copy()
            lp[k] = np.float32(np.float64(lp[k]) + h)
            lm[k] = np.float32(np.float64(lm[k]) - h)
            _, mp, _ = oracle.decode_uniform(code, lp[None], n, True, oracle.F64)
            _, mm, _ = oracle.decode_uniform(code, lm[None], n, True, oracle.F64)
            fd = (float(mp[0]) - float(mm[0])) / (np.float64(lp[k]) - np.float64(lm[k]))
            assert abs(fd - g[k]) < 1e-6
            checked += 1
    assert checked > 0


def _union_bound(ebn0_db, spec, rate):
    ebn0 = 10 ** (ebn0_db / 10)
    return sum(c * 0.5 * math.erfc(math.sqrt(d * rate * ebn0))
               for d, c in zip(spec["d"], spec["c_d"]))


def test_ber_against_union_bound():
    """Monte-Carlo BER of the fp64 oracle sits at or below the union bound of
    the textbook spectrum, with at least 100/n-valid error counts (§IX-B)."""
    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "textbook_spectra.json")))["K7_133_171"]
    for eb, nf in ((3.0, 600), (3.5, 1200)):
        b = make_uniform_batch(CODE_K7, nf, 2048, eb, seed=77)
        bits, _, _ = oracle.decode_uniform(CODE_K7, b.llr, 2048, True, oracle.F64)
        errs = int((bits != b.msg).sum())
        nbits = b.msg.size
        ber = errs / nbits
        bound = _union_bound(eb, spec, 0.5)
        assert errs >= 100, "too few errors for a valid BER point"
        assert ber <= 1.3 * bound
        assert ber >= bound / 20


def test_quantizer_pins():
    """q = saturate_127(round_half_even(fl32(l * s))), values worked by hand:
    halves go to the even neighbour, magnitudes past 127 saturate (never to
    -128), infinities saturate, NaN maps to 0."""
    x = np.array([0.5, 1.5, 2.5, -2.5, 3.5, -0.5, 0.49999997, 126.5, 127.49, 127.5, 128.0,
                  1000.0, -1000.0, np.inf, -np.inf, np.nan, 0.0, -0.0], np.float32)
    want = np.array([0, 2, 2, -2, 4, 0, 0, 126, 127, 127, 127, 127, -127, 127, -127, 0, 0, 0],
                    np.int8)
    np.testing.assert_array_equal(oracle.quantize_i8(x, 1.0), want)
    # the product is rounded to float32 before rounding to an integer:
    # 0.1f * 25 = 2.5000000372529 in exact arithmetic, 2.5f after rounding -> 2
    np.testing.assert_array_equal(oracle.quantize_i8(np.array([0.1], np.float32), 25.0), [2])
    # scale 4: 0.375 -> 1.5 -> 2, 0.625 -> 2.5 -> 2, -0.875 -> -3.5 -> -4
    np.testing.assert_array_equal(
        oracle.quantize_i8(np.array([0.375, 0.625, -0.875], np.float32), 4.0), [2, 2, -4])


def test_mixed_codes_one_call():
    """Frames of different codes (16 to 256 states, long frames first) in one
    call decode exactly as each code's frames decoded alone."""
    from workload import CODE_K5, CODE_K9, make_mixed_batch
    codes = [CODE_K5, CODE_K7, CODE_K9]
    mb = make_mixed_batch(codes, 60, 64, 1500, 1.0, 5.0, seed=21)
    n = mb.n_info.astype(np.int64)
    K = np.array([codes[c].K for c in mb.code_idx])
    fr = np.zeros(len(n), oracle.FRAME_DTYPE)
    for f in range(len(n)):
        fr[f] = (mb.llr_offset[f], mb.bit_offset[f], n[f] + K[f] - 1, 0, n[f], 1, 0, mb.code_idx[f])
    order = np.argsort(-(n + K))  # long K=5 frames before short K=9 frames
    fr = fr[order]
    q = oracle.quantize_i8(mb.llr, 6.0)
    n_bits = int(mb.bit_offset.max() + 2048)
    for threads in (1, 3):
        bits, metric, _, _ = oracle.decode_frames(codes, fr, q, oracle.I64, n_bits, n_threads=threads)
        for c in range(3):
            sel = fr["code"] == c
            sub = fr[sel].copy()
            sub["code"] = 0
            b1, m1, _, _ = oracle.decode_frames([codes[c]], sub, q, oracle.I64, n_bits, n_threads=1)
            np.testing.assert_array_equal(metric[sel], m1)
            for row in sub:
                a, k = int(row["bit_offset"]), int(row["n_out"])
                np.testing.assert_array_equal(bits[a:a + k], b1[a:a + k])


def test_stored_fp64_ber_counts():
    """The stored double-precision error counts of the equal-BER sweep
    (tests/golden/ber_fp64_k7_4096x8192.json, written by make_ber_fp64.py)
    fall with Eb/N0, sit below the K=7 union bound from 4 dB up (the bound
    is loose below), and the 4 dB point is reproduced by the oracle."""
    import math
    from workload import make_uniform_batch
    path = os.path.join(os.path.dirname(__file__), "golden", "ber_fp64_k7_4096x8192.json")
    pts = json.load(open(path))["points"]
    assert [p["ebn0_db"] for p in pts] == list(range(7))
    errs = [p["f64_errors"] for p in pts]
    assert all(a >= b for a, b in zip(errs, errs[1:]))
    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "textbook_spectra.json")))["K7_133_171"]
    for p in pts:
        if p["ebn0_db"] < 4:
            continue
        ebn0 = 10 ** (p["ebn0_db"] / 10)
        bound = sum(c * 0.5 * math.erfc(math.sqrt(d * 0.5 * ebn0)) for d, c in zip(spec["d"], spec["c_d"]))
        assert p["f64_errors"] / p["bits"] <= bound
    p4 = pts[4]
    b = make_uniform_batch(CODE_K7, 4096, 8192, 4.0, seed=2004)
    bits, _, _ = oracle.decode_uniform(CODE_K7, b.llr, 8192, True, oracle.F64)
    assert int((bits != b.msg).sum()) == p4["f64_errors"]


@pytest.mark.parametrize("code,ns", [(CODE_K7, (13, 14, 15, 16)), (CODE_K5, (14, 16)),
                                     (CODE_K9, (10, 11, 12))], ids=["K7", "K5", "K9_r13"])
def test_bruteforce_long_frames_with_ties(code, ns):
    """Exhaustive ML over every message of the longest frames the search
    covers (2^16 messages for K=7 and K=5, 2^12 for K=9 rate 1/3), tie-heavy
    int8 soft values and continuous ones: the exact-integer radix-2 oracle,
    the literal radix-4 recursion and the double-precision oracle return the
    brute-force message (smallest under the colex rule on ties) and metric."""
    rng = np.random.default_rng(900 + code.K)
    for n in ns:
        S = n + code.K - 1
        for trial in range(2):
            l = tie_heavy(rng, S * code.beta)
            bb, mb = bruteforce.ml_decode(code, l, n, exact_int=True)
            for mode in (oracle.I64, oracle.R4_I64):
                ob, om, _ = oracle.decode_uniform(code, l[None], n, True, mode)
                assert np.array_equal(ob[0], bb), (n, trial, mode)
                assert int(om[0]) == int(mb)
        x = rng.normal(0, 2, S * code.beta).astype(np.float32)
        bb, mb = bruteforce.ml_decode(code, x, n)
        ob, om, _ = oracle.decode_uniform(code, x[None], n, True, oracle.F64)
        assert np.array_equal(ob[0], bb)
        assert abs(float(om[0]) - mb) <= 1e-9 * max(1.0, abs(mb))
