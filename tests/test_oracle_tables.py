"""Pins of the oracle's trellis tables against facts the paper prints and
against textbook properties of the three codes.  CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from workload import CODE_K5, CODE_K7, CODE_K9, Code

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLD, "paper_structure.json")))
SPECTRA = json.load(open(os.path.join(GOLD, "textbook_spectra.json")))

# The paper lists (171, 133); the K=7 workloads list (133, 171).  Structural
# facts do not depend on the order; both are exercised.
K7_PAPER = Code.from_octal(7, ["171", "133"])
ALL_CODES = [CODE_K5, CODE_K7, K7_PAPER, CODE_K9]


def test_generator_binary_forms():
    g = PAPER["generators_binary"]
    assert format(int("171", 8), "07b") == g["171"]
    assert format(int("133", 8), "07b") == g["133"]


@pytest.mark.parametrize("code", ALL_CODES, ids=lambda c: "K%d_b%d" % (c.K, c.beta))
def test_butterfly_index_map(code):
    """Eq. (radix2:S): states 2f, 2f+1 both lead to f and f + 2^(K-2)."""
    nxt, _, prv = oracle.trellis(code)
    K = code.K
    for f in range(1 << (K - 2)):
        for i in (2 * f, 2 * f + 1):
            assert nxt[i, 0] == f
            assert nxt[i, 1] == f + (1 << (K - 2))
        assert list(prv[f]) == [2 * f, 2 * f + 1]
        assert list(prv[f + (1 << (K - 2))]) == [2 * f, 2 * f + 1]


@pytest.mark.parametrize("code", ALL_CODES, ids=lambda c: "K%d_b%d" % (c.K, c.beta))
def test_outer_inner_corollary(code):
    """Eq. (radix2:boRelatNot): outer branches equal, inner = complement."""
    K = code.K
    for g in code.gens:
        assert (g >> (K - 1)) & 1 and g & 1  # premise holds for all three codes
    nxt, out, _ = oracle.trellis(code)
    full = (1 << code.beta) - 1
    for f in range(1 << (K - 2)):
        i0, i1 = 2 * f, 2 * f + 1
        a00, a01 = out[i0, 0], out[i0, 1]
        a10, a11 = out[i1, 0], out[i1, 1]
        assert a00 == a11
        assert a01 == a10 == (a00 ^ full)


def test_output_relation_general():
    """Eqs. (radix2:boRelatBegin..End): every branch output of a butterfly is
    the main one XOR the taps on the input bit and on the state LSB."""
    code = Code.from_octal(7, ["155", "117"])  # MSB set, LSB set only for the second
    K = code.K
    _, out, _ = oracle.trellis(code)
    msb = sum((((g >> (K - 1)) & 1) << b) for b, g in enumerate(code.gens))
    lsb = sum(((g & 1) << b) for b, g in enumerate(code.gens))
    for f in range(1 << (K - 2)):
        i0, i1 = 2 * f, 2 * f + 1
        base = out[i0, 0]
        assert out[i0, 1] == base ^ msb
        assert out[i1, 0] == base ^ lsb
        assert out[i1, 1] == base ^ msb ^ lsb


def _theta(code, f):
    """Theta_f of Eq. (radix2:branchOutMat): rows (i0,j0),(i1,j0),(i0,j1),(i1,j1)."""
    _, out, _ = oracle.trellis(code)
    rows = [out[2 * f, 0], out[2 * f + 1, 0], out[2 * f, 1], out[2 * f + 1, 1]]
    return tuple(tuple(1 - 2 * ((w >> b) & 1) for b in range(code.beta)) for w in rows)


@pytest.mark.parametrize("code", [CODE_K7, K7_PAPER], ids=["133_171", "171_133"])
def test_theta_classes_k7(code):
    fact = PAPER["theta_classes_k7"]
    thetas = [_theta(code, f) for f in range(1 << (code.K - 2))]
    assert len(thetas) == fact["n_butterflies"]
    uniq = {}
    for t in thetas:
        uniq[t] = uniq.get(t, 0) + 1
    assert len(uniq) == fact["n_classes"] == 2 ** code.beta
    assert set(uniq.values()) == {fact["per_class"]}


def test_q_counts():
    K = PAPER["q_radix2_16x16"]["K"]
    assert (1 << (K - 2)) // 16 == PAPER["q_radix2_16x16"]["Q"] == 2 ** (K - 6)
    # one 16x16 op per two stages for the whole trellis
    assert 1 / 2 == PAPER["q_dragonfly_groups"]["Q"]


@pytest.mark.parametrize("code", ALL_CODES, ids=lambda c: "K%d_b%d" % (c.K, c.beta))
def test_radix4_index_map(code):
    """Eq. (radix4:S): i_y = 4f+y reach m and then j_z = f + z 2^(K-3)."""
    nxt, _, _ = oracle.trellis(code)
    K = code.K
    for f in range(1 << (K - 3)):
        lefts = [4 * f + y for y in range(4)]
        mids = {2 * f, 2 * f + 1, 2 * f + (1 << (K - 2)), 2 * f + (1 << (K - 2)) + 1}
        rights = {f + z * (1 << (K - 3)) for z in range(4)}
        m_reached = {nxt[i, u] for i in lefts for u in (0, 1)}
        assert m_reached == mids
        j_reached = {nxt[m, u] for m in mids for u in (0, 1)}
        assert j_reached == rights
        # exactly one two-stage path between every left and right state (§VII, Theorem)
        for i in lefts:
            ends = [nxt[nxt[i, a], b] for a in (0, 1) for b in (0, 1)]
            assert sorted(ends) == sorted(rights)


def _bits(x, b, a):
    """The bit operator of Eq. (bit): x_{b:a} = bits a+1..b (1-based) of x."""
    return (x >> a) % (1 << (b - a))


def test_bit_operator_example():
    ex = PAPER["bit_operator_example"]
    assert _bits(ex["x"], 4, 1) == ex["x_4_1"]
    assert _bits(ex["x"], 4, 0) == ex["x_4_0"]


def _general_state(K, rho, f, y, x, corrected=True):
    """Eq. (general:S).  The printed post-bubble term y_{rho-x-1:0} is one bit
    short under the operator above; the corrected form keeps rho-x bits."""
    pre = _bits(y, rho, rho - x) << (K - x - 1)
    bub = f << (rho - x)
    post = _bits(y, rho - x, 0) if corrected else _bits(y, max(rho - x - 1, 0), 0)
    return pre + bub + post


@pytest.mark.parametrize("code", ALL_CODES, ids=lambda c: "K%d_b%d" % (c.K, c.beta))
def test_general_state_formula(code):
    K = code.K
    nxt, _, _ = oracle.trellis(code)
    for rho in range(1, K - 1):
        for f in range(1 << (K - 1 - rho)):
            for x in range(rho):
                here = {_general_state(K, rho, f, y, x) for y in range(1 << rho)}
                there = {_general_state(K, rho, f, y, x + 1) for y in range(1 << rho)}
                assert len(here) == 1 << rho
                assert {nxt[s, u] for s in here for u in (0, 1)} == there
    # rho = 2 reproduces Eq. (radix4:S)
    f = 3
    assert [_general_state(K, 2, f, y, 0) for y in range(4)] == [4 * f + y for y in range(4)]
    assert [_general_state(K, 2, f, y, 1) for y in range(4)] == [
        2 * f, 2 * f + 1, 2 * f + (1 << (K - 2)), 2 * f + (1 << (K - 2)) + 1]
    assert [_general_state(K, 2, f, y, 2) for y in range(4)] == [f + y * (1 << (K - 3)) for y in range(4)]
    # the form as printed fails at the middle stage
    assert [_general_state(K, 2, f, y, 1, corrected=False) for y in range(4)] != [
        2 * f, 2 * f + 1, 2 * f + (1 << (K - 2)), 2 * f + (1 << (K - 2)) + 1]


def _theta_hat(code, f):
    """Super-branch matrix of dragonfly f (Eq. (radix4:branchOutMat)): row
    4z+y holds the 2*beta signs of the path i_y -> m -> j_z."""
    nxt, out, _ = oracle.trellis(code)
    K, beta = code.K, code.beta
    rows = []
    for z in range(4):
        j = f + z * (1 << (K - 3))
        for y in range(4):
            i = 4 * f + y
            for a in (0, 1):
                m = nxt[i, a]
                for b in (0, 1):
                    if nxt[m, b] == j:
                        word = out[i, a] | (out[m, b] << beta)
            rows.append(tuple(1 - 2 * ((word >> k) & 1) for k in range(2 * beta)))
    return tuple(rows)


@pytest.mark.parametrize("code", [CODE_K7, K7_PAPER], ids=["133_171", "171_133"])
def test_dragonflies_distinct_k7(code):
    fact = PAPER["dragonflies_k7_all_distinct"]
    mats = [_theta_hat(code, f) for f in range(1 << (code.K - 3))]
    assert len(mats) == fact["n_dragonflies"]
    assert len(set(mats)) == fact["n_distinct"] == 2 ** (2 * code.beta)


def _left_perm_equivalent(a, b):
    """True if b equals a with the left states (y) permuted identically in every
    right-rooted block P_j."""
    import itertools
    for perm in itertools.permutations(range(4)):
        if all(b[4 * z + y] == a[4 * z + perm[y]] for z in range(4) for y in range(4)):
            return perm
    return None


@pytest.mark.parametrize("code", [CODE_K7, K7_PAPER], ids=["133_171", "171_133"])
def test_dragonfly_groups_k7(code):
    mats = [_theta_hat(code, f) for f in range(16)]
    groups = []
    for f in range(16):
        for g in groups:
            if _left_perm_equivalent(mats[g[0]], mats[f]) is not None:
                g.append(f)
                break
        else:
            groups.append([f])
    want = [PAPER["dragonfly_groups_k7"]["DG%d" % k] for k in range(4)]
    assert sorted(groups) == sorted(want)
    # derived (figure not printed): the permutation is y -> y xor a
    for g in want:
        lead = g[0]
        for f, a in zip(g, (0, 1, 3, 2)):
            perm = _left_perm_equivalent(mats[lead], mats[f])
            assert perm == tuple(y ^ a for y in range(4))


def _spectrum(code, wmax):
    """Output-weight spectrum of paths leaving state 0 and first returning,
    by dynamic programming over the oracle's tables."""
    nxt, out, _ = oracle.trellis(code)
    ns = 1 << (code.K - 1)
    pc = [bin(int(w)).count("1") for w in range(1 << code.beta)]
    cnt = np.zeros((ns, wmax + 1), dtype=object)
    info = np.zeros((ns, wmax + 1), dtype=object)
    a = [0] * (wmax + 1)
    c = [0] * (wmax + 1)
    s1, w1 = nxt[0, 1], pc[out[0, 1]]
    cnt[s1, w1] += 1
    info[s1, w1] += 1
    for _ in range(400):
        ncnt = np.zeros_like(cnt)
        ninfo = np.zeros_like(info)
        live = False
        for s in range(1, ns):
            for w in range(wmax + 1):
                if cnt[s, w] == 0:
                    continue
                for u in (0, 1):
                    t, nw = nxt[s, u], w + pc[out[s, u]]
                    if nw > wmax:
                        continue
                    if t == 0:
                        a[nw] += cnt[s, w]
                        c[nw] += info[s, w] + u * cnt[s, w]
                    else:
                        ncnt[t, nw] += cnt[s, w]
                        ninfo[t, nw] += info[s, w] + u * cnt[s, w]
                        live = True
        cnt, info = ncnt, ninfo
        if not live:
            break
    return a, c


def test_textbook_spectrum_k7():
    ref = SPECTRA["K7_133_171"]
    a, c = _spectrum(CODE_K7, max(ref["d"]))
    d_free = min(d for d in range(len(a)) if a[d])
    assert d_free == ref["d_free"]
    assert [a[d] for d in ref["d"]] == ref["a_d"]
    assert [c[d] for d in ref["d"]] == ref["c_d"]
    # odd weights never occur for this code
    assert all(a[d] == 0 for d in range(1, len(a), 2))


@pytest.mark.parametrize("code,key", [(CODE_K5, "K5_23_35"), (CODE_K9, "K9_557_663_711")])
def test_textbook_spectrum_k5_k9(code, key):
    """Free distance, path counts a_d and information weights c_d of the
    first five distances of the other two codes."""
    ref = SPECTRA[key]
    a, c = _spectrum(code, max(ref["d"]))
    assert min(d for d in range(len(a)) if a[d]) == ref["d_free"]
    assert [a[d] for d in ref["d"]] == ref["a_d"]
    assert [c[d] for d in ref["d"]] == ref["c_d"]


@pytest.mark.parametrize("code", ALL_CODES, ids=lambda c: "K%d_b%d" % (c.K, c.beta))
def test_encoders_agree(code):
    """The transmitter's encoder (workload) and the oracle's are independent
    implementations of the encoder equation; they must agree."""
    from workload import encode_bits
    rng = np.random.default_rng(7)
    for n, term in [(0, True), (1, True), (37, True), (64, False), (200, True)]:
        m = rng.integers(0, 2, size=n, dtype=np.uint8)
        a = oracle.encode(code, m, term)
        b = encode_bits(code, m, term)
        assert a.shape == b.shape and np.array_equal(a, b)


def test_impulse_response_k7():
    """A single 1 into the encoder emits each generator MSB-first: for
    (133, 171) the pairs read 11 01 11 11 00 10 11 (weight 10 = d_free)."""
    m = np.zeros(1, np.uint8)
    m[0] = 1
    c = oracle.encode(CODE_K7, m, True)
    assert "".join("%d%d" % (x[0], x[1]) for x in c) == "11011111001011"
    assert int(c.sum()) == SPECTRA["K7_133_171"]["d_free"]


def test_encoder_linear_and_zero():
    rng = np.random.default_rng(3)
    for code in ALL_CODES:
        a = rng.integers(0, 2, 50, dtype=np.uint8)
        b = rng.integers(0, 2, 50, dtype=np.uint8)
        assert np.array_equal(oracle.encode(code, a ^ b), oracle.encode(code, a) ^ oracle.encode(code, b))
        assert not oracle.encode(code, np.zeros(50, np.uint8)).any()
