"""Exhaustive maximum-likelihood decoding for short frames (n <= 16).

TEST INFRASTRUCTURE ONLY.  An independent code path from the C oracle: it
enumerates every message, encodes it with its own vectorised shift register
(the encoder equation of §II-A), sums the correlation metric of Eq. (BM) over
the whole codeword and keeps the best.  Among messages with equal best metric
it returns the one whose integer value sum_t m_t 2^t is smallest: the rule that
the lower-predecessor tie break of Eq. (PM) produces (two paths merging at a
state differ last in the bit that leaves the register, so preferring the lower
predecessor prefers a 0 in the latest differing bit).
"""
from __future__ import annotations

import numpy as np


def _parity_table(K: int, gens) -> np.ndarray:
    """out[reg] = beta-bit output word of a K-bit register value."""
    regs = np.arange(1 << K, dtype=np.int64)
    out = np.zeros(1 << K, dtype=np.int64)
    for b, g in enumerate(gens):
        x = regs & int(g)
        p = np.zeros_like(x)
        while np.any(x):
            p ^= x & 1
            x >>= 1
        out |= p << b
    return out


def all_metrics(code, llr, n: int, terminated: bool = True, known_start: bool = True,
                exact_int: bool = False) -> np.ndarray:
    """Metric of every candidate, indexed by the integer value of its input bits.

    With ``known_start`` the candidates are the 2^n messages (register starts
    at zero).  Without it, K-1 extra oldest bits choose the start state and
    the index is (message << (K-1)) | start_bits, i.e. the start state bits
    are the oldest, least significant ones.
    """
    K, gens = int(code.K), list(code.gens)
    beta = len(gens)
    table = _parity_table(K, gens)
    S = n + (K - 1 if terminated else 0)
    pre = 0 if known_start else K - 1
    nv = 1 << (n + pre)
    v = np.arange(nv, dtype=np.int64)
    if pre:
        # start state = the K-1 oldest bits, oldest (stage -(K-1)) in the LSB
        start_bits = v & ((1 << pre) - 1)
        msg = v >> pre
        state = np.zeros(nv, dtype=np.int64)
        for k in range(pre):  # shift the prefix in, oldest first
            u = (start_bits >> k) & 1
            state = ((u << (K - 1)) | state) >> 1
    else:
        msg = v
        state = np.zeros(nv, dtype=np.int64)
    l = np.asarray(llr).reshape(S, beta)
    acc = np.zeros(nv, dtype=np.int64 if exact_int else np.float64)
    for t in range(S):
        u = (msg >> t) & 1 if t < n else np.zeros(nv, dtype=np.int64)
        reg = (u << (K - 1)) | state
        w = table[reg]
        for b in range(beta):
            sgn = 1 - 2 * ((w >> b) & 1)
            if exact_int:
                acc += sgn * int(l[t, b])
            else:
                acc += sgn.astype(np.float64) * float(l[t, b])
        state = reg >> 1
    if terminated:
        # the tail drives every register back to zero
        assert np.all(state == 0)
    return acc


def ml_decode(code, llr, n: int, terminated: bool = True, known_start: bool = True,
              exact_int: bool = False):
    """Best message bits (uint8 [n]) and its metric; ties -> smallest integer value."""
    m = all_metrics(code, llr, n, terminated, known_start, exact_int)
    best = int(np.argmax(m))  # first occurrence = smallest index
    pre = 0 if known_start else code.K - 1
    msgv = best >> pre
    bits = np.array([(msgv >> t) & 1 for t in range(n)], dtype=np.uint8)
    return bits, m[best]


def best_two(code, llr, n: int, terminated: bool = True, exact_int: bool = False):
    """(best metric, second-best metric over all other messages)."""
    m = all_metrics(code, llr, n, terminated, True, exact_int)
    k = int(np.argmax(m))
    best = m[k]
    m2 = np.delete(m, k)
    return best, (m2.max() if m2.size else -np.inf)
