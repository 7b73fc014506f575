"""Transmitter and AWGN channel of the verification system (§IX-B), seeded.

Conventions (stated once, used by every caller):

* A code is (K, beta, generators).  Generator ``g`` is a K-bit tap mask whose
  bit K-1 multiplies the current input bit and bit 0 the input K-1 stages
  back, as in the encoder equation of §II-A.  Output bit ``b`` of a stage uses
  the ``b``-th generator in the order the code lists them.
* Message bits are drawn first, then the noise, from one
  ``numpy.random.default_rng(seed)`` stream per workload.
* BPSK maps coded bit 0 to +1 and 1 to -1.  The noise variance is
  sigma^2 = 1 / (2 R 10^(EbN0/10)) with R = 1/beta; the soft value handed to
  the decoder is LLR = 2 y / sigma^2 (positive favours bit 0, §II-C), stored
  as float32, time-major: stage t occupies elements [t*beta, (t+1)*beta).

The encoder here is the transmitter of the simulated link; the CPU oracle
carries its own, independent encoder, and a test checks the two agree.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np


@dataclass(frozen=True)
class Code:
    K: int
    gens: tuple  # generator tap masks, one per output bit

    @property
    def beta(self) -> int:
        return len(self.gens)

    @property
    def n_states(self) -> int:
        return 1 << (self.K - 1)

    @staticmethod
    def from_octal(K: int, gens_octal: Sequence[str]) -> "Code":
        return Code(K, tuple(int(str(g), 8) for g in gens_octal))


CODE_K5 = Code.from_octal(5, ["23", "35"])
CODE_K7 = Code.from_octal(7, ["133", "171"])
CODE_K9 = Code.from_octal(9, ["557", "663", "711"])


def sigma2_for(ebn0_db: float, beta: int) -> float:
    """Noise variance per real dimension for unit-energy BPSK at rate 1/beta."""
    rate = 1.0 / beta
    return 1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))


def int8_scale_for(ebn0_db: float, beta: int) -> float:
    """Scale that maps LLR = 2y/sigma^2 onto 32*y before int8 rounding."""
    return 16.0 * sigma2_for(ebn0_db, beta)


def encode_bits(code: Code, msg: np.ndarray, terminate: bool = True) -> np.ndarray:
    """Encode message rows.  msg: uint8 [..., N] -> coded uint8 [..., S, beta].

    S = N + K - 1 when ``terminate`` (K-1 zero tail bits appended), else N.
    The encoder starts in the all-zero state.
    """
    msg = np.asarray(msg, dtype=np.uint8)
    K = code.K
    if terminate:
        pad = np.zeros(msg.shape[:-1] + (K - 1,), dtype=np.uint8)
        x = np.concatenate([msg, pad], axis=-1)
    else:
        x = msg
    S = x.shape[-1]
    # history[..., t, k] = input bit at t - (K-1-k) (zero before the start)
    hist = np.zeros(x.shape[:-1] + (K - 1,), dtype=np.uint8)
    xp = np.concatenate([hist, x], axis=-1)  # xp[..., t + K - 1] = x[..., t]
    out = np.zeros(x.shape[:-1] + (S, code.beta), dtype=np.uint8)
    for b, g in enumerate(code.gens):
        acc = np.zeros(x.shape[:-1] + (S,), dtype=np.uint8)
        for k in range(K):
            if (g >> k) & 1:
                # tap k multiplies the input K-1-k stages back
                lag = K - 1 - k
                acc ^= xp[..., K - 1 - lag: K - 1 - lag + S]
        out[..., b] = acc
    return out


def transmit(code: Code, msg: np.ndarray, noise: np.ndarray, ebn0_db,
             terminate: bool = True) -> np.ndarray:
    """Encode, BPSK-modulate, add sigma*noise, return float32 LLRs [..., S*beta].

    ``noise`` has the shape of the coded stream [..., S*beta] (standard
    normal draws).  ``ebn0_db`` is a scalar or one value per leading row.
    """
    coded = encode_bits(code, msg, terminate)
    shp = coded.shape[:-2] + (coded.shape[-2] * coded.shape[-1],)
    x = 1.0 - 2.0 * coded.reshape(shp).astype(np.float64)
    s2 = np.vectorize(lambda e: sigma2_for(float(e), code.beta))(np.asarray(ebn0_db, dtype=np.float64))
    s2 = np.asarray(s2, dtype=np.float64)
    if s2.ndim:
        s2 = s2.reshape(s2.shape + (1,) * (x.ndim - s2.ndim))
    y = x + np.sqrt(s2) * noise
    return (2.0 * y / s2).astype(np.float32)


@dataclass
class Batch:
    """A batch of independent frames plus everything needed to check it."""
    code: Code
    msg: np.ndarray            # uint8 [F, N]
    llr: np.ndarray            # float32 [F, S*beta]
    ebn0_db: float
    terminated: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def n_frames(self) -> int:
        return self.msg.shape[0]

    @property
    def n_info(self) -> int:
        return self.msg.shape[1]

    @property
    def n_stages(self) -> int:
        return self.n_info + (self.code.K - 1 if self.terminated else 0)


def make_uniform_batch(code: Code, n_frames: int, n_info: int, ebn0_db: float,
                       seed: int, terminated: bool = True) -> Batch:
    """Equal-length frames (the single-frame and the 4096-frame workloads)."""
    rng = np.random.default_rng(seed)
    msg = rng.integers(0, 2, size=(n_frames, n_info), dtype=np.uint8)
    S = n_info + (code.K - 1 if terminated else 0)
    noise = rng.standard_normal(size=(n_frames, S * code.beta))
    llr = transmit(code, msg, noise, ebn0_db, terminated)
    return Batch(code, msg, llr, ebn0_db, terminated)


def make_stream(code: Code, n_info: int, ebn0_db: float, seed: int):
    """One continuous, unterminated stream starting in state 0.

    Returns (msg uint8 [N], llr float32 [N*beta]).
    """
    rng = np.random.default_rng(seed)
    msg = rng.integers(0, 2, size=(n_info,), dtype=np.uint8)
    noise = rng.standard_normal(size=(n_info * code.beta,))
    llr = transmit(code, msg, noise, ebn0_db, terminate=False)
    return msg, llr


@dataclass
class MixedBatch:
    """Frames of uneven length and mixed codes, packed back to back."""
    codes: list                # list[Code]
    code_idx: np.ndarray       # int32 [F]
    n_info: np.ndarray         # int32 [F]
    ebn0_db: np.ndarray        # float64 [F]
    msgs: list                 # list of uint8 [N_f]
    llr: np.ndarray            # float32, all frames concatenated
    llr_offset: np.ndarray     # int64 [F]: element index of each frame's stage 0
    bit_offset: np.ndarray     # int64 [F]: output bit index, multiple of 32

    @property
    def n_frames(self) -> int:
        return len(self.msgs)


def make_mixed_batch(codes: Sequence[Code], n_frames: int, n_min: int, n_max: int,
                     ebn0_lo: float, ebn0_hi: float, seed: int) -> MixedBatch:
    """Log-uniform lengths in [n_min, n_max], code uniform over ``codes``,
    Eb/N0 uniform in [ebn0_lo, ebn0_hi]; all frames terminated.

    Draw order: lengths, code indices, Eb/N0 values, then per frame (in frame
    order) its message bits followed by its noise.
    """
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_frames))).astype(np.int32)
    n = np.clip(n, n_min, n_max)
    cidx = rng.integers(0, len(codes), size=n_frames).astype(np.int32)
    eb = rng.uniform(ebn0_lo, ebn0_hi, size=n_frames)
    msgs, llrs = [], []
    llr_off = np.zeros(n_frames, dtype=np.int64)
    bit_off = np.zeros(n_frames, dtype=np.int64)
    pos = 0
    bpos = 0
    for f in range(n_frames):
        c = codes[int(cidx[f])]
        m = rng.integers(0, 2, size=(int(n[f]),), dtype=np.uint8)
        S = int(n[f]) + c.K - 1
        z = rng.standard_normal(size=(S * c.beta,))
        llrs.append(transmit(c, m, z, float(eb[f]), terminate=True))
        msgs.append(m)
        llr_off[f] = pos
        bit_off[f] = bpos
        pos += S * c.beta
        bpos += ((int(n[f]) + 31) // 32) * 32
    llr = np.concatenate(llrs).astype(np.float32)
    return MixedBatch(list(codes), cidx, n, eb, msgs, llr, llr_off, bit_off)
