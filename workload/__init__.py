"""Seeded synthetic inputs for the Viterbi decoder: the transmitter side only.

This package is the single source of inputs shared by the GPU decoder, the CPU
oracle, the tests and the benchmark.  It holds the random draws (message bits,
Gaussian noise) and the simulated transmitter and channel of the paper's
verification system (§IX-B: uniform bits -> convolutional encoder -> BPSK over
AWGN -> soft values).  It contains no part of the decoder: no branch metric,
no add-compare-select, no traceback and no quantiser.
"""
from .channel import (  # noqa: F401
    Code,
    CODE_K5,
    CODE_K7,
    CODE_K9,
    sigma2_for,
    int8_scale_for,
    transmit,
    encode_bits,
    make_uniform_batch,
    make_stream,
    make_mixed_batch,
)
