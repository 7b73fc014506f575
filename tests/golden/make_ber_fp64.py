"""Write ber_fp64_k7_4096x8192.json: bit errors of the double-precision
oracle on the equal-BER sweep's batches (4096 terminated frames x 8192 info
bits, K=7 (133,171), BPSK/AWGN at 0..6 dB, seed 2000 + dB, the float32 soft
values the GPU decodes).  The benchmark's equal-BER sweep reads the counts
to state the int8 radix-4 decoder's loss against double precision.

Calls only the oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_ber_fp64.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workload import CODE_K7, make_uniform_batch  # noqa: E402

F, N = 4096, 8192


def main():
    pts = []
    for db in range(0, 7):
        t0 = time.perf_counter()
        b = make_uniform_batch(CODE_K7, F, N, float(db), seed=2000 + db)
        bits, _, _ = oracle.decode_uniform(CODE_K7, b.llr, N, True, oracle.F64)
        errs = int((bits != b.msg).sum())
        pts.append({"ebn0_db": db, "bits": int(b.msg.size), "f64_errors": errs})
        print("%d dB: %d errors (%.1f s)" % (db, errs, time.perf_counter() - t0), flush=True)
    out = {"_about": "Bit errors of the double-precision oracle (radix 2, ties to the lower "
                     "previous state) on the equal-BER sweep batches: %d terminated frames x %d "
                     "info bits, K=7 (133,171), seed 2000 + Eb/N0 in dB, BPSK over AWGN with "
                     "LLR = 2y/sigma^2 stored as float32.  Written by make_ber_fp64.py." % (F, N),
           "points": pts}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ber_fp64_k7_4096x8192.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
