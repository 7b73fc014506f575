"""Compile the HIP library libmivit.so in-tree for gfx950 with hipcc.

Each source compiles to its own object in parallel (one hipcc per source),
then one link step makes the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmivit.so")
SOURCES = ["mivit_kernels.hip", "mivit_fwd_rot.hip", "mivit_traceback.hip", "mivit_r4p.hip",
           "mivit_fwd_wide.hip", "mivit_api.cpp", "mivit_pipe.cpp", "mivit_noalloc.hip",
           "mivit_r4_mfma.hip"]
ARCH = os.environ.get("MIVIT_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=%s" % ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # keep the device compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _filter(stderr: str):
    # the host pass warns that it does not know the packed-fp32 feature
    return [ln for ln in stderr.splitlines() if "not a recognized feature" not in ln]


def _compile(src: str, obj: str):
    cmd = ["hipcc"] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    return src, proc.returncode, _filter(proc.stderr)


def build(verbose: bool = False) -> str:
    """Always recompile (the caller decides when); returns the library path."""
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory(prefix="mivit_build_") as tmpd:
        objs = [os.path.join(tmpd, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_compile, SOURCES, objs))
        errs = []
        for src, rc, msgs in results:
            if rc != 0:
                errs.append("%s:\n%s" % (src, "\n".join(msgs)))
            elif verbose and msgs:
                print("\n".join(msgs), file=sys.stderr)
        if errs:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["hipcc", "--offload-arch=%s" % ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            raise RuntimeError("link failed:\n" + "\n".join(_filter(proc.stderr)))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
