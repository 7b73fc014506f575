"""CPU-only builds with AddressSanitizer and UndefinedBehaviorSanitizer:
the oracle (a driver calls every exported oracle routine on frames of many
shapes, tests/sanitize/oracle_driver.c) and the C ABI's host-side argument
validation; both must finish without a sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off",
           os.path.join(ROOT, "oracle", "viterbi_oracle.c"),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
           "-o", exe, "-lpthread", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "oracle sanitizer driver: ok" in out.stdout


HIPCC = shutil.which("hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


@pytest.mark.skipif(HIPCC is None or not os.path.exists(CLANG), reason="ROCm compilers not available")
def test_capi_validation_under_asan_ubsan(tmp_path):
    """The C ABI's host-side plan and argument code (mivit_api.cpp,
    mivit_pipe.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
    on the host pass only, linked with stand-ins for the kernel launchers
    (tests/sanitize/capi_stubs.cpp): the rejection cases of test_capi.py
    (tests/sanitize/capi_driver.cpp) run without a GPU and without a report."""
    csrc = os.path.join(ROOT, "paper_2011_13579_amd", "csrc")
    srcs = [os.path.join(csrc, "mivit_api.cpp"), os.path.join(csrc, "mivit_pipe.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "capi_stubs.cpp"),
            os.path.join(ROOT, "tests", "sanitize", "capi_driver.cpp")]
    objs = []
    procs = []
    for s in srcs:
        o = str(tmp_path / (os.path.splitext(os.path.basename(s))[0] + ".o"))
        objs.append(o)
        # sanitizers on the host pass only (each -fsanitize after -Xarch_host)
        cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer",
               "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
               "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all", "-c", s,
               "-o", o]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                      text=True))
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-4000:]
    exe = str(tmp_path / "capi_asan")
    link = [CLANG, "-fsanitize=address,undefined"] + objs + [
        "-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]
    subprocess.run(link, check=True, capture_output=True, text=True)
    # the HIP runtime keeps its allocations until exit: leak checking off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "capi sanitizer driver: ok" in out.stdout
