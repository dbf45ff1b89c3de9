"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C sources and the library's host builders (tree_host.cpp: the
cluster tree, the order-tree batches and the balanced k-d batches) are built
with gcc/g++ -fsanitize=address,undefined into one test program
(tests/sanitize/driver.cpp) that runs them on small sets, degenerate ones
included (repeated points, a lattice, a flat set, empty and single-point
sets), checks that the two builders agree bit for bit, and exercises every
kernel of the oracle's direct sum, treecode (both MAC modes, with and without
the separation rule) and cluster-cluster variant.  A sanitizer report aborts
the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_1902_02250_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                    reason="needs gcc and g++")
def test_host_code_under_sanitizers(tmp_path):
    objs = []
    for f in sorted(os.listdir(ORACLE)):
        if f.endswith(".c"):
            o = str(tmp_path / (f + ".o"))
            subprocess.check_call(["gcc", "-std=gnu11", "-ffp-contract=off", "-c",
                                   os.path.join(ORACLE, f), "-o", o] + SAN)
            objs.append(o)
    hip = ["-I", "/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
    for src in (os.path.join(CSRC, "tree_host.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "driver.cpp")):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call(["g++", "-std=c++17", "-ffp-contract=off", "-c", src, "-o", o,
                               "-I", CSRC, "-I", ORACLE, "-I", os.path.join(ROOT, "include")]
                              + hip + SAN)
        objs.append(o)
    exe = str(tmp_path / "driver")
    subprocess.check_call(["g++", "-o", exe] + objs + SAN + ["-lpthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed checks" in r.stdout
