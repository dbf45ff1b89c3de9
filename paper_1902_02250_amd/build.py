"""Build libbltc.so (the C ABI of include/bltc.h) for gfx950 with hipcc.

Every source is compiled on its own (in parallel) and linked in-tree into
paper_1902_02250_amd/lib/libbltc.so.  The evaluation kernel's template matrix
(kernel x precision x degree x variant) is split by (kernel, precision): its
source is compiled once per pair with -DBLTC_P2P_KERN/-DBLTC_P2P_PREC, and
once without them for the dispatcher.  Files whose FP64 arithmetic must round
exactly as written (tree, grids, MAC, argument handling) are compiled with
-ffp-contract=off; the evaluation kernels allow fused multiply-adds.  Packed
FP32 instructions are disabled for all device code.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libbltc.so")
BUILD = os.path.join(HERE, "_build")

HOST_UNITS = ["host.cpp", "api_tree.cpp", "api_eval.cpp", "api_select.cpp", "api_dual.cpp",
              "api_noalloc.cpp", "tree_host.cpp"]
SOURCES = HOST_UNITS + ["k_prep.hip", "k_lists.hip", "k_upward.hip", "k_p2p.hip",
                        "k_direct.hip", "k_mlp.hip", "k_select.hip", "k_tree.hip", "k_dual.hip",
                        "k_sample.hip", "k_dual_walk.hip", "k_kd.hip"]
EXACT = set(HOST_UNITS) | {"k_prep.hip", "k_lists.hip", "k_tree.hip", "k_select.hip",
                           "k_dual_walk.hip", "k_kd.hip"}

# (kernel, precision) pairs of the evaluation kernel, one object each:
# Stokeslet, rotlet, full (0, 1, 2) x FP64, FP32/FP64-sum, FP32/compensated
# (0, 1, 2), and the FP64 polynomial test kernel (100, 0); heaviest first.
P2P_VARIANTS = [(2, 0), (2, 2), (2, 1), (1, 0), (1, 2), (1, 1), (0, 0), (0, 2), (0, 1),
                (100, 0)]

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(job):
    src, variant = job if isinstance(job, tuple) else (job, None)
    stem = os.path.splitext(src)[0]
    defs = []
    if variant is not None:
        stem += "_k%d_p%d" % variant
        defs = ["-DBLTC_P2P_KERN=%d" % variant[0], "-DBLTC_P2P_PREC=%d" % variant[1]]
    obj = os.path.join(BUILD, stem + ".o")
    contract = "-ffp-contract=off" if src in EXACT else "-ffp-contract=fast"
    lang = ["-x", "hip"]
    cmd = ([_hipcc()] + COMMON + [contract] + defs + lang +
           ["-c", os.path.join(CSRC, src), "-o", obj])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src} {defs}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    work = [("k_p2p.hip", v) for v in P2P_VARIANTS] + SOURCES
    jobs = min(len(work), max(1, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, work))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
