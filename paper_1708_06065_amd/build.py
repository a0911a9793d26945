"""Build liblair.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1708_06065_amd.build        # or build() from Python

The library lands in paper_1708_06065_amd/_lib/liblair.so; object files go
to paper_1708_06065_amd/_build/.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "liblair.so")
ARCH = os.environ.get("LAIR_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["k_setup.hip", "k_cycle.hip", "k_batch.hip", "k_krylov.hip", "k_nodal.hip", "k_split.hip", "lair_api.cpp",
               "setup.cpp", "solve.cpp", "noalloc.cpp",
               "profile.cpp", "alloc.cpp"]
CXX_SOURCES = ["rs_split.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(HERE, "..", "include")]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          # no packed FP32 instructions (v_pk_*_f32)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


# Per-file device flags.  The register-tiled node solves unroll their step
# loops over 9 column slots; past the default size limit the unrolling stops
# and the register tiles fall back to scratch memory.
FILE_FLAGS = {"k_setup.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}


def _compile(src, hip):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + (DEVICE + FILE_FLAGS.get(src, []) if hip else []) + \
        ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" %
                           (" ".join(cmd), r.stdout, r.stderr))
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = [(s, True) for s in HIP_SOURCES] + [(s, False) for s in CXX_SOURCES]
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        outs = list(ex.map(lambda j: _compile(*j), jobs))
    objs = [o for o, _ in outs]
    if verbose:
        for _, err in outs:
            if err.strip():
                print(err)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + \
        ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
