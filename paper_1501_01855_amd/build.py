"""Build the HIP library libovl.so for gfx950 (in-tree, explicit hipcc).

Every HIP source is compiled with packed-FP32 instructions disabled; the
generator file is also compiled without floating-point contraction so that
its fields are bit-identical to the host reference generator.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libovl.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["context.hip", "dslash.hip", "blas.hip", "mscg.hip", "solver.hip", "zolo.cpp", "dense.cpp",
           "gen.hip", "lowmodes.hip", "eigspace.hip", "adjoint.hip", "noalloc.hip", "stream.hip", "lanczos.hip", "capi.hip"]
ARCH = os.environ.get("OVL_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]
PER_FILE = {"gen.hip": ["-ffp-contract=off"]}


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-c", *COMMON, *PER_FILE.get(src, []), "-x", "hip", os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{r.stderr}")
    return obj


def build(jobs=8):
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)
