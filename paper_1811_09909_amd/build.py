"""Build libhdg.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1811_09909_amd.build   (or build() from Python)
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# HDG_LIB_OUT / HDG_BUILD_DIR / HDG_EXTRA_FLAGS build a variant elsewhere
LIB = os.environ.get("HDG_LIB_OUT", os.path.join(HERE, "_lib", "libhdg.so"))
OUT_DIR = os.path.dirname(LIB)
OBJ_DIR = os.environ.get("HDG_BUILD_DIR", os.path.join(ROOT, "_build"))
SOURCES = ["refelem.cpp", "umesh.cpp", "api.cpp", "element.hip", "build.hip", "trace.hip", "tail.hip", "blas.hip",
           "noalloc.hip", "unstructured.hip"]
ARCH = os.environ.get("HDG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (hipcc only; the host pass ignores it)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
] + os.environ.get("HDG_EXTRA_FLAGS", "").split()


def _compile(src):
    obj = os.path.join(OBJ_DIR, src + ".o")
    cmd = ["hipcc", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS
    if src.endswith(".hip"):
        cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose=True, jobs=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
