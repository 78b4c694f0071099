"""Build librandqlp.so in-tree with hipcc for gfx950.

Usage: python -m paper_2110_01011_amd.build_lib  (or build() from Python).
Each .hip translation unit is compiled to an object file under _build/ and
linked into paper_2110_01011_amd/librandqlp.so.  The library carries the
SHA-256 of its sources and compile flags (randqlp_build_id()); the binding
refuses to load a library whose id differs from the sources beside it.
"""
import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librandqlp.so")
SOURCES = ["philox.hip", "gemm.hip", "gemm_f64.hip", "gemm16.hip", "panel.hip", "learned.hip",
           "batched.hip", "sparse.hip", "randqlp.hip"]
ARCH = os.environ.get("RANDQLP_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 instructions stay off (they are not used by these kernels)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def source_id():
    """SHA-256 (hex) of every source file and flag the library is built from."""
    h = hashlib.sha256()
    files = [os.path.join(CSRC, f) for f in SOURCES] + [
        os.path.join(CSRC, "rqlp_internal.h"), os.path.join(ROOT, "include", "randqlp.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS[:-2]).encode())  # flags without the include path
    return h.hexdigest()


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the ROCm toolchain is required to build librandqlp")
    return path


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *HIPCC_FLAGS, f"-DRQLP_BUILD_ID=\"{source_id()}\"", "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
