"""Builds the HIP library libstrassen.so for gfx950, in-tree.

    python paper_1808_07984_amd/build.py      (or __graft_entry__.build())

(Run it as a script: importing the package would first load the library.)

Every source is compiled by hipcc (device code for gfx950 only) in parallel,
then linked into paper_1808_07984_amd/_build/libstrassen.so, which the Python
binding loads.  The library is self-contained: it links only the HIP runtime.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(OUT_DIR, "libstrassen.so")
ARCH = "gfx950"

SOURCES = ["api.cpp", "plan.cpp", "scale.hip", "form.hip", "noalloc.hip", "probe.hip", "gemm_f32_dispatch.cpp", "gemm_m16_dispatch.cpp",
           "gemm_bf16.hip", "gemm_f16.hip", "gemm_bf16x3p_nn.hip"] + [
    "gemm_bf16x3_%s.hip" % lay for lay in ("nn", "nt", "tn", "tt")] + [
    "gemm_f32_%s_%s.hip" % (lay, tile) for lay in ("nn", "nt", "tn", "tt") for tile in ("s", "l")]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + INCLUDE, "-I" + CSRC]
# Packed fp32 instructions are disabled for all device code.
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-ffp-contract=fast", "-munsafe-fp-atomics"]


def source_id():
    """sha256 over the library's sources (csrc/ and include/, file names and
    bytes, sorted): the build id compiled into the library, which the
    binding compares with the sources next to it before loading it."""
    import hashlib
    h = hashlib.sha256()
    for d in (CSRC, INCLUDE):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".cpp", ".hpp", ".h")):
                h.update(name.encode())
                with open(os.path.join(d, name), "rb") as f:
                    h.update(f.read())
    return h.hexdigest()


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src, verbose, build_id):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OUT_DIR, src + ".o")
    cmd = [_hipcc()] + COMMON
    if src == "api.cpp":
        cmd += ['-DSTRASSEN_BUILD_ID="%s"' % build_id]
    if src.endswith(".hip"):
        cmd += DEVICE
    cmd += ["-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr[-8000:]))
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    build_id = source_id()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, build_id), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-8000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
