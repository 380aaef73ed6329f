"""Build libggf.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Objects are compiled in parallel into paper_2412_01737_amd/_build/ and linked
into paper_2412_01737_amd/libggf.so.  Packed-FP32 instructions are disabled
for the device code (the -packed-fp32-ops target feature).  The SHA-256 of the
sources (csrc/ and include/ggf.h) is compiled into the library and read back by
ggf_source_digest(), so a run can check that the library it loaded was built
from the sources beside it.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libggf.so")
ARCH = os.environ.get("GGF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["ggf_api.cpp", "ggf_factor.hip", "ggf_sweep.hip", "ggf_probe.hip", "ggf_nn.hip"]


def source_digest() -> str:
    """SHA-256 over the library's sources: every file of csrc/ (sorted by name) and include/ggf.h."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if not f.startswith("."))
    for path in files + [os.path.join(ROOT, "include", "ggf.h")]:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile(src: str, digest: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-c", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Wall", "-Wno-unused-variable", "-Wno-unused-function"]
    if src == "ggf_api.cpp":
        cmd += [f"-DGGF_SOURCE_DIGEST=\"{digest}\""]
    if src.endswith(".hip"):
        cmd += ["-x", "hip", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-ffp-contract=fast"]
    cmd += [os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    digest = source_digest()
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, digest), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
