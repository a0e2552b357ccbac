"""Build libiaat.so for gfx950: run the install-time kernel-family generator,
then compile the HIP sources with hipcc into the package directory.

    python -m paper_2208_09822_amd.build [-v]
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
GEN_DIR = os.path.join(CSRC, "generated")
OBJ_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libiaat.so")
ROOT = os.path.dirname(PKG)

SOURCES = ["kernels.hip", "batched.hip", "precision.hip", "traditional.hip", "xgemm.hip", "api.cpp", "serve.cpp", "tiler.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "--offload-arch=gfx950", "-mcode-object-version=5",
          # packed FP32 instructions off (results of some packed forms are unreliable)
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def generate() -> None:
    os.makedirs(GEN_DIR, exist_ok=True)
    from paper_2208_09822_amd.gen import gen_family
    gen_family.main(["gen_family", os.path.join(GEN_DIR, "family.inc")])


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s%s" % (src, r.stdout, r.stderr))
    # hipcc's host pass does not know the device feature flag; drop that noise
    noise = [l for l in r.stderr.splitlines() if "not a recognized feature" not in l and l.strip()]
    if noise and verbose:
        print("\n".join(noise))
    return obj


def build(verbose: bool = False) -> str:
    sys.path.insert(0, ROOT)
    generate()
    os.makedirs(OBJ_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
