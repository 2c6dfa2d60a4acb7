"""Build the opsp HIP library (libopsp.so) in-tree for gfx950.

Usage: ``python -m paper_2206_07244_amd._build`` or ``build()`` from Python.
Every source under ``csrc/`` is compiled by hipcc and linked into
``paper_2206_07244_amd/libopsp.so``; the library exports the C ABI of
``include/opsp.h``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_obj")
LIB = os.path.join(HERE, "libopsp.so")
ARCH = os.environ.get("OPSP_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off: only scalar/float2 code is written
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-result", "-Wno-unused-variable",
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


# Library variants: name -> (extra compile flags, library file).  The default
# is the product; "multi_access" swaps the single compare-and-swap hash probe
# for the read-then-swap probe of the paper's hashing ablation (Section 6.3.2).
VARIANTS = {
    "": ([], LIB),
    "multi_access": (["-DOPSP_HASH_MULTI_ACCESS=1"],
                     os.path.join(HERE, "libopsp_multi_access.so")),
}


def _compile(src: str, variant: str = "") -> str:
    flags, _ = VARIANTS[variant]
    odir = OBJ if not variant else os.path.join(OBJ, variant)
    os.makedirs(odir, exist_ok=True)
    obj = os.path.join(odir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *flags, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    # keep warnings visible but short
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip())
    if err:
        sys.stderr.write(err[:4000] + "\n")
    return obj


MICROBENCH_SRC = os.path.join(HERE, "microbench", "lds_atomics.hip")
MICROBENCH_LIB = os.path.join(HERE, "libopsp_microbench.so")


def build_microbench(verbose: bool = False) -> str:
    """The LDS-atomics microbenchmark (not part of the library)."""
    tmp = MICROBENCH_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *CFLAGS, "-shared", "-o", tmp, MICROBENCH_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {MICROBENCH_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, MICROBENCH_LIB)
    if verbose:
        print("built", MICROBENCH_LIB)
    return MICROBENCH_LIB


def build(verbose: bool = False, variants=("", "multi_access")) -> str:
    """Compile and link every library variant; returns the product library."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    for variant in variants:
        lib = VARIANTS[variant][1]
        with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            objs = list(ex.map(lambda f: _compile(f, variant), srcs))
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, lib)
        if verbose:
            print("built", lib)
    build_microbench(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
