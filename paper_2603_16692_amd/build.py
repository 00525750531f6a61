"""Build libks.so (the HIP KeySwitch library) in-tree with hipcc for gfx950."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libks.so")
# The debug build: the same kernels, with every call first checking that its
# inputs are canonical residues (ks_api.cpp compiled with KS_DEBUG_CHECKS).
DEBUG_LIB = os.path.join(HERE, "libks_debug.so")
SOURCES = ["ks_host.cpp", "ks_api.cpp", "ks_kernels.hip"]
DEBUG_SOURCES = ["ks_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # floating-point steps are written out explicitly where they matter
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, debug: bool = False) -> str:
    obj = os.path.join(OBJ, src + (".debug.o" if debug else ".o"))
    cmd = [HIPCC] + FLAGS + (["-DKS_DEBUG_CHECKS=1"] if debug else []) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip():
        sys.stderr.write(err + "\n")
    return obj


def _link(lib: str, objs) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + list(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)


def build() -> str:
    """libks.so and its debug twin libks_debug.so (same kernels)."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + [(src, True) for src in DEBUG_SOURCES]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        objs = dict(zip(jobs, ex.map(lambda j: _compile(*j), jobs)))
    _link(LIB, [objs[(src, False)] for src in SOURCES])
    _link(DEBUG_LIB, [objs[(src, src in DEBUG_SOURCES)] for src in SOURCES])
    return LIB


if __name__ == "__main__":
    print(build())
