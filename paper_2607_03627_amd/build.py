"""Build libuclp.so (HIP kernels + C ABI host runtime) for gfx950 in-tree.

    python -m paper_2607_03627_amd.build

hipcc cross-compiles without a GPU.  The library lands next to this file,
where the Python binding loads it.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libuclp.so")
SOURCES = ["kernels.hip", "uclp.cpp"]
ARCH = os.environ.get("UCLP_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the
# library (device code unchanged), for the CPU tests of validation, presolve
# and tile building.  Each sanitizer flag is scoped to the host pass.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-shared-libsan"]
ASAN_LIB = os.path.join(ROOT, "_build", "libuclp_asan.so")


def sanitizer_runtime() -> str:
    """The clang AddressSanitizer runtime the sanitized library links against
    (to preload into an uninstrumented Python)."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], check=True,
                         capture_output=True, text=True).stdout.strip()
    return out


def build(verbose: bool = False, sanitize: bool = False) -> str:
    objs = []
    common = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
              # packed FP32 instructions are disabled for every HIP translation unit
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include")]
    if sanitize:
        common = [c if c != "-O3" else "-O1" for c in common] + HOST_SANITIZE
        os.makedirs(os.path.dirname(ASAN_LIB), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(CSRC, src + (".asan.o" if sanitize else ".o"))
        cmd = [hipcc(), *common, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    out = ASAN_LIB if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if sanitize:
        cmd[1:1] = HOST_SANITIZE
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    for o in objs:
        os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
