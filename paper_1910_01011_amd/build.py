"""Build the HIP library ``libbem_mi355x.so`` for gfx950 with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbem_mi355x.so")
SOURCES = ["bem_api.cpp", "mesh.cpp", "krylov.cpp", "autotune.cpp", "k_farfield.hip", "k_singular.hip", "k_linalg.hip", "k_field.hip", "k_dense.hip", "k_gemm.hip", "k_osrc.hip", "k_single_layer.hip", "hmatrix.cpp", "k_hmatrix.hip", "noalloc.hip", "serving.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
            # no packed FP32 instructions anywhere in the device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]


SANITIZED = os.path.join(HERE, "libbem_mi355x_san.so")
# host code only: each sanitizer flag applies to the host compilation
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def build(verbose: bool = False, jobs: int = 6, sanitize: bool = False) -> str:
    """Compile the library; with ``sanitize`` a second library whose host code
    is built with AddressSanitizer and UndefinedBehaviorSanitizer (the device
    code is unchanged), loaded when BEM_LIBRARY names it."""
    objdir = os.path.join(HERE, "_build_san" if sanitize else "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [HIPCC, *flags(), *(HOST_SANITIZE if sanitize else []), "-x", "hip", "-c", os.path.join(CSRC, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for pr in procs:
        _wait(pr)
    out = SANITIZED if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *(["-Xarch_host", "-fsanitize=address",
                                                                  "-Xarch_host", "-fsanitize=undefined"]
                                                                 if sanitize else []), "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _wait(item):
    src, proc = item
    out, _ = proc.communicate()
    text = out.decode(errors="replace")
    # the host pass does not know the packed-fp32 target feature: harmless
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if proc.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"hipcc failed for {src}")
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
