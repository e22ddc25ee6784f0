"""Compile the C part of the oracle with gcc (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


SANITIZED = "_bem_oracle_san.so"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile the oracle; with ``sanitize`` a second library built with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code only), loaded
    when BEM_ORACLE_LIB names it (run under gcc's libasan, see
    tests/run_host_sanitizers.py)."""
    src = os.path.join(HERE, "bem_oracle.c")
    out = os.path.join(HERE, SANITIZED if sanitize else "_bem_oracle.so")
    tmp = out + ".tmp"
    opt = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] if sanitize else ["-O2"]
    cmd = ["gcc", *opt, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
