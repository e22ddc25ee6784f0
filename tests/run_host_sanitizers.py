"""Run the CPU test suite against host-sanitizer builds (CPU only).

Two passes, each in its own process, because the two builds use different
sanitizer runtimes and Python itself is not instrumented (the runtime is
preloaded; leak reports are off, since the interpreter keeps its objects):

1. the oracle (``oracle/bem_oracle.c``) built by gcc with AddressSanitizer and
   UndefinedBehaviorSanitizer, under gcc's runtime, for the oracle's pins;
2. the library's host code (mesh validation, tree planning, footprints,
   argument checks of every entry point; ``mesh.cpp``, ``hmatrix.cpp``,
   ``bem_api.cpp``, ``serving.cpp``, ...) built by hipcc with the sanitizers on
   the host side only, under clang's runtime, for the host-side library tests.

Any sanitizer report aborts the pass with a non-zero exit status.

    python tests/run_host_sanitizers.py [extra pytest arguments]
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(env_extra, tests, extra):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *tests, *extra]
    print("+", " ".join(f"{k}={v}" for k, v in env_extra.items()), " ".join(cmd), flush=True)
    return subprocess.run(cmd, cwd=ROOT, env=env).returncode


def main(extra):
    from oracle import build as obuild
    import importlib.util
    spec = importlib.util.spec_from_file_location("_bem_build", os.path.join(ROOT, "paper_1910_01011_amd", "build.py"))
    lbuild = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(lbuild)
    obuild.build(sanitize=True)
    lbuild.build(sanitize=True)
    gcc_rt = ":".join(subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True,
                                     check=True).stdout.strip() for n in ("libasan.so", "libubsan.so"))
    clang_rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))[-1]
    rc = _run({"LD_PRELOAD": gcc_rt, "BEM_ORACLE_LIB": obuild.SANITIZED},
              sorted(glob.glob(os.path.join("tests", "test_oracle_*.py"))), extra)
    rc2 = _run({"LD_PRELOAD": clang_rt, "BEM_LIBRARY": os.path.basename(lbuild.SANITIZED)},
               ["tests/test_library_host.py", "tests/test_serving_host.py", "tests/test_planning_host.py",
                "tests/test_inputs_meshes.py"], extra)
    return rc or rc2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
