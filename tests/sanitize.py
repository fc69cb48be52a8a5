"""Sanitizer runs of the CPU test suite (a tool, not collected by pytest).

Two runs of ``pytest tests -m "not gpu"``, each with one instrumented build
loaded in place of the usual one and its sanitizer runtime preloaded into
Python:

1. the oracle built with gcc ``-fsanitize=address,undefined``;
2. the library built with hipcc, AddressSanitizer and UndefinedBehavior-
   Sanitizer on its host code only (each ``-fsanitize`` behind ``-Xarch_host``;
   the device code is built as usual): the neighbourhood builder, the C ABI,
   argument checks, workspace planning.

Leak detection is off (the Python interpreter itself keeps memory until exit);
any other finding aborts the run.  Usage: ``python tests/sanitize.py``.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout.strip()


def clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's AddressSanitizer runtime was not found under /opt/rocm/llvm")
    return hits[-1]


def instrumented(lib):
    out = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    if "__asan_report" not in out:
        sys.exit(f"{lib} carries no AddressSanitizer hooks")
    return lib


def run_suite(env_extra, what):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    print(f"== {what}", flush=True)
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env)
    if r.returncode != 0:
        sys.exit(f"{what}: the CPU suite failed under the sanitizer (exit {r.returncode})")


def main():
    import oracle
    from paper_1809_05018_amd import build_lib

    tmp = tempfile.mkdtemp(prefix="pmrf_san_")
    lib_oracle = oracle.build(("-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                               "-g"), out=os.path.join(tmp, "liboracle_san.so"))
    instrumented(lib_oracle)
    run_suite({"ORACLE_LIB": lib_oracle, "LD_PRELOAD": f"{gcc_runtime('libasan.so')} {gcc_runtime('libubsan.so')}"},
              "oracle built with gcc -fsanitize=address,undefined")

    lib = os.path.join(tmp, "libpmrf_san.so")
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"):
        host_san += ["-Xarch_host", f]
    srcs = [os.path.join(build_lib.CSRC, s) for s in build_lib.SOURCES]
    subprocess.run([build_lib.hipcc(), *build_lib.flags(), *host_san, "-g", "-o", lib, *srcs], check=True)
    instrumented(lib)
    run_suite({"PMRF_LIB": lib, "LD_PRELOAD": clang_asan_runtime()},
              "library host code built with -Xarch_host -fsanitize=address,undefined")
    print("sanitizer runs passed", flush=True)


if __name__ == "__main__":
    main()
