"""Runs the CPU test-suite (-m "not gpu") against the sanitized builds: the
oracle and the host code of libhesp compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (clang), one sanitizer runtime preloaded into Python.

    python tests/sanitized_cpu_suite.py [extra pytest arguments]

Builds oracle/liboracle_san.so and paper_1602_05510_amd/libhesp_san.so, then
runs pytest in a child process with HESP_SANITIZE=1; exits with its status.
Leak detection is off (the interpreter itself is not instrumented); any other
report aborts the run.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main() -> int:
    from oracle import oracle as O
    from paper_1602_05510_amd import build as B
    O.build(sanitize=True)
    B.build(sanitize=True)
    rt = subprocess.check_output([O.CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    env = dict(os.environ, HESP_SANITIZE="1", LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           *sys.argv[1:]]
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    sys.exit(main())
