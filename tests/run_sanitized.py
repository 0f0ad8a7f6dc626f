"""Runs the CPU test suite against host-sanitized builds (AddressSanitizer and
UndefinedBehaviorSanitizer), on a machine without a GPU:

  1. the oracle built with gcc -fsanitize=address,undefined, loaded through
     ORACLE_LIB with gcc's runtimes preloaded: every `-m "not gpu"` test;
  2. libkadabra built with the sanitizers on its host pass (input validation,
     parameter handling, the C ABI), loaded through KADABRA_LIB with clang's
     ASan runtime preloaded: the C ABI tests.

Undefined behaviour aborts the run (no recovery); leak checking is off (the
Python interpreter's own allocations would be reported).  Run from the
repository root:  python tests/run_sanitized.py
"""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def run(env_extra, args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", **env_extra)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *args]
    print("+", " ".join(f"{k}={v}" for k, v in env_extra.items()), " ".join(cmd), flush=True)
    return subprocess.call(cmd, cwd=ROOT, env=env)


def main() -> int:
    import oracle
    from paper_1903_09422_amd import build as kbuild

    gcc_rt = [subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
              for n in ("libasan.so", "libubsan.so")]
    clang_rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not clang_rt:
        print("clang ASan runtime not found", file=sys.stderr)
        return 2
    rc = run({"ORACLE_LIB": oracle.build(sanitize=True), "LD_PRELOAD": ":".join(gcc_rt)},
             ["tests", "-m", "not gpu", "-x"])
    if rc:
        return rc
    return run({"KADABRA_LIB": kbuild.build(sanitize=True), "LD_PRELOAD": clang_rt[-1]},
               ["tests/test_capi_cpu.py", "-x"])


if __name__ == "__main__":
    sys.exit(main())
