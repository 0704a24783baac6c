"""Run the host-side tests against the AddressSanitizer + UndefinedBehaviorSanitizer build
of the library (CPU only: clustering, local regrid, argument checking and the C-ABI's
error paths are host code).

    python -m paper_2404_02950_amd.sanitize_check [--build] [pytest args...]

The sanitizer runtime is preloaded ahead of anything already preloaded (the interpreter
itself is not instrumented), leak detection is off (the interpreter keeps allocations to
its exit), and any report fails the run."""
import glob
import os
import subprocess
import sys

from . import build_lib

HOST_TESTS = ["tests/test_abi_cpu.py", "tests/test_host_tools.py", "tests/test_local_regrid_host.py",
              "tests/test_regrid_carry_host.py"]


def _asan_runtime() -> str:
    hits = sorted(glob.glob(os.path.join(os.path.dirname(build_lib._clangxx()), "..", "lib", "clang", "*",
                                         "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise SystemExit("AddressSanitizer runtime not found beside ROCm's clang")
    return os.path.realpath(hits[-1])


def main(argv) -> int:
    if "--build" in argv or not os.path.exists(build_lib.SAN_LIB):
        build_lib.build(sanitize=True)
    argv = [a for a in argv if a != "--build"]
    root = os.path.dirname(build_lib.PKG)
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = _asan_runtime() + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["SHAMR_LIB"] = build_lib.SAN_LIB
    cmd = [sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider"] + (argv or HOST_TESTS)
    return subprocess.call(cmd, cwd=root, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
